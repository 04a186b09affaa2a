"""Host replica of the index arithmetic of the particle kernel's LDS window of
buffer-cell LB velocities (the exchange step of Alg. 1 reads the LB velocity
of a buffer particle's fine cell, Sec. 2.3).

The workgroup of a tile of Tx x Ty x Tz cells of the shifted grid copies the
fine cells [tile origin - 1, tile end) of every axis (buffer rows only) into
LDS; a buffer particle then reads entry (I - I0, J - J0, K - K0) of that
window, or global memory when the entry lies outside it.  With the grid shift
uniform in [0, a) a particle binned into shifted cell i sits in unshifted fine
cell i - 1 or i, so only particles across the periodic wrap of a tile (or a
window larger than the table) should need global memory.  The replica below
restates the kernel's formulas (binning in the particle precision, fine cell
in binary64, the window's fill and lookup) and checks on random geometries
that every lookup that hits reads the entry the fill stored for the
particle's own fine cell, that every index stays in range, and that the
misses are of the expected kind only."""
import os
import re

import numpy as np
import pytest

_HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2004_00304_amd", "csrc", "common.hpp")
MAX_UFC = int(re.search(r"constexpr int MAX_UFC = (\d+);", open(_HDR).read()).group(1))


def _floor_int(v):
    return np.floor(v).astype(np.int64)


def _geometry(rng, dim):
    r = int(rng.choice([1, 2, 3, 4]))
    nx = int(rng.integers(2, 24))
    nz = int(rng.integers(2, 12)) if dim == 3 else 1
    nsy = int(rng.integers(3, 10))            # slab height in LB rows
    buf_lo = int(rng.integers(0, 2))
    buf_hi = int(rng.integers(1, 2))
    if buf_lo + buf_hi >= nsy:
        buf_lo = 0
    R = nsy * r                                 # fine rows of the slab
    Cx, Cz = nx * r, (nz * r if dim == 3 else 1)
    opts = [(1, 1, 1), (2, 1, 1), (2, 2, 1), (4, 2, 1), (4, 4, 1), (8, 4, 1), (8, 8, 1), (16, 8, 1)] if dim == 2 else \
        [(1, 1, 1), (2, 2, 1), (2, 2, 2), (4, 2, 2), (4, 4, 2), (4, 4, 4), (4, 4, 8), (8, 4, 4), (16, 8, 1),
         (8, 2, 8), (4, 2, 8), (8, 2, 4), (8, 1, 8)]
    T = opts[int(rng.integers(len(opts)))]
    return dict(dim=dim, r=r, R=R, Cx=Cx, Cz=Cz, CyB=R + 1, NB=(buf_lo + buf_hi) * r,
                rbl=buf_lo * r, rbh=R - buf_hi * r, T=T, nx=nx, nz=nz, nsy=nsy)


def _check(g, rng, dtype, n=4000):
    dim, r = g["dim"], g["r"]
    Tx, Ty, Tz = g["T"]
    # particle positions in the slab (y relative to its lower face) and the
    # grid shift, both in the particle precision
    x = rng.uniform(0, g["nx"], n).astype(dtype)
    y = rng.uniform(0, g["nsy"], n).astype(dtype)
    z = (rng.uniform(0, g["nz"], n) if dim == 3 else np.zeros(n)).astype(dtype)
    a = 1.0 / r
    sh = (rng.uniform(0, a, 3)).astype(dtype)
    rr = dtype(r)
    # shifted cell, as bin_coord / bin_row (particle precision, then floor)
    ix = _floor_int((x + sh[0]) * rr)
    ix = np.where(ix >= g["Cx"], ix - g["Cx"], ix)
    iy = np.minimum(_floor_int((y + sh[1]) * rr), g["CyB"] - 1)
    iz = _floor_int((z + sh[2]) * rr) if dim == 3 else np.zeros(n, np.int64)
    iz = np.where(iz >= g["Cz"], iz - g["Cz"], iz)
    tx, ty, tz = ix // Tx, iy // Ty, iz // Tz
    # fine cell of the exchange (binary64, clamped)
    I = np.clip(_floor_int(x.astype(np.float64) * r), 0, g["Cx"] - 1)
    J0 = np.clip(_floor_int(y.astype(np.float64) * r), 0, g["R"] - 1)
    K = np.clip(_floor_int(z.astype(np.float64) * r), 0, g["Cz"] - 1) if dim == 3 else np.zeros(n, np.int64)
    buf = (J0 < g["rbl"]) | (J0 >= g["rbh"])
    # lookup, as in the exchange
    uwx, uwy, uwz = Tx + 1, Ty + 1, (Tz + 1 if dim == 3 else 1)
    uI0, uJ0, uK0 = tx * Tx - 1, ty * Ty - 1, (tz * Tz - 1 if dim == 3 else np.zeros(n, np.int64))
    uc_ok = ((uJ0 < g["rbl"]) | (uJ0 + uwy - 1 >= g["rbh"])) & (uwx * uwy * uwz <= MAX_UFC)
    ax = I - uI0
    ax = np.where(ax < 0, ax + g["Cx"], ax)
    ay = J0 - uJ0
    az = (K - uK0) if dim == 3 else np.zeros(n, np.int64)
    az = np.where(az < 0, az + g["Cz"], az)
    hit = buf & uc_ok & (ax < uwx) & (ay >= 0) & (ay < uwy) & (az < uwz)
    ci = ax + uwx * (ay + uwy * az)
    assert np.all(ci[hit] < MAX_UFC) and np.all(ci[hit] >= 0)
    # the fill stores, at entry (ax, ay, az), fine cell ((I0 + ax) mod Cx,
    # J0 + ay, (K0 + az) mod Cz), and only for buffer rows
    fI = ((uI0 + ax) % g["Cx"] + g["Cx"]) % g["Cx"]
    fJ = uJ0 + ay
    fK = ((uK0 + az) % g["Cz"] + g["Cz"]) % g["Cz"] if dim == 3 else np.zeros(n, np.int64)
    filled = (fJ >= 0) & (fJ < g["R"]) & ((fJ < g["rbl"]) | (fJ >= g["rbh"]))
    assert np.all(filled[hit])
    assert np.array_equal(fI[hit], I[hit]) and np.array_equal(fJ[hit], J0[hit]) and np.array_equal(fK[hit], K[hit])
    # the fill's global index stays inside the buffer-cell array
    Jb = np.where(fJ < g["rbl"], fJ, fJ - (g["R"] - g["NB"]))
    fc = (fK * g["NB"] + Jb) * g["Cx"] + fI
    assert np.all((fc[hit] >= 0) & (fc[hit] < g["Cx"] * g["NB"] * g["Cz"]))
    # misses: only a window too large for the table, or a particle whose
    # shifted cell wrapped across the periodic x or z face (its fine cell then
    # lies at the far end of the channel).  Rounding is monotone in either
    # precision, so the shifted cell is the fine cell or the one above it.
    miss = buf & ~hit
    wrapped = (ix < I) | ((iz < K) if dim == 3 else np.zeros(n, bool))
    ok_miss = ~uc_ok | wrapped
    assert np.all(ok_miss[miss]), (g, int(miss.sum()), int((miss & ~ok_miss).sum()))
    return int(buf.sum()), int(hit.sum()), int(miss.sum())


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_window_lookup_reads_the_particles_own_cell(dim, dtype):
    rng = np.random.default_rng(11 + dim + (dtype is np.float32))
    tot = np.zeros(3, np.int64)
    for _ in range(300):
        g = _geometry(rng, dim)
        tot += _check(g, rng, dtype)
    nbuf, nhit, nmiss = tot
    assert nbuf > 100000
    # the fallback is the exception: wraps and oversized windows only
    assert nhit >= 0.8 * nbuf, (nbuf, nhit, nmiss)


def test_film_tiles_fit_the_table():
    """The thin film's 8 x 2 x 8 tiles need (9)(3)(9) = 243 entries and the 3D
    channel's 4 x 2 x 8 tiles 135 (the library only picks shapes whose window
    fits); every default 2D shape fits as well, and a 16 x 8 x 1 tile (306
    entries) does not, which the parity case for an oversized window uses."""
    assert 9 * 3 * 9 <= MAX_UFC and 5 * 3 * 9 <= MAX_UFC
    for T in [(1, 1), (2, 1), (2, 2), (4, 2), (4, 4), (8, 4), (8, 8), (16, 8)]:
        assert (T[0] + 1) * (T[1] + 1) <= MAX_UFC
    assert 17 * 9 * 2 > MAX_UFC
