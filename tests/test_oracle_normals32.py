"""Pins of the oracle's binary32 normal deviates (drawn for particles stored
in binary32, by the exchange step of Sec. 2.3 and by MPCD-AT, Eq. 6).

The generator is Box-Muller on four 24-bit uniforms of one Philox block, with
ln and sin/cos of 2 pi u evaluated as binary32 series.  What pins it:
  * ln against an extended-precision logarithm on the generator's grid
    (multiples of 2^-24) and at every binade edge: within 2 units in the last
    place (the series' own error is 1.6; dropping its last term gives 2.5, a
    binary32 ln 2 one unit off gives 3.6);
  * sin and cos of 2 pi u against extended precision, within 1.5 units of
    2^-24 (measured 1.15; a dropped series term gives 5.5 or 60, pi/2 one
    unit off 1.8), exact at the quadrant points, and at u = 1/8 both equal
    to sqrt(1/2) rounded to binary32 (pi/2 one unit off breaks that too);
  * the normals equal the FP64 Box-Muller transform of the same uniforms
    (radius sqrt(-2 ln(1 - a_even)), z0 = rho cos, z1 = rho sin, z2 the
    cosine of the second pair) to binary32 accuracy;
  * their sample moments and the Kolmogorov-Smirnov distance to the standard
    normal over 600,000 deviates."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O

G = 2.0 ** -24


def _grid():
    edges = [0.0, G, 2 * G, 1 - G, 1 - 2 * G, 0.5 - G, 0.5, 0.5 + G]
    for q in range(1, 8):  # octant boundaries and their neighbours
        edges += [q / 8 - G, q / 8, q / 8 + G]
    for k in range(1, 25):  # 1 - a across every binade of (0, 1]
        edges += [2.0 ** -k, 1 - 2.0 ** -k]
    rng = np.random.default_rng(3)
    rand = rng.integers(0, 2 ** 24, size=30000).astype(np.float64) * G
    return np.concatenate([np.array(edges), rand]).astype(np.float32)


def test_ln32_within_two_ulp():
    a = _grid()
    x = (1.0 - a.astype(np.float64)).astype(np.float32)  # exact: a is a multiple of 2^-24
    got = O.ln32(x)
    assert got[0] == 0.0  # ln 1
    L = np.longdouble
    ref = np.log(x.astype(L))
    ulp = np.spacing(np.abs(ref.astype(np.float32))).astype(L)
    ulp[ref == 0] = L(np.finfo(np.float32).tiny)
    e = np.abs(got.astype(L) - ref) / ulp
    assert float(e.max()) <= 2.0, (float(e.max()), float(x[e.argmax()]))
    # the smallest argument of the generator, 2^-24: ln = -24 ln 2
    assert abs(float(O.ln32(G)[0]) - (-24 * math.log(2.0))) <= 2 * np.spacing(np.float32(16.6))


def test_sincos32_within_one_and_a_half_units():
    a = _grid()
    s, c = O.sincos32(a)
    L = np.longdouble
    ang = 2 * np.arccos(L(-1)) * a.astype(L)
    es = float(np.abs(s.astype(L) - np.sin(ang)).max() / L(G))
    ec = float(np.abs(c.astype(L) - np.cos(ang)).max() / L(G))
    assert es <= 1.5 and ec <= 1.5, (es, ec)
    # quadrant points are exact
    for u, (sq, cq) in ((0.0, (0.0, 1.0)), (0.25, (1.0, 0.0)), (0.5, (0.0, -1.0)), (0.75, (-1.0, 0.0))):
        sv, cv = O.sincos32([u])
        assert sv[0] == sq and cv[0] == cq, (u, sv, cv)
    # u = 1/8: the angle pi/4, both sqrt(1/2) rounded to binary32
    sv, cv = O.sincos32([0.125])
    r = np.float32(math.sqrt(0.5))
    assert sv[0] == r and cv[0] == r, (sv, cv)


def test_normals32_are_box_muller_of_the_block():
    w = O.philox_stream([7, 9], 0, 20000)
    for dim in (2, 3):
        z = O.normals32(w, dim).astype(np.float64)
        a = (w >> 8).astype(np.float64) * G
        r0 = np.sqrt(-2.0 * np.log(1.0 - a[:, 0]))
        r1 = np.sqrt(-2.0 * np.log(1.0 - a[:, 2]))
        want = np.stack([r0 * np.cos(2 * np.pi * a[:, 1]), r0 * np.sin(2 * np.pi * a[:, 1]),
                         r1 * np.cos(2 * np.pi * a[:, 3]) if dim == 3 else np.zeros(len(a))], axis=1)
        # binary32 radius and angle: a few units of 2^-24 relative to the radius
        err = np.abs(z - want) / np.maximum(np.concatenate([r0[:, None], r0[:, None], r1[:, None]], 1), 1.0)
        assert err.max() <= 4e-7, (dim, err.max())
        if dim == 2:
            assert np.all(z[:, 2] == 0.0)


def test_normals32_distribution():
    w = O.philox_stream([3, 5], 1 << 20, 200000)
    z = O.normals32(w, 3).astype(np.float64).ravel()
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert abs(np.mean(z ** 4) - 3.0) < 5 * math.sqrt(96.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the largest radius of 24-bit uniforms: sqrt(-2 ln 2^-24) = 5.77
    assert np.abs(z).max() <= math.sqrt(-2.0 * math.log(G)) + 1e-5


def test_binary32_particles_draw_binary32_normals():
    """The exchange of a binary32 slab redraws a buffer particle as
    u + sqrt(kT/m) z, z the binary32 normals of block 0 of its stream
    (element = id, LB step, substep << 8 | 3); a binary64 slab keeps the
    binary64 transform of two blocks."""
    from paper_2004_00304_amd import workloads as W
    ids = np.arange(64, dtype=np.uint32) * 7919
    pos = np.tile(np.array([[1.1], [5.0], [1.7]]), (1, len(ids)))  # lower buffer rows are y in [4, 6)
    vel = np.zeros((3, len(ids)))
    u = np.tile(np.array([[0.01], [0.0], [-0.02]]), (1, len(ids)))
    for fp in (32, 64):
        q = W.make(dim=3, n=(8, 16, 4), ylo=4, yhi=12, buf_lo=2, buf_hi=2, kT=0.7, mass=2.0, part_fp=fp,
                   g=(0.0, 0.0, 0.0), substeps=1, seed=(5 << 32) | 11, instance=3)
        pr = O.Probe(q)
        assert pr.in_buffer(pos[:, 0])
        _, v = pr.exchange_stream(9, 1, ids, pos, vel, u)
        key = [11, 5 ^ 3]
        sd = math.sqrt(0.7 / 2.0)
        for k, i in enumerate(ids):
            w0 = O.philox([int(i), 9, (1 << 8) | 3, 0], key)
            if fp == 32:
                z = O.normals32(w0[None, :], 3)[0].astype(np.float64)
                want = (u[:, k] + sd * z).astype(np.float32).astype(np.float64)
                # streaming keeps the velocity (no force), up to the sign of
                # v_y if the particle met a reflecting face
                assert v[0, k] == want[0] and v[2, k] == want[2] and abs(v[1, k]) == abs(want[1]), (k, v[:, k], want)
            else:
                w1 = O.philox([int(i), 9, (1 << 8) | 3, 1], key)
                z0, z1 = O.box_muller(O.u01(int(w0[0]), int(w0[1])), O.u01(int(w0[2]), int(w0[3])))
                z2, _ = O.box_muller(O.u01(int(w1[0]), int(w1[1])), O.u01(int(w1[2]), int(w1[3])))
                want = u[:, k] + sd * np.array([z0, z1, z2])
                assert v[0, k] == want[0] and v[2, k] == want[2] and abs(v[1, k]) == abs(want[1]), (k, v[:, k], want)


def test_mpcd_at_of_binary32_particles_uses_binary32_normals():
    """MPCD-AT (Eq. 6) of an interior cell of a binary32 slab: the random
    velocities are sqrt(kT/m) z rounded to binary32, z the binary32 normals
    of block 0 of each particle's AT stream (element = id, substep << 8 | 9)."""
    from paper_2004_00304_amd import workloads as W
    q = W.make(dim=3, n=(8, 16, 4), ylo=4, yhi=12, buf_lo=2, buf_hi=2, kT=0.4, mass=1.5, part_fp=32,
               collision=1, g=(0.0, 0.0, 0.0), substeps=2, seed=77, instance=0)
    pr = O.Probe(q)
    rng = np.random.default_rng(2)
    n = 9
    ids = (np.arange(n) * 104729 + 5).astype(np.int32)
    vel = rng.normal(0.0, 0.5, (3, n)).astype(np.float32).astype(np.float64)
    sh = np.zeros(3)
    c = 10  # any interior cell: no wall cuts it
    v, vcm = pr.collide_cell(c, 6, 1, sh, vel, ids)
    sd = math.sqrt(0.4 / 1.5)
    w = np.array([O.philox([int(i), 6, (1 << 8) | 9, 0], [77, 0]) for i in ids])
    z = O.normals32(w, 3).astype(np.float64)
    vran = (sd * z.T).astype(np.float32).astype(np.float64)
    want, wcm = O.at_collide(3, vel, vran)
    assert np.array_equal(v, want.astype(np.float32).astype(np.float64))
    assert np.allclose(vcm, vel.mean(axis=1), rtol=0, atol=1e-15)
