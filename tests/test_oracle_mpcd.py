"""Pins of the oracle's particle part: SRD collision (Eq. 4, local
conservation of mass, momentum and energy), binning into shifted collision
cells (brute force on tiny inputs), ballistic streaming (Eq. 3), wall
bounce-back, the Maxwell-Boltzmann exchange step (Alg. 1), interpolation to
the fine grid (Alg. 2), one-way coupling, and the feedback reading."""
import numpy as np
import pytest
from scipy import stats

from paper_2004_00304_amd import workloads as W


# ---------------------------------------------------------------- SRD rule

@pytest.mark.parametrize("dim", [2, 3])
def test_srd_conserves_momentum_energy(oracle_lib, dim):
    rng = np.random.default_rng(11)
    for n in (1, 2, 3, 7, 20, 64):
        v = rng.standard_normal((dim, n)) + rng.uniform(-1, 1, (dim, 1))
        ax = rng.standard_normal(3)
        ax /= np.linalg.norm(ax)
        for alpha in (130.0, 90.0, 17.3):
            for sgn in (1.0, -1.0):
                v2, vcm = oracle_lib.srd_rotate(dim, v, alpha, sgn, ax)
                P, P2 = v.sum(1), v2.sum(1)
                E, E2 = (v * v).sum(), (v2 * v2).sum()
                scaleP = np.abs(v).sum()
                assert np.abs(P2 - P).max() <= 1e-12 * scaleP
                assert abs(E2 - E) <= 1e-12 * E
                assert np.abs(vcm - v.mean(1)).max() <= 1e-14 * (1 + np.abs(v).max())
                if n == 1:
                    assert np.abs(v2 - v).max() < 1e-15


def test_srd_2d_rotation_angle(oracle_lib):
    """Relative velocities turn by exactly +alpha or -alpha (Eq. 4)."""
    rng = np.random.default_rng(12)
    v = rng.standard_normal((2, 9))
    for sgn in (1.0, -1.0):
        v2, vcm = oracle_lib.srd_rotate(2, v, 130.0, sgn)
        w, w2 = v - vcm[:, None], v2 - vcm[:, None]
        ang = np.arctan2(w[0] * w2[1] - w[1] * w2[0], (w * w2).sum(0))
        assert np.allclose(ang, sgn * np.radians(130.0), atol=1e-13)
        assert np.allclose(np.linalg.norm(w, axis=0), np.linalg.norm(w2, axis=0), rtol=1e-14)


def test_srd_3d_axis_invariant(oracle_lib):
    rng = np.random.default_rng(13)
    v = rng.standard_normal((3, 11))
    ax = rng.standard_normal(3)
    ax /= np.linalg.norm(ax)
    v2, vcm = oracle_lib.srd_rotate(3, v, 120.0, 1.0, ax)
    w, w2 = v - vcm[:, None], v2 - vcm[:, None]
    assert np.allclose(ax @ w, ax @ w2, atol=1e-14)
    wp = w - np.outer(ax, ax @ w)
    wp2 = w2 - np.outer(ax, ax @ w2)
    cosang = (wp * wp2).sum(0) / (np.linalg.norm(wp, axis=0) * np.linalg.norm(wp2, axis=0))
    assert np.allclose(cosang, np.cos(np.radians(120.0)), atol=1e-13)
    # orientation: (wp x wp2) is along +axis
    cr = np.cross(wp.T, wp2.T) @ ax
    assert (cr > 0).all()


def test_srd_virtual_particles_centre_of_mass(oracle_lib):
    """Wall cells: the centre of mass includes the virtual momentum and mass."""
    v = np.array([[0.5, -0.1, 0.3], [0.2, 0.4, -0.6]])
    pv = np.array([0.7, -0.2, 0.0])
    v2, vcm = oracle_lib.srd_rotate(2, v, 130.0, 1.0, p_virt=pv, m_virt=5.0)
    assert np.allclose(vcm, (v.sum(1) + pv[:2]) / 8.0, rtol=1e-15)
    # the rotation is about the augmented centre of mass: |v - vcm| is kept
    assert np.allclose(np.linalg.norm(v - vcm[:, None], axis=0), np.linalg.norm(v2 - vcm[:, None], axis=0))


# ---------------------------------------------------------------- sorting and binning

def test_counting_sort_bruteforce(oracle_lib):
    rng = np.random.default_rng(21)
    for n, nc in ((0, 3), (1, 1), (17, 4), (64, 16), (500, 37)):
        cell = rng.integers(0, nc, n).astype(np.int32)
        count, start, order = oracle_lib.counting_sort(cell, nc)
        assert (count == np.bincount(cell, minlength=nc)).all()
        assert (start == np.concatenate([[0], np.cumsum(count)[:-1]])).all()
        assert (order == np.argsort(cell, kind="stable")).all()


@pytest.mark.parametrize("dim", [2, 3])
def test_binning_bruteforce_tiny(oracle_lib, dim):
    """Every particle lies inside the bounds of its shifted cell and of no
    other cell (checked against every cell, with periodic wrap)."""
    if dim == 2:
        p = W.periodic_2d(n=(2, 2, 1), refine=2, ppc=4, alpha_deg=90.0)
    else:
        p = W.make(dim=3, n=(2, 2, 2), walls_y=0, ylo=0, yhi=2, buf_lo=0, buf_hi=0, refine=1,
                   ppc=6, g=(0, 0, 0), feedback=0, alpha_deg=90.0)
    o = oracle_lib.Oracle(p)
    r = p["refine"]
    a = 1.0 / r
    L = np.array(p["n"][:dim], float)
    C = (L * r).astype(int)
    for _ in range(4):
        o.step(1)
        pos, _ = o.particles()
        sh = o.shift()
        assert ((sh >= 0) & (sh < a)).all()
        b = o.binning()
        ncell = int(np.prod(C))
        assert len(b["count"]) == ncell
        for k in range(o.Np):
            hits = []
            for c in range(ncell):
                idx = np.unravel_index(c, C[::-1])[::-1]
                inside = True
                for d in range(dim):
                    lo = idx[d] * a - sh[d]
                    x = pos[d, k]
                    # periodic images
                    ok = any(lo <= x + m * L[d] < lo + a for m in (-1, 0, 1))
                    inside &= ok
                if inside:
                    hits.append(c)
            assert hits == [b["cell"][k]]
        assert (b["count"] == np.bincount(b["cell"], minlength=ncell)).all()
        assert (b["order"] == np.argsort(b["cell"], kind="stable")).all()


def test_shift_statistics(oracle_lib):
    o = oracle_lib.Oracle(W.periodic_2d(n=(2, 2, 1), ppc=1))
    sh = []
    for _ in range(200):
        o.step(1)
        sh.append(o.shift())
    sh = np.array(sh) * 2  # a = 1/2
    for d in range(2):
        assert stats.kstest(sh[:, d], "uniform").pvalue > 1e-3


# ---------------------------------------------------------------- streaming and walls

def test_ballistic_streaming_periodic(oracle_lib):
    """With alpha = 0 the collision is the identity and particles fly
    ballistically under the constant acceleration: r(T) = r0 + v0 T + g T^2/2
    (mod L), v(T) = v0 + g T (Eq. 3)."""
    g = (3e-3, -2e-3, 0.0)
    p = W.periodic_2d(n=(4, 4, 1), ppc=3, alpha_deg=0.0, g=g, substeps=4)
    o = oracle_lib.Oracle(p)
    pos0, vel0 = o.particles()
    o.step(3)
    pos, vel = o.particles()
    T = 3.0
    gg = np.array(g[:2])[:, None]
    exp_v = vel0 + gg * T
    exp_r = np.mod(pos0 + vel0 * T + 0.5 * gg * T * T, 4.0)
    assert np.abs(vel - exp_v).max() < 1e-13
    dr = np.abs(pos - exp_r)
    dr = np.minimum(dr, 4.0 - dr)
    assert dr.max() < 1e-12


def test_wall_bounce_back(oracle_lib):
    """Bounce-back at the walls reverses the velocity at the crossing instant
    (no-slip) and keeps every particle in the channel."""
    p = W.walled_2d(n=(4, 4, 1), refine=1, ppc=2, alpha_deg=0.0, g=(0, 0, 0), substeps=1,
                    grid_shift=0)
    o = oracle_lib.Oracle(p)
    pos0, vel0 = o.particles()
    n = o.Np
    # particle 0 heads into the bottom wall, particle 1 into the top wall
    pos0[:, 0] = (1.3, 0.2)
    vel0[:, 0] = (0.5, -0.8)
    pos0[:, 1] = (2.5, 3.9)
    vel0[:, 1] = (-0.25, 0.3)
    o.set_particles(pos0, vel0)
    o.step(1)
    pos, vel = o.particles()
    # bottom: crossing after 0.25, then 0.75 back up with v = (-0.5, +0.8)
    assert np.allclose(pos[:, 0], (1.3 + 0.5 * 0.25 - 0.5 * 0.75, 0.8 * 0.75), atol=1e-14)
    assert np.allclose(vel[:, 0], (-0.5, 0.8), atol=1e-15)
    tc = 0.1 / 0.3
    assert np.allclose(pos[:, 1], (2.5 - 0.25 * tc + 0.25 * (1 - tc), 4.0 - 0.3 * (1 - tc)), atol=1e-14)
    assert np.allclose(vel[:, 1], (0.25, -0.3), atol=1e-15)
    assert (pos[1] >= 0).all() and (pos[1] < 4).all()
    assert o.Np == n


# ---------------------------------------------------------------- exchange and interpolation

def test_reinjection_is_maxwellian(oracle_lib):
    """Buffer particles get velocities drawn from the Maxwell-Boltzmann
    distribution about the LB velocity with variance kT/m (Alg. 1)."""
    p = W.small_2d(n=(40, 24, 1), g=(0, 0, 0), alpha_deg=0.0, substeps=1, feedback=0, kT=0.2,
                   mass=2.0)
    o = oracle_lib.Oracle(p)
    pos0, _ = o.particles()
    o.step(1)
    _, vel = o.particles()
    J = np.floor((pos0[1] - p["ylo"]) * p["refine"]).astype(int)
    R = (p["yhi"] - p["ylo"]) * p["refine"]
    buf = (J < p["buf_lo"] * p["refine"]) | (J >= R - p["buf_hi"] * p["refine"])
    sd = np.sqrt(p["kT"] / p["mass"])
    for d in range(2):
        z = vel[d, buf] / sd
        assert stats.kstest(z, "norm").pvalue > 1e-3
        assert abs(stats.skew(z)) < 0.05 and abs(stats.kurtosis(z)) < 0.1
    # interior particles keep the initial thermal velocities
    assert buf.sum() == o.Np // 2


def test_interpolation_exact_for_linear_field(oracle_lib):
    """Bilinear interpolation (Alg. 2) reproduces a field linear in y exactly."""
    p = W.small_2d(feedback=0)
    o = oracle_lib.Oracle(p)
    nx, ny, _ = p["n"]
    y = np.arange(ny) + 0.5
    ux = 1e-3 + 2e-4 * y
    uy = -3e-4 + 1e-4 * y
    f = np.stack([oracle_lib.feq(2, 1.0, (ux[j] - 0.5 * p["g"][0], uy[j])) for j in range(ny)], axis=1)
    o.set_f(np.repeat(f[:, None, :, None], nx, axis=3))
    o.refresh_ufine()
    uf = o.ufine()
    r = p["refine"]
    R = o.R
    for J in list(range(p["buf_lo"] * r)) + list(range(R - p["buf_hi"] * r, R)):
        Y = p["ylo"] + (J + 0.5) / r
        assert np.allclose(uf[0, 0, J], 1e-3 + 2e-4 * Y, rtol=0, atol=1e-16)
        assert np.allclose(uf[1, 0, J], -3e-4 + 1e-4 * Y, rtol=0, atol=1e-16)
    interior = slice(p["buf_lo"] * r, R - p["buf_hi"] * r)
    assert (uf[:, :, interior] == 0).all()


# ---------------------------------------------------------------- whole-step invariants

@pytest.mark.parametrize("maker", [W.small_2d, W.small_3d, W.walled_2d])
def test_particles_conserved_and_inside(oracle_lib, maker):
    p = maker()
    o = oracle_lib.Oracle(p)
    n0 = o.Np
    o.step(3)
    pos, vel = o.particles()
    assert o.Np == n0
    nx, ny, nz = p["n"]
    assert ((pos[0] >= 0) & (pos[0] < nx)).all()
    assert ((pos[1] >= p["ylo"]) & (pos[1] < p["yhi"])).all()
    if p["dim"] == 3:
        assert ((pos[2] >= 0) & (pos[2] < nz)).all()
    b = o.binning()
    assert b["count"].sum() == n0
    assert np.isfinite(vel).all()


@pytest.mark.parametrize("dim", [2, 3])
def test_periodic_box_momentum_energy(oracle_lib, dim):
    """In a periodic box with g = 0, SRD collisions and streaming conserve
    total momentum and kinetic energy (local conservation, Sec. 2.2)."""
    if dim == 2:
        p = W.periodic_2d(n=(6, 6, 1))
    else:
        p = W.make(dim=3, n=(4, 4, 4), walls_y=0, ylo=0, yhi=4, buf_lo=0, buf_hi=0, refine=2,
                   ppc=5, g=(0, 0, 0), feedback=0, alpha_deg=120.0)
    o = oracle_lib.Oracle(p)
    _, v0 = o.particles()
    o.step(5)
    _, v1 = o.particles()
    assert np.abs(v1.sum(1) - v0.sum(1)).max() < 1e-12 * np.abs(v0).sum()
    assert abs((v1 ** 2).sum() - (v0 ** 2).sum()) < 1e-12 * (v0 ** 2).sum()
    assert np.abs(v1 - v0).max() > 0.1  # velocities did change


def test_equipartition_and_maxwellian_bulk(oracle_lib):
    """Equilibrium: <m v_d^2> = kT per component, Maxwellian after mixing."""
    p = W.periodic_2d(n=(16, 16, 1), ppc=10, kT=0.5, mass=1.5)
    o = oracle_lib.Oracle(p)
    o.step(10)
    _, v = o.particles()
    for d in range(2):
        assert abs(p["mass"] * (v[d] ** 2).mean() - p["kT"]) < 0.02 * p["kT"]
        assert stats.kstest(v[d] / np.sqrt(p["kT"] / p["mass"]), "norm").pvalue > 1e-3


def test_gravity_momentum_gain_periodic(oracle_lib):
    """Every particle gains g dt of velocity per MPCD step (body force)."""
    g = (1e-3, 0.0, 0.0)
    p = W.periodic_2d(n=(6, 6, 1), g=g)
    o = oracle_lib.Oracle(p)
    _, v0 = o.particles()
    o.step(4)
    _, v1 = o.particles()
    assert abs((v1[0].sum() - v0[0].sum()) - o.Np * g[0] * 4) < 1e-10
    assert abs(v1[1].sum() - v0[1].sum()) < 1e-10


def test_init_exact_occupancy(oracle_lib):
    p = W.small_3d()
    o = oracle_lib.Oracle(p)
    pos, vel = o.particles()
    r = p["refine"]
    I = np.floor(pos[0] * r).astype(int)
    J = np.floor((pos[1] - p["ylo"]) * r).astype(int)
    K = np.floor(pos[2] * r).astype(int)
    cl = (K * o.R + J) * (p["n"][0] * r) + I
    assert (np.bincount(cl) == p["ppc"]).all()
    assert (cl == np.arange(o.Np) // p["ppc"]).all()
    for d in range(3):
        assert stats.kstest(vel[d] / np.sqrt(p["kT"]), "norm").pvalue > 1e-3


def test_one_way_coupling_leaves_lb_untouched(oracle_lib):
    """With one-way coupling the LB fields are exactly those of an LB-only run
    (the LB is unaffected by the particles)."""
    p = W.small_2d(feedback=0)
    a = oracle_lib.Oracle(p)
    b = oracle_lib.Oracle({**p, "mpcd": 0})
    a.step(4)
    b.step(4)
    assert (a.f() == b.f()).all()


def test_feedback_sets_node_velocity_to_particle_mean(oracle_lib):
    """Feedback reading with a window of one LB step: with cells equal to LB
    nodes (r = 1, no shift, S = 1) a collision keeps each node's particle
    momentum, so after the next LB step every interior node's velocity
    equals the mean velocity of its particles at the end of the previous
    step."""
    p = W.small_2d(refine=1, grid_shift=0, substeps=1, ppc=30, g=(0, 0, 0), feedback=1, fb_window=1)
    o = oracle_lib.Oracle(p)
    o.step(2)
    pos, vel = o.particles()
    o.step(1)
    _, u, _ = o.moments()
    nx = p["n"][0]
    ix = np.floor(pos[0]).astype(int)
    iy = np.floor(pos[1]).astype(int)
    for y in range(p["ylo"] + p["buf_lo"], p["yhi"] - p["buf_hi"]):
        for x in range(nx):
            sel = (ix == x) & (iy == y)
            if not sel.any():
                continue
            # the sample was taken right after streaming of the last MPCD
            # step; with S = 1 and a cell-aligned grid the collision keeps the
            # node's momentum, so the post-collision particle mean equals it
            assert np.allclose(u[:2, 0, y, x], vel[:, sel].mean(1), atol=1e-13)


@pytest.mark.parametrize("window,init_flow", [(4, 0), (7, 1)])
def test_feedback_running_mean(oracle_lib, window, init_flow):
    """Feedback reading with a window of W LB steps: after n LB steps an
    interior node carries the weighted sum
    (1 - 1/W)^(n-1) u0 + sum_k (1/W)(1 - 1/W)^(n-1-k) ubar_k over the sample
    means ubar_k of LB steps k = 1 .. n-1 (the projection of LB step n uses
    the samples of step n - 1; the first step has none), u0 the node's
    initial velocity; the node's velocity equals it, and so does the running
    mean the oracle reports."""
    g = (1e-4, 0.0, 0.0) if init_flow else (0.0, 0.0, 0.0)
    p = W.small_2d(refine=1, grid_shift=0, substeps=1, ppc=30, g=g, feedback=1, fb_window=window,
                   init_flow=init_flow)
    o = oracle_lib.Oracle(p)
    lam = 1.0 / window
    nx, ylo, yhi = p["n"][0], p["ylo"], p["yhi"]
    rows = range(ylo + p["buf_lo"], yhi - p["buf_hi"])
    means = []
    n = 9
    for _ in range(n):
        o.step(1)
        acc = o.step_acc()[0]  # [R][nx][4], r = 1: one fine row per node row
        means.append(acc[:, :, 1:3] / acc[:, :, :1])
    _, u, _ = o.moments()
    fb = o.fb_u()
    for y in rows:
        J = y - ylo
        yc = y + 0.5
        H, nu, tau = p["n"][1], (p["tau"] - 0.5) / 3.0, p["tau"]
        u0 = (g[0] * yc * (H - yc) / (2 * nu) + g[0] * (16 * tau * tau - 16 * tau + 1) / (24 * nu)) if init_flow else 0.0
        exp = np.zeros((nx, 2))
        exp[:, 0] = (1 - lam) ** (n - 1) * u0
        for k in range(1, n):
            exp += lam * (1 - lam) ** (n - 1 - k) * means[k - 1][J]
        assert np.allclose(fb[:2, 0, J, :].T, exp, rtol=0, atol=1e-13)
        assert np.allclose(u[:2, 0, y, :].T, exp, rtol=0, atol=1e-13)


def test_profile_counts(oracle_lib):
    p = W.small_2d()
    o = oracle_lib.Oracle(p)
    o.step(1)
    o.sample(1)
    o.step(3)
    acc, nsteps = o.profile()
    # every particle is sampled once per LB step (after the streaming of its
    # last MPCD step) while sampling is on
    assert nsteps == 3
    assert acc[:, 0].sum() == o.Np * 3
    o.sample(0)
    o.step(1)
    acc2, nsteps2 = o.profile()
    assert nsteps2 == 3 and (acc2 == acc).all()


def test_profile_is_row_average_of_samples(oracle_lib):
    """With alpha = 0 the collision is the identity, so with one MPCD step per
    LB step the samples taken after streaming are the particle states seen
    after each step: the profile is their per-fine-row sum (brute force)."""
    p = W.small_2d(alpha_deg=0.0, substeps=1)
    o = oracle_lib.Oracle(p)
    o.sample(1)
    ref = np.zeros((o.R, 4))
    for _ in range(3):
        o.step(1)
        pos, vel = o.particles()
        J = np.clip(np.floor((pos[1] - p["ylo"]) * p["refine"]).astype(int), 0, o.R - 1)
        ref[:, 0] += np.bincount(J, minlength=o.R)
        for d in range(2):
            ref[:, 1 + d] += np.bincount(J, weights=vel[d], minlength=o.R)
    acc, _ = o.profile()
    assert (acc[:, 0] == ref[:, 0]).all()
    assert np.abs(acc[:, 1:3] - ref[:, 1:3]).max() < 1e-11


def test_feedback_samples_only_interior_rows(oracle_lib):
    """The feedback projects the interior slab nodes only, so its per-LB-step
    samples are taken in the interior fine rows (every particle there, once)
    and none in the buffer rows, while the time-averaged profile takes every
    row."""
    p = W.small_2d(alpha_deg=0.0, substeps=1)
    o = oracle_lib.Oracle(p)
    o.sample(1)
    o.step(1)
    pos, _ = o.particles()
    r = p["refine"]
    R = (p["yhi"] - p["ylo"]) * r
    J = np.clip(np.floor((pos[1] - p["ylo"]) * r).astype(int), 0, R - 1)
    acc = o.step_acc()[0]  # [R][nx][4]
    rows = acc[:, :, 0].sum(axis=1)
    interior = (np.arange(R) >= p["buf_lo"] * r) & (np.arange(R) < R - p["buf_hi"] * r)
    assert (rows[~interior] == 0).all()
    assert (rows[interior] == np.bincount(J, minlength=R)[interior]).all()
    prof, _ = o.profile()
    assert (prof[:, 0] == np.bincount(J, minlength=R)).all()
