"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeds, element by element.  FP64: every field within 1e-11 of its scale;
binning (cell of every particle, cell counts) bit-exact.  Binary32 particle
stores: within 2e-6 of the thermal scale, binning bit-exact."""
import numpy as np
import pytest

from paper_2004_00304_amd import workloads as W
from tests.gpu_util import RTOL32, RTOL64, assert_parity, banner, compare_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_2004_00304_amd import lbmpcd
    return O, lbmpcd


CASES = {
    "channel_2d_fp64": (W.channel_2d(), 10, RTOL64),
    "small_2d_oneway": (W.small_2d(feedback=0), 6, RTOL64),
    "small_2d_ragged_tiles": (W.small_2d(n=(37, 24, 1), tile=(8, 4, 0)), 5, RTOL64),
    "small_3d_fp64": (W.small_3d(), 5, RTOL64),
    "small_3d_fp32": (W.small_3d(part_fp=32), 5, RTOL32),
    "small_3d_lb32": (W.small_3d(lb_fp=32, part_fp=32), 4, 2e-6),
    "walled_2d": (W.walled_2d(), 6, RTOL64),
    "walled_2d_fp32": (W.walled_2d(part_fp=32, ppc=5), 6, RTOL32),
    # particle mass other than 1: the virtual wall particles' velocity sum
    # (variance (N0 - n) kT/m) and every kT/m of the exchange
    "walled_2d_mass2": (W.walled_2d(mass=2.0, kT=0.5), 6, RTOL64),
    "walled_2d_fp32_mass05": (W.walled_2d(part_fp=32, ppc=5, mass=0.5, kT=0.2), 6, RTOL32),
    "at_walled_2d_mass2": (W.walled_2d(collision=1, mass=2.0), 6, RTOL64),
    "small_2d_mass3": (W.small_2d(mass=3.0), 5, RTOL64),
    # the feedback's running mean: a window of one LB step (the last sample
    # alone) and of seven, from the Poiseuille start
    "fb_window1_2d": (W.small_2d(fb_window=1), 6, RTOL64),
    "fb_window7_3d_flow": (W.small_3d(fb_window=7, init_flow=1, g=(1e-4, 0, 0)), 6, RTOL64),
    "periodic_2d": (W.periodic_2d(), 6, RTOL64),
    "no_shift": (W.small_2d(grid_shift=0), 4, RTOL64),
    "poiseuille_init": (W.small_2d(init_flow=1, g=(2e-5, 0, 0)), 4, RTOL64),
    # launch shapes: the results do not depend on how the step is cut into work
    "shape_small_tiles_wg512": (W.small_3d(tile_target=160, wg_threads=512), 4, RTOL64),
    "shape_large_tiles": (W.small_2d(tile_target=1280), 4, RTOL64),
    "shape_wg512_fp32": (W.small_3d(part_fp=32, wg_threads=512), 4, RTOL32),
    "shape_linear_order_fp32": (W.small_3d(part_fp=32, schedule=1), 4, RTOL32),
    # the tile's LDS window of buffer-cell LB velocities read by the exchange:
    # a window larger than its table (17 x 9 x 2 cells: every buffer particle
    # reads global memory) and a tile wider than the channel (the window wraps
    # onto itself); the feedback makes the LB velocity vary along x and z
    "lbwin_too_large_3d": (W.small_3d(tile=(16, 8, 1), init_flow=1, g=(1e-4, 0, 0)), 5, RTOL64),
    "lbwin_tile_wider_than_channel_2d": (W.small_2d(n=(3, 24, 1), tile=(16, 4, 0), init_flow=1, g=(1e-4, 0, 0)),
                                         6, RTOL64),
    # MPCD with Andersen thermostat (Eq. 6), the paper's own collision rule
    "at_small_2d": (W.small_2d(collision=1), 6, RTOL64),
    "at_small_3d": (W.small_3d(collision=1), 5, RTOL64),
    "at_walled_2d": (W.walled_2d(collision=1), 6, RTOL64),
    "at_small_3d_fp32": (W.small_3d(part_fp=32, collision=1), 5, RTOL32),
    # edge cases: a refinement that is not a power of two (cell index by
    # division), a = 1, one particle per cell (empty and singleton cells), one
    # MPCD step per LB step, a domain smaller than one tile
    "refine3_2d": (W.small_2d(refine=3), 5, RTOL64),
    "refine3_3d_fp32": (W.small_3d(refine=3, part_fp=32), 4, RTOL32),
    "refine1_2d": (W.small_2d(refine=1, ppc=20), 5, RTOL64),
    "ppc1_3d": (W.small_3d(ppc=1), 5, RTOL64),
    "substeps1_2d": (W.small_2d(substeps=1), 6, RTOL64),
    "tiny_2d": (W.small_2d(n=(4, 12, 1), ylo=4, yhi=8, buf_lo=1, buf_hi=1), 6, RTOL64),
    # Chapman-Enskog exchange about a sheared LB (envelope ~1.3: about a
    # quarter of the first attempts are rejected)
    "ce_small_2d": (W.small_2d(reinject=1, init_flow=1, g=(1e-4, 0, 0), ce_nu=2.0), 6, RTOL64),
    "ce_small_2d_oneway": (W.small_2d(reinject=1, init_flow=1, g=(1e-4, 0, 0), ce_nu=2.0, feedback=0),
                           4, RTOL64),
    "ce_small_3d": (W.small_3d(reinject=1, init_flow=1, g=(1e-4, 0, 0), ce_nu=2.0), 5, RTOL64),
    "ce_small_3d_fp32": (W.small_3d(reinject=1, init_flow=1, g=(1e-4, 0, 0), ce_nu=2.0, part_fp=32),
                         5, RTOL32),
    # driven along z: the yz component of the tensor carries the shear
    "ce_small_3d_gz": (W.small_3d(reinject=1, init_flow=1, g=(0, 0, 1e-4), ce_nu=2.0), 5, RTOL64),
    "ce_at_small_2d": (W.small_2d(reinject=1, init_flow=1, g=(1e-4, 0, 0), collision=1), 6, RTOL64),
    "ce_at_small_3d": (W.small_3d(reinject=1, init_flow=1, g=(1e-4, 0, 0), ce_nu=1.0, collision=1),
                       5, RTOL64),
    # slab on the bottom wall, one buffer towards the LB (virtual wall
    # particles, specular reflection at the LB face), SRD at 90 degrees with
    # its own (negative) post-collision stress coefficient
    "ce_near_wall_2d": (W.make(n=(16, 24, 1), ylo=0, yhi=10, buf_lo=0, buf_hi=2, refine=2, ppc=8,
                               alpha_deg=90.0, reinject=1, init_flow=1, g=(2e-4, 0, 0), feedback=0), 6, RTOL64),
}


def _params(p):
    return {k: v for k, v in p.items() if k not in ("tile",)}


@pytest.mark.parametrize("name", list(CASES))
def test_parity(env, name):
    O, lbmpcd = env
    p, steps, rtol = CASES[name]
    banner(f"parity {name} steps={steps} n={p['n']} dim={p['dim']}")
    sim = lbmpcd.Sim(p)
    orc = O.Oracle(_params(p))
    sim.step(steps)
    orc.step(steps)
    rep = compare_state(sim, orc, p, rtol)
    banner(f"{name}: {rep}")
    assert_parity(rep, rtol)


def test_parity_lb_only(env):
    O, lbmpcd = env
    for dim in (2, 3):
        p = W.make(dim=dim, n=(9, 12, 7) if dim == 3 else (33, 17, 1), mpcd=0, tau=0.7, g=(3e-5, 0, 0))
        banner(f"lb-only dim={dim}")
        sim = lbmpcd.Sim(p)
        orc = O.Oracle(p)
        sim.step(25)
        orc.step(25)
        rep = compare_state(sim, orc, p, RTOL64)
        assert_parity(rep, 1e-13)


def test_parity_step_splitting(env):
    """Results do not depend on how the steps are split across calls or on
    reading the particles in between (the pending collision is completed the
    same way)."""
    O, lbmpcd = env
    p = W.small_2d()
    a = lbmpcd.Sim(p)
    b = lbmpcd.Sim(p)
    orc = O.Oracle(p)
    a.step(6)
    for k in range(3):
        b.step(2)
        if k < 2:
            b.particles()  # completes the pending collision between calls
    orc.step(6)
    ra = compare_state(a, orc, p, RTOL64)
    rb = compare_state(b, orc, p, RTOL64)
    assert_parity(ra, RTOL64)
    assert_parity(rb, RTOL64)


def test_parity_profile_sampling(env):
    O, lbmpcd = env
    p = W.small_2d()
    sim = lbmpcd.Sim(p)
    orc = O.Oracle(p)
    sim.step(2)
    orc.step(2)
    sim.sample(1)
    orc.sample(1)
    sim.step(3)
    orc.step(3)
    pg = sim.profile()
    po, nsteps = orc.profile()
    assert sim.stats()["sampled_steps"] == nsteps == 3
    assert (pg[:, 0] == po[:, 0]).all()
    assert np.abs(pg[:, 1:3] - po[:, 1:3]).max() <= 1e-11 * np.abs(po[:, 0]).max()


def test_parity_set_state_roundtrip(env):
    O, lbmpcd = env
    p = W.small_2d()
    sim = lbmpcd.Sim(p)
    orc = O.Oracle(p)
    rng = np.random.default_rng(4)
    pos, vel = orc.particles()
    vel = vel + 0.01 * rng.standard_normal(vel.shape)
    orc.set_particles(pos, vel)
    sim.set_state("vel", vel.reshape(-1))
    f = orc.f() * (1 + 1e-3 * rng.standard_normal(orc.f().shape))
    orc.set_f(f)
    sim.set_state("pop", f.reshape(-1))
    sim.step(3)
    orc.step(3)
    rep = compare_state(sim, orc, p, RTOL64)
    assert_parity(rep, RTOL64)


@pytest.mark.parametrize("kw", [dict(), dict(reinject=1, init_flow=1, g=(1e-4, 0.0, 0.0)), dict(mixed=1)],
                         ids=["maxwell_boltzmann", "chapman_enskog", "mixed_feedback"])
def test_batched_instances_match_standalone(env, kw):
    """A batch of uneven channels in one context equals each channel run
    alone through the oracle (instance i keyed by (seed, i)); with the
    Chapman-Enskog exchange each instance has its own tensor scale; in the
    mixed batch the middle channel couples one way and the others project
    with windows of their own."""
    O, lbmpcd = env
    if kw.get("mixed"):
        ps = [W.small_2d(n=(24 + 8 * i, 20 + 2 * i, 1), ylo=6, yhi=14, ppc=5 + i, instance=i, init_flow=1,
                         g=(1e-4, 0, 0), feedback=int(i != 1), fb_window=3 + 5 * i) for i in range(3)]
    else:
        ps = [W.small_2d(n=(24 + 8 * i, 20 + 2 * i, 1), ylo=6, yhi=14, ppc=5 + i, instance=i,
                         **(dict(kw, ce_nu=0.5 + i) if kw else {})) for i in range(3)]
    sim = lbmpcd.Sim(ps)
    sim.step(4)
    bins = [sim.binning(i) for i in range(len(ps))]
    for i, p in enumerate(ps):
        orc = O.Oracle(p)
        orc.step(4)
        rep = compare_state(sim, orc, p, RTOL64, inst=i, binning=bins[i])
        banner(f"batch inst {i}: {rep}")
        assert_parity(rep, RTOL64)


@pytest.mark.parametrize("kw", [dict(), dict(collision=1)], ids=["srd", "mpcd_at"])
def test_cell_start_and_node_average(env, kw):
    """CELL_START equals the oracle's stable counting sort offsets (bit-exact)
    and NODE_MPCD_U the mean of the oracle's per-step samples pooled over the
    fine rows of each node (FP64 tolerance)."""
    O, lbmpcd = env
    p = W.small_3d(**kw)
    sim = lbmpcd.Sim(p)
    orc = O.Oracle(_params(p))
    sim.step(3)
    orc.step(3)
    start = sim.cell_start()
    b_o = orc.binning()
    assert np.array_equal(start, b_o["start"])
    un = sim.node_mpcd_u()  # [dim][nz][nsy][nx]
    acc = orc.step_acc()     # [nz][R][nx][4] per fine row
    r = p["refine"]
    nz, R, nx, _ = acc.shape
    pooled = acc.reshape(nz, R // r, r, nx, 4).sum(axis=2)
    cnt = pooled[..., 0]
    ref = np.where((cnt > 0)[..., None], pooled[..., 1:1 + p["dim"]] / np.maximum(cnt, 1)[..., None], 0.0)
    ref = np.moveaxis(ref, -1, 0)
    scale = np.sqrt(p["kT"] / p["mass"])
    err = np.abs(un - ref).max() / scale
    banner(f"node averages: max err {err:.2e} of the thermal velocity; cells {start.size}")
    assert err <= RTOL64


def test_chapman_enskog_at_zero_strain_is_maxwell_boltzmann(env):
    """With the LB at rest (no force, one-way coupling) the tensor vanishes
    to rounding, every first attempt is accepted, and the run draws exactly
    the Maxwell-Boltzmann run's numbers: the two agree to the FP64 parity
    tolerance (the cell sums are FP64 atomics in no fixed order, so two GPU
    runs agree to rounding, not bit for bit; one different draw would be an
    O(1) difference)."""
    O, lbmpcd = env
    p0 = W.small_3d(g=(0.0, 0.0, 0.0), feedback=0)
    banner("chapman-enskog zero strain")
    a = lbmpcd.Sim(p0)
    b = lbmpcd.Sim(dict(p0, reinject=1))
    a.step(3)
    b.step(3)
    assert np.abs(b.tfine()).max() < 1e-15
    rep = compare_state(b, _Mirror(a), p0, RTOL64)
    assert_parity(rep, RTOL64)


class _Mirror:
    """A GPU run presented with the oracle's accessors, for run-to-run
    comparisons through compare_state."""

    def __init__(self, sim):
        self.s = sim

    def f(self):
        return self.s.f(0)

    def moments(self):
        return self.s.fields(0)

    def binning(self):
        return self.s.binning(0)

    def particles(self):
        return self.s.particles(0)

    def ufine(self):
        return self.s.ufine(0)


def test_tfine_needs_the_chapman_enskog_exchange(env):
    O, lbmpcd = env
    sim = lbmpcd.Sim(W.small_2d())
    sim.step(1)
    with pytest.raises(lbmpcd.LbmpcdError) as e:
        sim.tfine()
    assert e.value.code == 5


def test_tile_overflow_is_reported(env):
    """Tiles sized to their initial occupancy plus 64 slots (capacity factor
    1, 31 particles per cell, 8x8-cell tiles: 1984 particles in 2048 slots)
    overflow once the counts fluctuate (about 1.4 standard deviations); the
    kernels drop the excess in bounds (every reader clamps a tile's fill to
    its capacity) and the library reports E_OVERFLOW with the count."""
    O, lbmpcd = env
    banner("tile overflow")
    sim = lbmpcd.Sim(W.small_2d(ppc=31, tile=(8, 8, 0), capacity_factor=1.0))
    with pytest.raises(lbmpcd.LbmpcdError) as e:
        sim.step(10)
        sim.sync()
    assert e.value.code == 4 and "dropped" in str(e.value), str(e.value)


def test_sample_window_misses_are_counted(env):
    """Samples that fall outside their tile's LDS window go to global atomics
    and are counted.  With the default tiles at r = 2 and 4 the window holds
    every node the tile's particles reach except across the slab, so the
    misses are particles re-wrapped from one face to the other (far moves);
    at r = 1 the 3D window of a 4x4x4-cell tile spans 6x6x6 nodes, more than
    the table holds, and every feedback sample (the particles of the slab's
    interior rows; buffer rows are not sampled for the feedback) takes the
    global path (the results do not depend on the path: parity cases
    refine1_2d and small_3d)."""
    O, lbmpcd = env
    banner("sample window misses")
    for p in (W.small_3d(), W.small_2d()):
        sim = lbmpcd.Sim(p)
        sim.step(2)
        st = sim.stats()
        assert st["window_misses"] <= st["far_moves"] + 0.02 * st["particles"] * st["lb_steps"], st
    p = W.small_3d(refine=1, ppc=20)
    sim = lbmpcd.Sim(p)
    sim.step(2)
    st = sim.stats()
    # one feedback sample per particle of the slab's interior rows (3 of its
    # 5) per LB step; buffer rows are not sampled for the feedback
    interior = (p["yhi"] - p["ylo"] - p["buf_lo"] - p["buf_hi"]) / (p["yhi"] - p["ylo"])
    assert abs(st["window_misses"] / (2 * interior * st["particles"]) - 1) < 0.05, st


def test_chapman_enskog_xz_shear_parity(env):
    """The xz component of the Chapman-Enskog tensor: both sides start from
    the same populations of a shear wave u_x(z) (set through lbmpcd_set_state
    and the oracle's set_f) and run the coupled step with the exchange."""
    O, lbmpcd = env
    from tests.test_oracle_ce import shear_wave_f
    p = W.small_3d(reinject=1, g=(0.0, 0.0, 0.0), ce_nu=2.0, feedback=0)
    f = shear_wave_f(p, 0.02)
    banner("chapman-enskog xz shear parity")
    sim = lbmpcd.Sim(p)
    orc = O.Oracle(_params(p))
    sim.set_state(lbmpcd.POP, f)
    orc.set_f(f)
    sim.step(4)
    orc.step(4)
    rep = compare_state(sim, orc, p, RTOL64)
    banner(f"xz shear: {rep}")
    assert_parity(rep, RTOL64)
    assert np.abs(orc.tfine()[4]).max() > 1e-3


OVERFLOW_CASES = {
    "srd_fp32": dict(part_fp=32),
    "at_fp32": dict(part_fp=32, collision=1),
    "srd_fp64": dict(part_fp=64),
    "srd_fp32_deterministic": dict(part_fp=32, deterministic=1),
    "ce_fp32": dict(part_fp=32, reinject=1, init_flow=1, ce_nu=2.0),
}


@pytest.mark.parametrize("case", list(OVERFLOW_CASES))
def test_parity_overflow_pass(env, case):
    """Binary32 SRD, MPCD-AT, deterministic SRD and the Chapman-Enskog
    exchange, and binary64 SRD (256-thread workgroups), particles in tiles of 4x4x2 cells at 45 per cell (1440
    expected, 1984 slots) run as two launches per MPCD step: six slots per
    thread (1536 per tile), then a pass of 512 threads x 4 slots over the tiles that held
    more.  A tile's Poisson count passes 1536 now and then (the oracle's own
    binning of this seed does so by the twelfth LB step); such a tile is
    skipped by the first launch and processed whole by the second.  The run
    matches the oracle, and the largest tile fill seen is above 1536, so the
    second launch took part."""
    O, lbmpcd = env
    kw = OVERFLOW_CASES[case]
    part_fp = kw["part_fp"]
    p = W.small_3d(ppc=45, tile=(4, 4, 2), g=(1e-4, 0.0, 0.0), wg_threads=256, **kw)
    banner(f"parity overflow pass: 45 ppc, 4x4x2 tiles, 12 LB steps, {case}")
    sim = lbmpcd.Sim(p)
    orc = O.Oracle(_params(p))
    sim.step(12)
    orc.step(12)
    rtol = RTOL32 if part_fp == 32 else RTOL64
    rep = compare_state(sim, orc, p, rtol)
    st = sim.stats()
    banner(f"overflow pass: {rep}; max fill {st['max_fill']}")
    assert_parity(rep, rtol)
    assert st["max_fill"] > 1536 and st["dropped"] == 0, st
