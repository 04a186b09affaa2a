"""Long runs of the coupled step (one-way coupling, the paper's Alg. 1/2):
the time-averaged MPCD velocity profile against its analytic form and
against the oracle run on the same seed.

Analytic form (Sec. 3: Poiseuille flow; one-way coupling leaves the LB at
its exact discrete steady state): between the inner faces y_a, y_b of the
buffers the MPCD fluid is driven by the body force and held at the LB
velocity by the buffers, so
    u(y) = u_LB(y_a) + (u_LB(y_b) - u_LB(y_a)) (y - y_a) / (y_b - y_a)
           + g (y - y_a)(y_b - y) / (2 nu_M),
with nu_M the SRD viscosity of a 2D fluid with random grid shift
(kinetic part kT dt / m [N / ((N - 1 + e^-N)(1 - cos 2 alpha)) - 1/2],
collisional part a^2 (1 - cos alpha)(N - 1 + e^-N) / (12 dt N)), or, for
MPCD with Andersen thermostat, nu_M of Eq. 7 at dt = 1/S.  In these
channels the curvature term is a few percent of u, so the check is mostly
of the buffers transferring the LB velocity into the slab."""
import numpy as np
import pytest

from paper_2004_00304_amd import workloads as W
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_2004_00304_amd import lbmpcd
    return O, lbmpcd


def lb_poiseuille(p, y):
    """Exact discrete steady velocity of the forced LB channel with half-way
    bounce-back walls at 0 and H: the parabola plus the slip term of the
    Guo-forced BGK scheme."""
    H = p["n"][1]
    tau = p["tau"]
    nu = (tau - 0.5) / 3.0
    g = p["g"][0]
    return g * y * (H - y) / (2 * nu) + g * (16 * tau * tau - 16 * tau + 1) / (24 * nu)


def nu_srd_2d(p):
    a = 1.0 / p["refine"]
    dt = 1.0 / p["substeps"]
    N = p["ppc"]
    al = np.deg2rad(p["alpha_deg"])
    kin = p["kT"] * dt / p["mass"] * (N / ((N - 1 + np.exp(-N)) * (1 - np.cos(2 * al))) - 0.5)
    col = a * a * (1 - np.cos(al)) * (N - 1 + np.exp(-N)) / (12 * dt * N)
    return kin + col


def nu_at(p):
    """MPCD-AT viscosity, Eq. 7, at the MPCD step dt = 1/S."""
    a = 1.0 / p["refine"]
    dt = 1.0 / p["substeps"]
    N = p["ppc"]
    q = N - 1 + np.exp(-N)
    return p["kT"] * dt / p["mass"] * (N / q - 0.5) + a * a / (12 * dt) * q / N


def analytic(p, y):
    ya = p["ylo"] + p["buf_lo"]
    yb = p["yhi"] - p["buf_hi"]
    ua, ub = lb_poiseuille(p, ya), lb_poiseuille(p, yb)
    nu_m = nu_at(p) if p.get("collision", 0) == 1 else nu_srd_2d(p)
    return ua + (ub - ua) * (y - ya) / (yb - ya) + p["g"][0] * (y - ya) * (yb - y) / (2 * nu_m)


def two_way(p, y):
    """Steady profile of the two-way coupled channel (feedback on), SRD
    slab: the MPCD average is imposed on the LB nodes of the slab interior,
    so the LB between the wall and the first interior node row (centre
    y_a + 1/2) is a parabola with the LB viscosity and the wall slip of the
    forced BGK scheme, u = -g y^2/(2 nu_L) + B y + C, and the MPCD between
    the buffers' inner edges a parabola with nu_M through u(y_a) = U_a:
    u = U_a + g (y - y_a)(H - y_a - y)/(2 nu_M) (symmetric channel).
    Matching the LB at y_a and at the node y_a + 1/2 to the MPCD gives the
    slope B; with nu_M = nu_L the two are one Poiseuille parabola."""
    H = p["n"][1]
    g = p["g"][0]
    tau = p["tau"]
    nu_l = (tau - 0.5) / 3.0
    nu_m = nu_srd_2d(p)
    ya = p["ylo"] + p["buf_lo"]
    C = g * (16 * tau * tau - 16 * tau + 1) / (24 * nu_l)
    B = g * (ya + 0.25) / nu_l + g * (H - 2 * ya - 0.5) / (2 * nu_m)
    Ua = -g * ya * ya / (2 * nu_l) + B * ya + C
    return Ua + g * (y - ya) * (H - ya - y) / (2 * nu_m)


def interior_rows(p):
    r = p["refine"]
    R = (p["yhi"] - p["ylo"]) * r
    J = np.arange(p["buf_lo"] * r, R - p["buf_hi"] * r)
    return J, p["ylo"] + (J + 0.5) / r


def profile_u(prof, J):
    prof = np.asarray(prof).reshape(-1, 4)
    return prof[J, 1] / prof[J, 0]


@pytest.mark.parametrize("collision", [0, 1], ids=["srd", "mpcd_at"])
def test_longrun_profile_matches_analytic(env, collision):
    O, lbmpcd = env
    p = W.make(n=(128, 32, 1), tau=0.8, g=(4e-5, 0.0, 0.0), ylo=12, yhi=20, buf_lo=2, buf_hi=2, ppc=10,
               feedback=0, init_flow=1, collision=collision)
    sim = lbmpcd.Sim(p)
    sim.step(1000)
    sim.sample(1)
    sim.step(20000)
    J, y = interior_rows(p)
    u = profile_u(sim.profile(), J)
    ua = analytic(p, y)
    err = np.linalg.norm(u - ua) / np.linalg.norm(ua)
    nu_m = nu_at(p) if collision else nu_srd_2d(p)
    banner(f"long run vs analytic ({'MPCD-AT' if collision else 'SRD'}): rel L2 {err:.4f}; nu_M {nu_m:.4f}; "
           f"u {np.round(u, 5)}")
    assert err <= 0.01


def test_longrun_two_way_profile_matches_closed_form(env):
    """Feedback on (the running time average of the MPCD velocity projected
    onto the LB equilibria of the slab interior, window 50 LB steps), eight
    independent realizations of the channel (distinct Philox keys) in one
    batched context: every one stays bounded (rho within 5 %, no invalid
    particle or band node), and their mean time-averaged slab profile over
    100,000 LB steps follows the two-way closed form (two parabolas,
    nu_L = 0.1 and nu_M = 0.068) within 1 %, against 7-10 % from the one-way
    form.  The mean is needed: with feedback the MPCD's thermal noise drives
    the LB, whose mean flow then wanders on the viscous time (H^2/nu ~ 10^4
    LB steps), so one realization averaged over 100,000 steps lands 0.1-3 %
    from the closed form (measured 0.47 % for the mean of eight).  Projecting
    the instantaneous sample instead (a window of one LB step) drives this
    channel unstable within a few thousand steps in the oracle, and with
    positions left unchecked such a run once addressed memory out of range;
    both are fixed (the oracle's two-way pins and the range guards)."""
    O, lbmpcd = env
    ps = [W.make(n=(128, 32, 1), tau=0.8, g=(4e-5, 0.0, 0.0), ylo=12, yhi=20, buf_lo=2, buf_hi=2, ppc=10,
                 feedback=1, init_flow=1, instance=i) for i in range(8)]
    p = ps[0]
    J, y = interior_rows(p)
    u2, u1 = two_way(p, y), analytic(p, y)
    # the closed form itself: matched viscosities give the LB parabola
    q = dict(p, tau=0.5 + 3 * nu_srd_2d(p))
    assert np.allclose(two_way(q, y), lb_poiseuille(q, y), rtol=1e-12)
    sim = lbmpcd.Sim(ps)
    sim.step(3000)
    sim.sample(1)
    for _ in range(5):
        sim.step(20000)
        st = sim.stats()
        for i in range(len(ps)):
            rho, _, _ = sim.fields(i)
            assert 0.95 < rho.min() and rho.max() < 1.05, (i, rho.min(), rho.max())
        banner(f"two-way: invalid {st['bad_state']}")
        assert st["bad_state"] == 0
    us = np.array([profile_u(sim.profile(i), J) for i in range(len(ps))])
    each = [np.linalg.norm(u - u2) / np.linalg.norm(u2) for u in us]
    u = us.mean(axis=0)
    e2 = np.linalg.norm(u - u2) / np.linalg.norm(u2)
    e1 = np.linalg.norm(u - u1) / np.linalg.norm(u1)
    banner(f"two-way long run, mean of {len(ps)}: vs two-way form {e2:.4f}, vs one-way form {e1:.4f}; "
           f"each {np.round(each, 4).tolist()}; u {np.round(u, 5)}")
    assert e2 <= 0.01
    assert e1 >= 0.04


def test_longrun_profile_matches_oracle(env):
    """Same channel, same seed, 4000 LB steps in both: the FP64 trajectories
    agree until a rounding-level difference flips a cell, and the
    time-averaged profiles agree within 1% (relative L2 over the interior
    fine rows) either way."""
    O, lbmpcd = env
    p = W.make(n=(32, 16, 1), tau=0.8, g=(5e-5, 0.0, 0.0), ylo=4, yhi=12, buf_lo=2, buf_hi=2, ppc=5,
               feedback=0, init_flow=1)
    steps = 4000
    sim = lbmpcd.Sim(p)
    orc = O.Oracle(p)
    sim.step(200)
    orc.step(200)
    sim.sample(1)
    orc.sample(1)
    sim.step(steps)
    orc.step(steps)
    J, y = interior_rows(p)
    ug = profile_u(sim.profile(), J)
    acc, _ = orc.profile()
    uo = profile_u(acc, J)
    err = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    ea = np.linalg.norm(ug - analytic(p, y)) / np.linalg.norm(analytic(p, y))
    banner(f"long run GPU vs oracle: rel L2 {err:.2e} (vs analytic {ea:.4f})")
    assert err <= 0.01


def mpcd_viscosity(p):
    """The viscosity the library reports for the parameter set (lbmpcd_viscosity)."""
    from paper_2004_00304_amd import lbmpcd
    return lbmpcd.viscosity(p)[1]


@pytest.mark.parametrize("collision,ppc", [(0, 8), (1, 20)], ids=["srd", "mpcd_at"])
def test_mpcd_viscosity_from_poiseuille(env, collision, ppc):
    """Stand-alone MPCD Poiseuille flow between two walls (the slab is the
    whole channel, no buffers; the paper's first set of runs, Sec. 3.1): the
    time-averaged profile is fitted by u0 + c y (H - y), and g / (2 c) is
    the MPCD viscosity, against Eq. 7 (MPCD-AT) or the 2D SRD formula
    (lbmpcd_viscosity), within 5 %.  Both formulas are mean-field: measured
    here SRD at 8 per cell comes out 2 % above its formula, MPCD-AT 2 % above
    Eq. 7 at 20 and 50 per cell but 8 % above at 8 per cell (the paper runs
    MPCD-AT at 60 to 1000 per cell)."""
    O, lbmpcd = env
    p = W.walled_2d(n=(64, 16, 1), g=(2e-4, 0.0, 0.0), collision=collision, init_flow=1, ppc=ppc)
    sim = lbmpcd.Sim(p)
    sim.step(2000)
    sim.sample(1)
    sim.step(16000)
    r, H = p["refine"], p["n"][1]
    prof = np.asarray(sim.profile()).reshape(-1, 4)
    y = (np.arange(prof.shape[0]) + 0.5) / r
    u = prof[:, 1] / prof[:, 0]
    A = np.stack([np.ones_like(y), y * (H - y)], axis=1)
    (u0, c), *_ = np.linalg.lstsq(A, u, rcond=None)
    nu_fit = p["g"][0] / (2.0 * c)
    nu_th = mpcd_viscosity(p)
    banner(f"MPCD Poiseuille ({'MPCD-AT' if collision else 'SRD'}): nu fitted {nu_fit:.4f}, formula {nu_th:.4f}, "
           f"wall slip u0 {u0:.2e}, centre u {u.max():.4f}")
    assert abs(nu_fit / nu_th - 1.0) <= 0.05


def test_mpcd_viscosity_from_poiseuille_3d_srd(env):
    """The same fit in 3D (walls at y = 0 and 16, periodic x and z, SRD at
    120 degrees about random axes, 10 per cell): the library's 3D SRD formula
    (the kinetic and collisional terms of the SRD literature) within 5 %;
    measured 1.4 % above it (1.2 % at 20 per cell, 3.5 % at 90 degrees)."""
    O, lbmpcd = env
    p = W.make(dim=3, n=(16, 16, 8), walls_y=1, ylo=0, yhi=16, buf_lo=0, buf_hi=0, refine=2, ppc=10,
               feedback=0, tau=0.8, alpha_deg=120.0, g=(2e-4, 0.0, 0.0), init_flow=1)
    sim = lbmpcd.Sim(p)
    sim.step(2000)
    sim.sample(1)
    sim.step(12000)
    r, H = p["refine"], p["n"][1]
    prof = np.asarray(sim.profile()).reshape(-1, 4)
    y = (np.arange(prof.shape[0]) + 0.5) / r
    u = prof[:, 1] / prof[:, 0]
    A = np.stack([np.ones_like(y), y * (H - y)], axis=1)
    (u0, c), *_ = np.linalg.lstsq(A, u, rcond=None)
    nu_fit = p["g"][0] / (2.0 * c)
    nu_th = mpcd_viscosity(p)
    banner(f"MPCD Poiseuille 3D SRD: nu fitted {nu_fit:.4f}, formula {nu_th:.4f}")
    assert abs(nu_fit / nu_th - 1.0) <= 0.05


def test_near_wall_coupling_profile(env):
    """The paper's near-wall set-up (Sec. 3.3): the MPCD slab lies on the
    bottom wall and meets the LB through one buffer.  Between the wall (no
    slip) and the buffer's inner face y_b the MPCD profile is the LB velocity
    at y_b carried linearly plus the Poiseuille curvature of the MPCD fluid:
    u(y) = u_LB(y_b) y / y_b + g y (y_b - y) / (2 nu_M); relative L2 within 2 %
    over the interior fine rows."""
    O, lbmpcd = env
    p = W.make(n=(128, 32, 1), tau=0.8, g=(4e-5, 0.0, 0.0), ylo=0, yhi=8, buf_lo=0, buf_hi=2, ppc=10,
               feedback=0, init_flow=1, collision=1)
    sim = lbmpcd.Sim(p)
    sim.step(1000)
    sim.sample(1)
    sim.step(20000)
    r = p["refine"]
    yb = p["yhi"] - p["buf_hi"]
    J = np.arange(0, yb * r)
    y = (J + 0.5) / r
    u = profile_u(sim.profile(), J)
    nu_m = mpcd_viscosity(p)
    ua = lb_poiseuille(p, yb) * y / yb + p["g"][0] * y * (yb - y) / (2 * nu_m)
    err = np.linalg.norm(u - ua) / np.linalg.norm(ua)
    banner(f"near-wall coupling (MPCD-AT): rel L2 {err:.4f}; nu_M {nu_m:.4f}; u {np.round(u, 5)}")
    assert err <= 0.02
