"""The deterministic mode (parameter `deterministic`): the particle kernel's
sums -- cell velocity sums, MPCD-AT thermostat sums, the feedback's node
samples and the profile rows -- are fixed-point integer atomics, so two runs
of the same parameters give the same bits whatever order the atomics land
in.  Each case runs twice from a fresh context and every field is compared
bit for bit; the run also matches the oracle at the parity tolerance (the
fixed-point sums differ from FP64 sums by at most 2^-41 per value)."""
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
    from paper_2004_00304_amd import lbmpcd
    return torch, lbmpcd


CASES = {
    # binary32 particles, feedback (node samples through the LDS windows)
    "small_3d_fp32_feedback": ([W.small_3d(part_fp=32, deterministic=1)], 8, RTOL32),
    # walls, virtual particles and the MPCD-AT sums, binary64
    "walled_2d_at": ([W.walled_2d(collision=1, deterministic=1)], 10, RTOL64),
    # a batch of uneven channels sharing one launch
    "batch_2d": ([W.small_2d(n=(40 + 8 * i, 24, 1), instance=i, deterministic=1) for i in range(3)], 6, RTOL64),
}


def _run(lbmpcd, plist, steps):
    sim = lbmpcd.Sim(plist)
    sim.sample(1)
    sim.step(steps)
    sim.sync()
    out = {}
    # the binning (with the cell velocities) exists until particles are read
    for i in range(len(plist)):
        b = sim.binning(i)
        out[f"count{i}"], out[f"vcm{i}"] = b["count"], b["vcm"]
    for i, p in enumerate(plist):
        out[f"f{i}"] = sim.f(i)
        rho, u, pi = sim.fields(i)
        out[f"u{i}"], out[f"pi{i}"] = u, pi
        pos, vel = sim.particles(i)
        out[f"pos{i}"], out[f"vel{i}"] = pos, vel
        out[f"prof{i}"] = np.asarray(sim.profile(i))
        if p["feedback"]:
            out[f"node_u{i}"] = sim.node_mpcd_u(i)
            out[f"fb_u{i}"] = sim.node_fb_u(i)
    sim.close()
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_two_runs_are_bit_identical(env, name):
    torch, lbmpcd = env
    plist, steps, _ = CASES[name]
    a = _run(lbmpcd, plist, steps)
    b = _run(lbmpcd, plist, steps)
    diff = [k for k in a if not np.array_equal(a[k], b[k])]
    banner(f"{name}: {len(a)} fields compared, differing: {diff}")
    assert not diff


@pytest.mark.parametrize("name", list(CASES))
def test_deterministic_run_matches_the_oracle(env, oracle_lib, name):
    torch, lbmpcd = env
    plist, steps, rtol = CASES[name]
    sim = lbmpcd.Sim(plist)
    sim.step(steps)
    sim.sync()
    binnings = {i: sim.binning(i) for i in range(len(plist))}
    for i, p in enumerate(plist):
        orc = oracle_lib.Oracle(p)
        orc.step(steps)
        rep = compare_state(sim, orc, p, rtol, inst=i, binning=binnings[i])
        banner(f"{name}[{i}]: { {k: (f'{v:.1e}' if isinstance(v, float) else v) for k, v in rep.items()} }")
        assert_parity(rep, rtol)
    sim.close()
