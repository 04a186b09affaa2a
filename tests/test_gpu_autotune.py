"""The launch-shape autotuner on a small batched ensemble: it measures the
candidates, returns the fastest, and the tuned run still matches the oracle
instance by instance."""
import pytest

from paper_2004_00304_amd import workloads as W
from tests.gpu_util import RTOL64, assert_parity, banner, compare_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_2004_00304_amd import lbmpcd
    return O, lbmpcd


def small_ensemble(n=4):
    # uneven channels like the 256-instance ensemble, scaled down for the oracle
    return [W.make(n=(32 + 16 * i, 16 + 4 * i, 1), ylo=6 + i, yhi=10 + 2 * i, buf_lo=1, buf_hi=1,
                   ppc=5 + 3 * i, instance=i) for i in range(n)]


def test_autotune_picks_a_measured_candidate(env):
    O, lbmpcd = env
    ps = small_ensemble()
    t = lbmpcd.autotune(ps, lb_steps=2)
    banner(f"autotune: {t}")
    assert t["tried"] >= 8
    assert t["tile_target"] in lbmpcd.TUNE_TILE_TARGETS
    assert t["wg_threads"] in (256, 512)
    assert t["schedule"] in (0, 1)
    assert t["ms_per_step"] > 0
    assert t["ms_default"] < 0 or t["ms_per_step"] <= t["ms_default"]
    tuned = lbmpcd.with_tuning(ps, t)
    sim = lbmpcd.Sim(tuned)
    sim.step(3)
    bins = [sim.binning(i) for i in range(len(ps))]
    for i, p in enumerate(ps):
        orc = O.Oracle(p)
        orc.step(3)
        rep = compare_state(sim, orc, tuned[i], RTOL64, inst=i, binning=bins[i])
        banner(f"tuned inst {i}: {rep}")
        assert_parity(rep, RTOL64)
