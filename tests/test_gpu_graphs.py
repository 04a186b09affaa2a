"""Steady-state steps replayed from a captured HIP graph give the same state
as direct launches and as the oracle, replay after replay, with eager work and
synchronisations in between."""
import numpy as np
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
    return torch, O, lbmpcd


@pytest.mark.parametrize("maker", [W.small_2d, W.small_3d, lambda: W.small_2d(mpcd=0)])
def test_graph_replays_match(env, maker):
    torch, O, lbmpcd = env
    p = maker()
    g = lbmpcd.Sim(p)
    e = lbmpcd.Sim(p)
    e.graphs(False)
    orc = O.Oracle(p)
    for rep in range(3):
        g.step(5)  # 1 direct step (nothing pending after a read) + 2 graph replays
        e.step(5)
        orc.step(5)
        torch.cuda.synchronize()
        # eager work between replays
        x = torch.ones(1 << 20, device="cuda")
        (x * 2).sum().item()
        rg = compare_state(g, orc, p, RTOL64)
        re = compare_state(e, orc, p, RTOL64)
        banner(f"graph replay {rep}: {rg}")
        assert_parity(rg, RTOL64)
        assert_parity(re, RTOL64)


def test_graph_sampling_recaptures(env):
    torch, O, lbmpcd = env
    p = W.small_2d()
    g = lbmpcd.Sim(p)
    orc = O.Oracle(p)
    g.step(4)
    orc.step(4)
    g.sample(1)
    orc.sample(1)
    g.step(6)
    orc.step(6)
    g.sample(0)
    orc.sample(0)
    g.step(4)
    orc.step(4)
    pg = g.profile()
    po, n = orc.profile()
    assert n == 6 and g.stats()["sampled_steps"] == 6
    assert (pg[:, 0] == po[:, 0]).all()
    assert np.abs(pg[:, 1:3] - po[:, 1:3]).max() <= 1e-11 * po[:, 0].max()
    assert_parity(compare_state(g, orc, p, RTOL64), RTOL64)
