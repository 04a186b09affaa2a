"""Range guards of the particle and band kernels, forced from the host.

A particle that moves more than one period in one MPCD step, or whose
velocity is not finite, must never turn into a cell, tile or slot index
outside the channel: the kernel parks it at the slab's lower corner at rest
and counts it, and the next synchronising call reports E_STATE, as the oracle
does (its step returns the same code).  A band node with a non-finite density
is counted the same way.  Every kernel exits normally in these runs: the
state is invalid, the indices are not."""
import numpy as np
import pytest

from paper_2004_00304_amd import workloads as W
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbmpcd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_00304_amd import lbmpcd as L
    return L


@pytest.mark.parametrize("part_fp", [64, 32])
@pytest.mark.parametrize("bad", ["runaway", "nan", "inf"])
def test_invalid_particle_is_parked_and_reported(lbmpcd, part_fp, bad):
    p = W.small_3d(part_fp=part_fp, feedback=1)
    banner(f"guard: {bad} particle, binary{part_fp}")
    sim = lbmpcd.Sim(p)
    pos, vel = sim.particles()
    # a particle of the slab's interior rows (the exchange step would redraw
    # a buffer particle's velocity before it streams)
    k = int(np.flatnonzero((pos[1] > p["ylo"] + p["buf_lo"] + 0.2) & (pos[1] < p["yhi"] - p["buf_hi"] - 0.2))[0])
    nx, S = p["n"][0], p["substeps"]
    vel[:, k] = {"runaway": (3.0 * nx * S, 0.1, 0.0), "nan": (np.nan, 0.0, 0.0), "inf": (0.0, 0.0, np.inf)}[bad]
    sim.set_state(lbmpcd.PART_VEL, vel.reshape(-1))
    sim.step(1)
    with pytest.raises(lbmpcd.LbmpcdError) as e:
        sim.sync()
    assert e.value.code == 5 and "invalid" in str(e.value), str(e.value)
    st = sim.stats()
    assert st["bad_state"] >= 1 and st["dropped"] == 0, st
    # the latched error stops further steps
    with pytest.raises(lbmpcd.LbmpcdError):
        sim.step(1)


def test_valid_fast_particle_is_not_flagged(lbmpcd):
    """Half a period in one MPCD step is a valid (if absurd) move: wrapped,
    not counted."""
    p = W.small_3d(feedback=0)
    sim = lbmpcd.Sim(p)
    pos, vel = sim.particles()
    vel[:, 7] = (0.5 * p["n"][0] * p["substeps"], 0.0, 0.0)
    sim.set_state(lbmpcd.PART_VEL, vel.reshape(-1))
    sim.step(1)
    sim.sync()
    assert sim.stats()["bad_state"] == 0


def test_nonfinite_band_node_is_reported(lbmpcd):
    p = W.small_2d(feedback=0)
    banner("guard: non-finite band node")
    sim = lbmpcd.Sim(p)
    f = sim.f()
    f[:, 0, p["ylo"] + 1, 3] = np.nan
    sim.set_state(lbmpcd.POP, f.reshape(-1))
    sim.step(1)
    with pytest.raises(lbmpcd.LbmpcdError) as e:
        sim.sync()
    assert e.value.code == 5
    assert sim.stats()["bad_state"] >= 1
