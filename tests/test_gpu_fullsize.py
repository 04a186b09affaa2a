"""Parity at the full sizes of the throughput workloads, in the launch
configuration bench.py times (default tiles), on sampled outputs the oracle
computes one by one, plus properties that hold at any size.

3D channel: D3Q19 128x64x64, 167,772,160 binary32 particles.
Thin film:  D3Q19 512x256x256 binary32 populations, 335,544,320 particles.

Checked per run (binning of MPCD step (t-1, S-1) is bit-exact on the sample;
binary32 values within 2e-6 of the thermal scale):
  - cell of 2M sampled particles (oracle binning of the GPU positions);
  - occupancy = histogram of the cell ids, total = particle count;
  - SRD collision of 400 sampled cells (oracle collision of the GPU's
    pre-collision velocities vs the GPU's post-collision velocities and
    centre-of-mass velocities);
  - interpolation of the node velocities to every buffer fine cell;
  - one MPCD step (exchange + streaming) of 200k sampled particles, positions
    and velocities bit-exact (the oracle redraws about the GPU's buffer
    velocities and streams in binary32 as the kernel does); for the 3D
    channel with the Chapman-Enskog exchange the oracle draws with the GPU's
    tensor of each particle's buffer cell.
"""
import numpy as np
import pytest

from paper_2004_00304_amd import workloads as W
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu

TOL32 = 2e-6


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_2004_00304_amd import lbmpcd
    return torch, O, lbmpcd


def _check_run(torch, O, lbmpcd, p, steps, rng):
    dim = p["dim"]
    S = p["substeps"]
    sz = W.sizes(p)
    Np = sz["particles"]
    banner(f"full-size {p['n']} Np={Np} S={S}")
    sim = lbmpcd.Sim(p, device="cuda:0")
    probe = O.Probe(p)
    sim.step(steps)
    t_last = steps - 1
    sh = probe.shift(t_last, S - 1)
    st = sim.stats()
    assert st["dropped"] == 0 and st["misplaced"] == 0, st
    # the default tiles' sample windows fit in LDS: the samples that miss them
    # are particles re-wrapped across the slab or (one MPCD step per LB step)
    # a node beyond the window's margin, about as many as the far moves; a
    # window that did not fit would miss every sample
    samples = st["particles"] * st["lb_steps"]
    assert st["window_misses"] <= st["far_moves"] + 0.02 * samples, st

    pos = sim.get_state(lbmpcd.PART_POS).view(dim, Np)
    vpre = sim.get_state(lbmpcd.PART_VEL_PENDING).view(dim, Np)
    cell = sim.moments(lbmpcd.CELL_ID)
    count = sim.moments(lbmpcd.CELL_COUNT)
    vcm = sim.moments(lbmpcd.CELL_VCM).view(dim, -1)
    vpost = sim.get_state(lbmpcd.PART_VEL).view(dim, Np)

    # occupancy is the histogram of the cell ids
    hist = torch.bincount(cell.long(), minlength=sz["ncells"])
    assert int(hist.sum()) == Np
    assert torch.equal(hist.to(torch.int32), count)

    # binning of sampled particles, bit-exact
    ids = torch.from_numpy(rng.choice(Np, size=min(Np, 2_000_000), replace=False)).to(pos.device)
    ps = pos[:, ids].cpu().numpy()
    c_ref = probe.bin(sh, ps)
    mism = int((c_ref != cell[ids].cpu().numpy()).sum())
    banner(f"binning mismatches {mism} / {len(ids)}")
    assert mism == 0

    # collision of sampled occupied cells
    occ = torch.nonzero(count > 1).squeeze(1)
    pick = occ[torch.from_numpy(rng.choice(len(occ), size=400, replace=False)).to(occ.device)]
    member = torch.isin(cell, pick.to(torch.int32))
    idx = torch.nonzero(member).squeeze(1)
    cm = cell[idx].cpu().numpy()
    vp = vpre[:, idx].cpu().numpy()
    vq = vpost[:, idx].cpu().numpy()
    vc = vcm[:, pick].cpu().numpy()
    scale = np.sqrt(p["kT"] / p["mass"])
    worst = 0.0
    worst_cm = 0.0
    for j, c in enumerate(pick.cpu().numpy()):
        sel = np.nonzero(cm == c)[0]
        v_ref, vcm_ref = probe.collide_cell(int(c), t_last, S - 1, sh, vp[:, sel])
        worst = max(worst, float(np.abs(v_ref - vq[:, sel]).max()) / scale)
        worst_cm = max(worst_cm, float(np.abs(vcm_ref - vc[:, j]).max()) / scale)
    banner(f"collision: max |dv|/v_th = {worst:.3e}, max |dvcm|/v_th = {worst_cm:.3e}")
    assert worst <= TOL32 and worst_cm <= 1e-12

    # interpolation to the buffer fine cells from the GPU's node velocities
    u = sim.moments(lbmpcd.U).cpu().numpy().reshape((3,) + tuple(reversed(p["n"])))
    uf_ref = probe.interpolate(u)
    uf = sim.ufine()
    err_uf = float(np.abs(uf - uf_ref).max() / max(np.abs(uf_ref).max(), 1e-12))
    banner(f"interpolation rel err {err_uf:.3e}")
    assert err_uf < 1e-12

    # one more LB step with the particles completed: the first MPCD step is
    # exchange + streaming of the collided state; check it on sampled
    # particles against the oracle (positions and velocities bit-exact)
    pos0 = pos[:, :].clone()
    vel0 = vpost.clone()
    del vpre, vpost, pos
    ids2 = torch.from_numpy(rng.choice(Np, size=200_000, replace=False)).to(pos0.device)
    r0 = pos0[:, ids2].cpu().numpy()
    v0 = vel0[:, ids2].cpu().numpy()
    del pos0, vel0
    return sim, probe, ids2, r0, v0, t_last


def _check_stream(torch, O, lbmpcd, p, sim, probe, ids2, r0, v0, t_last):
    """With one MPCD step per LB step the state after the next lbmpcd_step,
    read before its collision, is exactly exchange + streaming."""
    dim = p["dim"]
    Np = W.sizes(p)["particles"]
    sim.step(1)
    t = t_last + 1
    pos1 = sim.get_state(lbmpcd.PART_POS).view(dim, Np)[:, ids2].cpu().numpy()
    vel1 = sim.get_state(lbmpcd.PART_VEL_PENDING).view(dim, Np)[:, ids2].cpu().numpy()
    uf = sim.ufine()
    r = p["refine"]
    I = np.clip(np.floor(r0[0] * r).astype(int), 0, uf.shape[3] - 1)
    J = np.clip(np.floor((r0[1] - p["ylo"]) * r).astype(int), 0, uf.shape[2] - 1)
    K = np.clip(np.floor(r0[2] * r).astype(int), 0, uf.shape[1] - 1) if dim == 3 else np.zeros_like(I)
    u = np.stack([uf[d, K, J, I] for d in range(dim)])
    tens = None
    if p.get("reinject", 0):
        tf = sim.tfine()
        tens = np.stack([tf[m, K, J, I] for m in range(6)])
        del tf
    pr, vr = probe.exchange_stream(t, 0, ids2.cpu().numpy().astype(np.uint32), r0, v0, u, tens)
    dpos = np.abs(pr - pos1)
    for k, Lk in enumerate(p["n"][:dim]):
        if k != 1:
            dpos[k] = np.minimum(dpos[k], Lk - dpos[k])
    scale = np.sqrt(p["kT"] / p["mass"])
    banner(f"stream: max |dpos| {dpos.max():.3e}, max |dv|/v_th {np.abs(vr - vel1).max() / scale:.3e}, "
           f"identical positions {np.mean(pr == pos1):.6f}, velocities {np.mean(vr == vel1):.6f}")
    # the probe redraws about the GPU's own buffer velocities and streams in
    # binary32 exactly as the kernel does: both bit-exact
    assert np.array_equal(pr, pos1)
    assert np.array_equal(vr, vel1)


def _channel_3d_ce():
    return W.make(**{**W.channel_3d(), "reinject": 1})


@pytest.mark.parametrize("maker,steps", [(W.channel_3d, 3), (W.thin_film_3d, 2), (_channel_3d_ce, 3)],
                         ids=["channel_3d", "thin_film_3d", "channel_3d_ce"])
def test_fullsize_sampled(env, maker, steps):
    torch, O, lbmpcd = env
    rng = np.random.default_rng(7)
    p = maker()
    sim, probe, ids2, r0, v0, t_last = _check_run(torch, O, lbmpcd, p, steps, rng)
    del sim
    torch.cuda.empty_cache()
    # the streaming check at the same sizes with one MPCD step per LB step
    q = dict(p, substeps=1)
    sim, probe, ids2, r0, v0, t_last = _check_run(torch, O, lbmpcd, q, steps, rng)
    _check_stream(torch, O, lbmpcd, q, sim, probe, ids2, r0, v0, t_last)
    del sim
    torch.cuda.empty_cache()
