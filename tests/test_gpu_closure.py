"""The learned closure on the GPU, through the C ABI, against the FP64 oracle
of oracle/mlp.py on identical BF16 operands: the matrix-core product, the
forward pass (1e-2 elementwise, 1e-3 in norm), loss and gradients (1e-2
relative L2 per layer), one Adam step on the FP32 parameters (1e-5 of the
step), the features of the LB state and the particle targets; then that a
trained surrogate reproduces the plain MPCD profile within 2%, is faster
than the plain step, and falls back when it is wrong."""
import time

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
    from oracle import mlp as M
    from paper_2004_00304_amd import lbmpcd
    return torch, M, lbmpcd


def channel(**kw):
    """A small 3D channel with the closure reserved (D3Q19, walls, Poiseuille
    start, slab with 1-row buffers, FP64)."""
    base = dict(dim=3, n=(16, 16, 8), tau=0.8, g=(1e-4, 0.0, 0.0), walls_y=1, init_flow=1, ylo=4, yhi=12,
                buf_lo=1, buf_hi=1, ppc=5, part_fp=64, lb_fp=64, alpha_deg=120.0, feedback=1, closure=1)
    base.update(kw)
    return W.make(**base)


def random_block(M, rng, scale=0.5):
    P = np.zeros(M.NPARAM)
    for (fo, fi), (ow, ob) in zip(M.LAYERS, M.OFFS):
        Wt = rng.normal(0, scale / np.sqrt(min(fi, M.NF)), (fo, fi))
        if fi == M.NFP:
            Wt[:, M.NF:] = 0.0
        P[ow:ow + fo * fi] = Wt.reshape(-1)
        P[ob:ob + fo] = rng.normal(0, 0.1, fo)
    st = np.concatenate([rng.normal(0, 1, M.NF), rng.uniform(0.5, 2, M.NF), rng.normal(0, 1, 9),
                         rng.uniform(0.5, 2, 9)])
    return np.concatenate([P, st]).astype(np.float32)


def raw_data(M, rng, block, n):
    st = block[M.NPARAM:].astype(np.float64)
    mx, sx, my, sy = M.split_stats(st)
    X = (mx + sx * rng.normal(size=(n, M.NF))).astype(np.float32)
    Y = (my + sy * rng.normal(size=(n, 9))).astype(np.float32)
    return X, Y


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("M_,N_,K_", [(100, 70, 300), (64, 64, 32), (1, 9, 128), (257, 128, 288)])
def test_gemm_bf16_matches_exact_product(env, M_, N_, K_):
    """C = A B^T with BF16 inputs: every product of two BF16 numbers is exact
    in FP32, so the only error is FP32 accumulation (~K 2^-24)."""
    torch, M, lbmpcd = env
    rng = np.random.default_rng(M_ + N_ + K_)
    A = torch.tensor(rng.normal(size=(M_, K_)), dtype=torch.bfloat16, device="cuda")
    B = torch.tensor(rng.normal(size=(N_, K_)), dtype=torch.bfloat16, device="cuda")
    Cg = lbmpcd.gemm_bf16(A, B).cpu().numpy().astype(np.float64)
    Ce = A.float().cpu().numpy().astype(np.float64) @ B.float().cpu().numpy().astype(np.float64).T
    err = np.abs(Cg - Ce).max() / np.abs(Ce).max()
    banner(f"gemm {M_}x{N_}x{K_}: max rel err {err:.2e}")
    assert err < 1e-5


def test_forward_and_gradient_match_oracle(env):
    torch, M, lbmpcd = env
    rng = np.random.default_rng(11)
    sim = lbmpcd.Sim(channel())
    block = random_block(M, rng)
    sim.closure_weights(block)
    assert np.array_equal(sim.closure_weights(), block)
    X, Y = raw_data(M, rng, block, 700)
    Xt, Yt = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    P32 = block[:M.NPARAM].astype(np.float64)
    st = block[M.NPARAM:].astype(np.float64)
    mx, sx, my, sy = M.split_stats(st)
    Xs = M.standardise(X, st)
    Ys = (M.network_targets(X, Y) - my) / sy

    out = sim.closure_forward(Xt).cpu().numpy().astype(np.float64)
    yo, _ = M.forward(P32, Xs)
    want = M.physical_outputs(X, yo * sy + my)
    scale = np.abs(want).max()
    el = np.abs(out - want).max() / scale
    nr = rel_l2(out, want)
    banner(f"forward: max {el:.2e}, norm {nr:.2e}")
    assert el <= 1e-2 and nr <= 1e-3

    loss, G = sim.closure_loss_grad(Xt, Yt)
    lo, Go = M.loss_grad(P32, Xs, Ys)
    banner(f"loss gpu {loss:.6g} oracle {lo:.6g}")
    assert abs(loss - lo) <= 1e-3 * lo
    for (fo, fi), (ow, ob) in zip(M.LAYERS, M.OFFS):
        ew = rel_l2(G[ow:ow + fo * fi], Go[ow:ow + fo * fi])
        eb = rel_l2(G[ob:ob + fo], Go[ob:ob + fo])
        banner(f"grad layer {fo}x{fi}: W {ew:.2e} b {eb:.2e}")
        assert ew <= 1e-2 and eb <= 1e-2


def test_adam_step_matches_oracle(env):
    """One training step over all rows in order: the GPU's own gradient goes
    through Adam on the FP32 parameters exactly as in the oracle."""
    torch, M, lbmpcd = env
    rng = np.random.default_rng(12)
    sim = lbmpcd.Sim(channel())
    block = random_block(M, rng)
    sim.closure_weights(block)
    X, Y = raw_data(M, rng, block, 300)
    Xt, Yt = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    _, G = sim.closure_loss_grad(Xt, Yt)
    lr = 1e-3
    sim.closure_train(Xt, Yt, epochs=1, batch=1 << 20, lr=lr)
    after = sim.closure_weights()[:M.NPARAM].astype(np.float64)
    P0 = block[:M.NPARAM].astype(np.float64)
    want, _, _ = M.adam(P0, G.astype(np.float64), np.zeros(M.NPARAM), np.zeros(M.NPARAM), 1, lr)
    err = np.abs(after - want).max()
    banner(f"adam step: max abs err {err:.2e} (step {lr})")
    assert err <= 1e-5 * lr + 1e-7 * np.abs(P0).max()


def test_features_and_targets_match_oracle(env):
    torch, M, lbmpcd = env
    p = channel()
    sim = lbmpcd.Sim(p)
    sim.step(3)
    X = sim.closure_features().cpu().numpy().astype(np.float64)
    Xo = M.features(sim.f(), p)
    colscale = np.maximum(np.abs(Xo).max(axis=0), 1e-12)
    err = (np.abs(X - Xo) / colscale).max()
    banner(f"features: max rel err {err:.2e}")
    assert err <= 2e-6

    Xc, Yc = sim.closure_collect(1)
    pos, vel = sim.particles()  # [3][N] each, the collided state the targets were taken from
    To = M.targets(pos.T, vel.T, p)
    Yg = Yc.cpu().numpy().astype(np.float64)
    sc = np.maximum(np.abs(To).max(axis=0), 1e-12)
    err = (np.abs(Yg - To) / sc).max()
    banner(f"targets: max rel err {err:.2e}")
    assert err <= 2e-6


@pytest.mark.parametrize("kw", [dict(), dict(n=(13, 16, 5), lb_fp=32, part_fp=32)], ids=["fp64", "ragged_fp32"])
def test_fused_prediction_equals_separate_products(env, kw):
    """The surrogate step's fused kernel (band moments, features and the four
    layers in one launch) against the separate path: the feature kernel, then
    one matrix-core product per layer.  Both round the same operands to BF16
    and accumulate the k steps in the same order, so they agree to the last
    bit unless an FP32 sum lands on a BF16 rounding tie; the bound is that of
    the forward pass against the oracle.  The ragged case has 520 slab nodes
    (four full blocks of 128 and a partial one) and FP32 populations."""
    torch, M, lbmpcd = env
    p = channel(**kw)
    sim = lbmpcd.Sim(p)
    sim.step(3)
    X = sim.closure_features()
    rng = np.random.default_rng(5)
    block = random_block(M, rng)
    Xn = X.cpu().numpy().astype(np.float64)
    block[M.NPARAM:] = M.stats_of(Xn, rng.normal(size=(Xn.shape[0], 9))).astype(np.float32)
    sim.closure_weights(block)
    Ys = sim.closure_forward(X).cpu().numpy().astype(np.float64)
    Yf = sim.closure_predict().cpu().numpy().astype(np.float64)
    assert Yf.shape == Ys.shape and np.all(np.isfinite(Yf))
    sc = np.maximum(np.abs(Ys).max(axis=0), 1e-30)
    el = (np.abs(Yf - Ys) / sc).max()
    nrm = rel_l2(Yf, Ys)
    banner(f"fused vs separate ({Xn.shape[0]} rows): max rel {el:.2e}, rel L2 {nrm:.2e}, "
           f"identical {np.mean(Yf == Ys):.4f}")
    assert el <= 1e-2
    assert nrm <= 1e-3


def oneway(**kw):
    """The paper's one-way coupling (feedback 0) on a wider channel: the LB
    does not see the particles, so the surrogate and the plain run share the
    LB state and their MPCD profiles compare directly."""
    base = dict(n=(32, 16, 16), feedback=0)
    base.update(kw)
    return channel(**base)


def _noise_floor(torch, X, Y):
    """The loss a perfect predictor of the window means would reach: half
    the mean square difference of consecutive windows of the same nodes
    (the targets' sampling noise), in the standardised units of the loss,
    averaged over the nine outputs.  Velocity targets are taken relative to
    the node's LB velocity, as the network fits them."""
    UC = 13 * 10 + 1
    R = []
    for x, y in zip(X, Y):
        r = y.clone().double()
        r[:, :3] -= x[:, UC:UC + 3].double()
        R.append(r)
    var = torch.cat(R).var(dim=0)
    dsq = torch.stack([((R[i] - R[i + 1]) ** 2).mean(dim=0) for i in range(0, len(R) - 1, 2)]).mean(dim=0)
    return float((0.5 * dsq / var).clamp(max=1.0).mean())


def _train_closure(lbmpcd, torch, channels, warm=300, windows=2, window=320):
    X, Y = [], []
    for p in channels:
        s = lbmpcd.Sim(p)
        s.step(warm)  # past the MPCD transient from the Poiseuille start
        for _ in range(windows):
            # long windows: the particle noise of the targets averages down
            x, y = s.closure_collect(window)
            X.append(x)
            Y.append(y)
        s.close()
    floor = _noise_floor(torch, X, Y)
    X = torch.cat(X)
    Y = torch.cat(Y)
    trainer = lbmpcd.Sim(channels[0])
    # the loss of the freshly initialised network (a pass with a vanishing step)
    first = trainer.closure_train(X, Y, epochs=1, batch=1024, lr=1e-30, seed=7)
    losses = np.concatenate([trainer.closure_train(X, Y, epochs=60, batch=1024, lr=2e-3),
                             trainer.closure_train(X, Y, epochs=60, batch=1024, lr=3e-4)])
    return trainer.closure_weights(), np.concatenate([first, losses]), X.shape[0], floor


@pytest.fixture(scope="module")
def trained(env):
    torch, M, lbmpcd = env
    cfgs = [oneway(g=(g, 0.0, 0.0), tau=tau) for g in (6e-5, 8e-5, 1e-4, 1.2e-4) for tau in (0.7, 0.8, 0.9)]
    t0 = time.perf_counter()
    block, losses, n, floor = _train_closure(lbmpcd, torch, cfgs)
    banner(f"trained on {n} samples in {time.perf_counter() - t0:.1f} s: loss {losses[0]:.4f} -> {losses[-1]:.4f} "
           f"(noise floor {floor:.4f})")
    return block, losses, floor


def test_training_reduces_the_loss(trained):
    """Against the freshly initialised network the loss falls well down; what
    remains is mostly particle noise of the standardised targets (transverse
    velocities, most stress components), which no network can predict.  The
    noise floor is measured from pairs of windows of the same nodes, and
    training removes most of the loss above it."""
    _, losses, floor = trained
    learned = (losses[0] - losses[-1]) / (losses[0] - floor)
    banner(f"loss: initial {losses[0]:.4f}, final {losses[-1]:.4f}, noise floor {floor:.4f}: "
           f"{100 * learned:.0f} % of the reducible loss learned; epochs {np.round(losses[1:], 4)}")
    assert losses[-1] < losses[0] - 0.05
    assert losses[-1] <= losses[1]
    assert learned >= 0.5


def _profile_u(prof, p):
    """Streamwise velocity of each LB node row between the buffers (the fine
    rows of a node pooled): the resolution the network predicts."""
    r = p["refine"]
    nsy = p["yhi"] - p["ylo"]
    prof = np.asarray(prof).reshape(nsy, r, 4).sum(axis=1)
    rows = range(p["buf_lo"], nsy - p["buf_hi"])
    return np.array([prof[y, 1] / prof[y, 0] for y in rows])


def _lb_profile_u(sim, p):
    """Streamwise LB velocity of each node row between the buffers, averaged
    over x and z: the network-free prediction of the MPCD profile."""
    _, u, _ = sim.fields()  # u [3][nz][ny][nx]
    rows = range(p["ylo"] + p["buf_lo"], p["yhi"] - p["buf_hi"])
    return np.array([u[0, :, y, :].mean() for y in rows])


@pytest.mark.parametrize("g,tau", [(9e-5, 0.8), (7e-5, 0.75)], ids=["g9e-5_tau0.8", "g7e-5_tau0.75"])
def test_surrogate_matches_plain_mpcd_and_is_faster(env, trained, g, tau):
    """Same channel, same LB (one-way coupling): the time-averaged MPCD
    profile of 2000 plain steps against the surrogate's, within 2% (relative
    L2 over the LB node rows between the buffers), at forces and a tau not
    trained on (the grid is g in {6, 8, 10, 12} 1e-5, tau in {0.7, 0.8,
    0.9}); and the surrogate step is faster than the plain one.  The
    network-free prediction -- the LB velocity itself -- misses the MPCD
    profile by more (measured 6.1 % against the surrogate's 0.9 % at tau 0.8,
    3.3 % against 1.9 % at tau 0.75, where the two viscosities are closer): in
    this half-slab channel the MPCD fluid's lower viscosity curves its profile
    away from the LB's, and the network has learnt that from the particles."""
    torch, M, lbmpcd = env
    block, _, _ = trained
    p = oneway(g=(g, 0.0, 0.0), tau=tau)

    def run(surrogate, steps):
        sim = lbmpcd.Sim(p)
        if surrogate:
            sim.closure_weights(block)
            sim.closure_enable(True, tol=0.02, check_every=0)
        sim.step(300)
        sim.sample(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        u = _profile_u(sim.profile(), p)
        if surrogate:
            assert sim.closure_status()["on"]
        return u, dt, _lb_profile_u(sim, p)

    up, t_plain, ulb = run(False, 2000)
    us, t_sur, _ = run(True, 400)
    err = rel_l2(us, up)
    err_lb = rel_l2(ulb, up)
    banner(f"surrogate vs plain profile: rel L2 {err:.4f} (LB velocity alone {err_lb:.4f}); ms/step plain "
           f"{1e3 * t_plain:.3f} surrogate {1e3 * t_sur:.3f}")
    assert np.all(np.isfinite(us))
    assert err <= 0.02
    assert err < 0.75 * err_lb
    assert t_sur < t_plain


def test_wrong_surrogate_falls_back(env, trained):
    """A network whose streamwise output is 3 standard deviations off: the
    periodic check measures it against plain MPCD and falls back."""
    torch, M, lbmpcd = env
    block, _, _ = trained
    bad = block.copy()
    bad[:M.NPARAM] = 0.0
    bad[M.OFFS[3][1]] = 3.0  # streamwise velocity 3 standard deviations off
    p = oneway(g=(9e-5, 0.0, 0.0))
    sim = lbmpcd.Sim(p)
    sim.step(300)
    sim.closure_weights(bad)
    sim.closure_enable(True, tol=0.02, check_every=10, check_steps=40)
    sim.step(30)
    st = sim.closure_status()
    banner(f"fallback: {st}")
    assert st["fell_back"] and not st["on"]
    assert st["last_err"] > 0.02
