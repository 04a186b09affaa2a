"""Pins of the closure oracle (CPU): BF16 rounding of chosen values, GELU
identities, the backward pass against central finite differences, Adam's
first steps in closed form, and the LB moment features on populations whose
moments are known exactly."""
import numpy as np
import pytest

from oracle import mlp as M


def test_parameter_count():
    # 271*128 + 128 + 2 (128*128 + 128) + 128*9 + 9 real parameters, W1's
    # inputs padded from 271 to 288
    assert M.NPARAM == 71177
    assert 271 * 128 + 128 + 2 * (128 * 128 + 128) + 128 * 9 + 9 == 69001


@pytest.mark.parametrize("x,want", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                 # halfway, ties to the even 1.0
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),  # halfway, ties to the even neighbour above
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),
    # 3e38 = 1.7632.. 2^127; 7 fraction bits: 225.69 / 128 rounds to 226 / 128
    (-2.5, -2.5), (3.0e38, 226.0 * 2.0 ** 120), (0.0, 0.0),
])
def test_bf16_rounding(x, want):
    got = float(M.bf16(np.array([x]))[0])
    assert got == pytest.approx(want, rel=1e-5)
    if x in (1.0, -2.5, 0.0):
        assert got == want


def test_gelu_identities():
    x = np.linspace(-6, 6, 101)
    # Phi(x) + Phi(-x) = 1  =>  gelu(x) - gelu(-x) = x
    assert np.allclose(M.gelu(x) - M.gelu(-x), x, atol=1e-15)
    assert M.gelu(np.array([0.0]))[0] == 0.0
    assert M.gelu_grad(np.array([0.0]))[0] == pytest.approx(0.5, abs=1e-16)
    assert M.gelu(np.array([10.0]))[0] == pytest.approx(10.0, rel=1e-15)
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    assert np.allclose(fd, M.gelu_grad(x), atol=1e-8)


def _random_net(rng, scale=0.3):
    P = np.zeros(M.NPARAM)
    for (fo, fi), (ow, ob) in zip(M.LAYERS, M.OFFS):
        W = rng.normal(0, scale / np.sqrt(fi), (fo, fi))
        if fi == M.NFP:
            W[:, M.NF:] = 0.0
        P[ow:ow + fo * fi] = W.reshape(-1)
        P[ob:ob + fo] = rng.normal(0, 0.1, fo)
    return P


def test_backward_matches_finite_differences():
    """Exact arithmetic (no rounding): central differences of the loss agree
    with the backward pass to 1e-6 relative on sampled parameters of every
    layer."""
    rng = np.random.default_rng(3)
    P = _random_net(rng)
    Xs = np.zeros((7, M.NFP))
    Xs[:, :M.NF] = rng.normal(size=(7, M.NF))
    Yt = rng.normal(size=(7, M.NOUT))
    loss, G = M.loss_grad(P, Xs, Yt, rnd=M.identity)
    idx = []
    for (fo, fi), (ow, ob) in zip(M.LAYERS, M.OFFS):
        idx += list(ow + rng.choice(fo * min(fi, M.NF), 4, replace=False))
        idx += list(ob + rng.choice(fo, 2, replace=False))
    h = 1e-5
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (M.loss_grad(Pp, Xs, Yt, rnd=M.identity)[0] - M.loss_grad(Pm, Xs, Yt, rnd=M.identity)[0]) / (2 * h)
        assert abs(fd - G[i]) <= 1e-6 * max(abs(G[i]), 1e-3), (i, fd, G[i])


def test_padding_inputs_get_no_gradient():
    rng = np.random.default_rng(4)
    P = _random_net(rng)
    Xs = M.standardise(rng.normal(size=(5, M.NF)), np.concatenate([np.zeros(M.NF), np.ones(M.NF),
                                                                    np.zeros(9), np.ones(9)]))
    _, G = M.loss_grad(P, Xs, rng.normal(size=(5, 9)))
    W1 = G[:M.NH * M.NFP].reshape(M.NH, M.NFP)
    assert np.all(W1[:, M.NF:] == 0.0)


def test_adam_closed_form():
    """With constant gradient g the bias-corrected moments are g and g^2, so
    every step moves by -lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    P = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    for t in range(1, 4):
        Pn, m, v = M.adam(P, g, m, v, t, lr=0.01)
        assert np.allclose(Pn - P, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        P = Pn


def _feq19(rho, u):
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    cu = M.C19 @ u
    return w * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (u @ u))


def test_features_of_uniform_equilibrium():
    """f = f_eq(rho, u) everywhere, no force: every stencil node reports rho,
    u and Pi = rho u u (the D3Q19 equilibrium reproduces the second moment),
    and the shear rate vanishes."""
    p = dict(n=(6, 8, 5), g=(0.0, 0.0, 0.0), ylo=3, yhi=5, tau=0.8)
    rho, u = 1.03, np.array([0.02, -0.01, 0.005])
    f = np.repeat(_feq19(rho, u)[:, None], 6 * 8 * 5, axis=1)
    F = M.features(f, p)
    assert F.shape == (6 * 2 * 5, 271)
    node = np.concatenate([[rho], u, [rho * u[a] * u[b] for a, b in M.PAIRS]])
    assert np.allclose(F[:, :270].reshape(-1, 27, 10), node, rtol=0, atol=1e-15)
    assert np.allclose(F[:, 270], 0.0, atol=1e-9)


def test_shear_rate_of_a_known_stress():
    """Adding f_neq_i = 9 w_i c_ix c_iy pi to an equilibrium at rest leaves
    rho and u unchanged and sets Pi_xy = pi exactly (sum w c_x^2 c_y^2 = 1/9
    on D3Q19); then S_xy = -pi / (2 rho tau / 3) and sqrt(2 S:S) =
    3 |pi| / (rho tau)."""
    p = dict(n=(4, 6, 4), g=(0.0, 0.0, 0.0), ylo=2, yhi=4, tau=0.9)
    rho, pi = 1.0, 2e-4
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    f0 = _feq19(rho, np.zeros(3)) + 9 * w * M.C19[:, 0] * M.C19[:, 1] * pi
    f = np.repeat(f0[:, None], 4 * 6 * 4, axis=1)
    F = M.features(f, p)
    assert np.allclose(F[:, 0], rho, atol=1e-15)
    assert np.allclose(F[:, 1:4], 0.0, atol=1e-15)
    assert np.allclose(F[:, 7], pi, rtol=1e-12)  # Pi_xy of the first stencil node
    assert np.allclose(F[:, 270], 3 * abs(pi) / (rho * 0.9), rtol=1e-12)


def test_stencil_wraps_and_clamps():
    """Stencil neighbours: x and z periodic, y clamped to the channel."""
    p = dict(n=(5, 4, 3), g=(0.0, 0.0, 0.0), ylo=0, yhi=2, tau=1.0)
    rho = 1.0 + 0.01 * np.arange(5 * 4 * 3).reshape(3, 4, 5)  # rho(z, y, x)
    f = _feq19(1.0, np.zeros(3))[:, None, None, None] * rho[None]
    F = M.features(f.reshape(19, -1), p)
    # node (x=0, y=0, z=0): first stencil entry (dz, dy, dx) = (-1, -1, -1)
    # -> z = 2 (wrap), y = 0 (clamp), x = 4 (wrap)
    assert F[0, 0] == pytest.approx(rho[2, 0, 4], rel=1e-14)
    # last entry (1, 1, 1) -> (z 1, y 1, x 1)
    assert F[0, 260] == pytest.approx(rho[1, 1, 1], rel=1e-14)


def test_targets_of_simple_particle_sets():
    """All particles of a node with one velocity: mean = v, stress 0; two
    particles +-w about u: stress m (w w + w w) per unit volume."""
    p = dict(n=(2, 4, 1), ylo=1, yhi=3)
    pos = np.array([[0.5, 1.5, 0.5], [0.2, 1.1, 0.9], [1.5, 2.5, 0.5], [1.4, 2.2, 0.1]])
    u = np.array([0.1, 0.0, -0.2])
    w = np.array([0.3, -0.1, 0.2])
    vel = np.array([u, u, u + w, u - w])
    T = M.targets(pos, vel, p)
    assert T.shape == (4, 9)
    assert np.allclose(T[0, :3], u) and np.allclose(T[0, 3:], 0.0, atol=1e-15)
    assert np.allclose(T[3, :3], u)
    want = [2 * w[a] * w[b] for a, b in M.PAIRS]
    assert np.allclose(T[3, 3:], want, rtol=1e-12)
    assert np.allclose(T[1], 0.0) and np.allclose(T[2], 0.0)
