"""Oracle of the learned closure: plain FP64 NumPy.  TEST INFRASTRUCTURE ONLY
(imported by tests/ and nothing else); it shares no code with the HIP path.

The closure is not part of the paper: the paper couples LB and MPCD through
the buffer (Sec. 2.3, Alg. 1/2) and reports MPCD profiles; a network that
predicts the MPCD averages from the LB moments is this project's addition.
Parity with any value printed in the paper is therefore unpinned; what pins
this file is mathematics: central finite differences of the loss (the
backward pass), closed forms of GELU and of a first Adam step, exact BF16
rounding of chosen values, and moment identities of the D3Q19 lattice
(Sec. 2.1: rho, u and Pi as moments of the populations).

Conventions mirror the HIP path so that both see the same operands:
  network   271 -> 128 -> 128 -> 128 -> 9, GELU(x) = x Phi(x) between layers;
  rounding  standardised inputs, weights, hidden activations and the
            gradients fed to products are rounded to BF16 (round to nearest
            even, after rounding to binary32); products accumulate exactly
            here (FP32 on the GPU), biases and pre-activations stay unrounded;
  loss      mean squared error over rows x 9 outputs, standardised units;
  Adam      Kingma & Ba with bias-corrected moments.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

NF, NFP, NH, NOUT = 271, 288, 128, 9
LAYERS = [(NH, NFP), (NH, NH), (NH, NH), (NOUT, NH)]  # (out, in) of each weight matrix


def offsets():
    """Offsets of W1 b1 W2 b2 W3 b3 W4 b4 in the flat parameter block."""
    o, out = 0, []
    for (fo, fi) in LAYERS:
        out.append((o, o + fo * fi))
        o += fo * fi + fo
    return out, o


OFFS, NPARAM = offsets()
NSTATS = 2 * NF + 2 * NOUT


def unpack(P):
    """Weights ([out][in]) and biases of the flat block."""
    Ws, bs = [], []
    for (fo, fi), (ow, ob) in zip(LAYERS, OFFS):
        Ws.append(np.asarray(P[ow:ow + fo * fi], np.float64).reshape(fo, fi))
        bs.append(np.asarray(P[ob:ob + fo], np.float64))
    return Ws, bs


def pack(Ws, bs):
    P = np.zeros(NPARAM)
    for (fo, fi), (ow, ob), W, b in zip(LAYERS, OFFS, Ws, bs):
        P[ow:ow + fo * fi] = W.reshape(-1)
        P[ob:ob + fo] = b
    return P


# ---- rounding ------------------------------------------------------------------

def bf16(x):
    """Round to binary32 (nearest), then to BF16 (nearest, ties to even)."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    out = (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def identity(x):
    return np.asarray(x, np.float64)


# ---- activation ----------------------------------------------------------------

def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


# ---- standardisation -------------------------------------------------------------

def stats_of(X, Y):
    """Mean and population standard deviation per column, the latter floored
    at 1e-3 of the mean's magnitude and at 1e-12 (the targets Y here are the
    network's, see network_targets)."""
    def ms(A):
        A = np.asarray(A, np.float64)
        m = A.mean(axis=0)
        s = np.sqrt(np.maximum((A * A).mean(axis=0) - m * m, 0.0))
        s = np.maximum(np.maximum(s, 1e-3 * np.abs(m)), 1e-12)
        return m, s
    mx, sx = ms(X)
    my, sy = ms(Y)
    return np.concatenate([mx, sx, my, sy])


def split_stats(st):
    st = np.asarray(st, np.float64)
    return st[:NF], st[NF:2 * NF], st[2 * NF:2 * NF + NOUT], st[2 * NF + NOUT:]


UC = 13 * 10 + 1  # u_x of the stencil's centre node among the features


def network_targets(X, Y):
    """What the network fits: the velocity relative to the node's own LB
    velocity (the centre stencil entry), the stress as is."""
    T = np.asarray(Y, np.float64).copy()
    T[:, :3] -= np.asarray(X, np.float64)[:, UC:UC + 3]
    return T


def physical_outputs(X, T):
    """Inverse of network_targets."""
    Y = np.asarray(T, np.float64).copy()
    Y[:, :3] += np.asarray(X, np.float64)[:, UC:UC + 3]
    return Y


def standardise(X, st, rnd=bf16):
    mx, sx, _, _ = split_stats(st)
    Xs = np.zeros((X.shape[0], NFP))
    Xs[:, :NF] = (np.asarray(X, np.float64) - mx) / sx
    return rnd(Xs)


# ---- passes ---------------------------------------------------------------------

def forward(P, Xs, rnd=bf16):
    """Xs: standardised (rounded) inputs [n][NFP].  Returns the output in
    standardised units and the cache of the backward pass."""
    Ws, bs = unpack(P)
    Wr = [rnd(W) for W in Ws]
    H = [Xs]
    Z = []
    for l in range(3):
        z = H[-1] @ Wr[l].T + bs[l]
        Z.append(z)
        H.append(rnd(gelu(z)))
    Y = H[-1] @ Wr[3].T + bs[3]
    return Y, dict(Wr=Wr, H=H, Z=Z)


def loss_grad(P, Xs, Yt, rnd=bf16):
    """Mean squared error and its gradient (flat block layout)."""
    Y, c = forward(P, Xs, rnd)
    n = Y.size
    d = Y - Yt
    loss = float((d * d).sum() / n)
    dZ = 2.0 * d / n
    gW, gb = [None] * 4, [None] * 4
    for l in range(3, -1, -1):
        dZr = rnd(dZ)
        gW[l] = dZr.T @ c["H"][l]
        gb[l] = dZ.sum(axis=0)
        if l == 0:
            break
        dZ = (dZr @ c["Wr"][l]) * gelu_grad(c["Z"][l - 1])
    return loss, pack(gW, gb)


def adam(P, G, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * G
    v = b2 * v + (1 - b2) * G * G
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return P - lr * mh / (np.sqrt(vh) + eps), m, v


# ---- coupling: features and targets --------------------------------------------

# D3Q19 velocities in the library's order (rest, +-x, +-y, +-z, xy, xz, yz pairs)
C19 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
                [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], np.float64)
PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def moments(f, g):
    """rho, u = j / rho + g / 2, Pi_ab = sum f (c_a c_b - delta_ab / 3); f: [19][z][y][x]."""
    f = np.asarray(f, np.float64)
    rho = f.sum(axis=0)
    j = np.tensordot(C19.T, f, axes=(1, 0))
    u = j / rho + 0.5 * np.asarray(g, np.float64)[:, None, None, None]
    Pi = np.stack([np.tensordot(C19[:, a] * C19[:, b] - (1.0 / 3.0 if a == b else 0.0), f, axes=(0, 0))
                   for a, b in PAIRS])
    return rho, u, Pi


def features(f, p):
    """[nslab][271] features of the slab nodes (x fastest, then y - ylo, then z)."""
    nx, ny, nz = p["n"]
    rho, u, Pi = moments(np.asarray(f).reshape(19, nz, ny, nx), p["g"])
    M = np.concatenate([rho[None], u, Pi])  # [10][z][y][x]
    ylo, yhi = p["ylo"], p["yhi"]
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ylo, yhi), np.arange(nx), indexing="ij")
    cols = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                sel = M[:, (zz + dz) % nz, np.clip(yy + dy, 0, ny - 1), (xx + dx) % nx]
                cols.append(sel.reshape(10, -1).T)
    F = np.concatenate(cols, axis=1)
    c = M[:, zz, yy, xx].reshape(10, -1)
    r, uc, P = c[0], c[1:4], c[4:10]
    S = [-(P[q] - r * uc[a] * uc[b]) / (2.0 * r * (1.0 / 3.0) * p["tau"]) for q, (a, b) in enumerate(PAIRS)]
    ss = sum((1.0 if q < 3 else 2.0) * S[q] ** 2 for q in range(6))
    return np.concatenate([F, np.sqrt(2.0 * ss)[:, None]], axis=1)


def targets(pos, vel, p, mass=1.0, steps=1):
    """[nslab][9] node mean velocity and kinetic stress sum m (v - u)(v - u)
    per unit volume, for particle sums accumulated over `steps` samples
    (pos, vel: [N][3] of one sample)."""
    nx, ny, nz = p["n"]
    ylo, yhi = p["ylo"], p["yhi"]
    nsy = yhi - ylo
    x = np.clip(np.floor(pos[:, 0]).astype(int), 0, nx - 1)
    y = np.clip(np.floor(pos[:, 1]).astype(int), ylo, yhi - 1)
    z = np.clip(np.floor(pos[:, 2]).astype(int), 0, nz - 1)
    s = (z * nsy + (y - ylo)) * nx + x
    ns = nx * nsy * nz
    cnt = np.bincount(s, minlength=ns).astype(np.float64)
    sv = np.stack([np.bincount(s, weights=vel[:, a], minlength=ns) for a in range(3)], axis=1)
    svv = np.stack([np.bincount(s, weights=vel[:, a] * vel[:, b], minlength=ns) for a, b in PAIRS], axis=1)
    u = np.where(cnt[:, None] > 0, sv / np.maximum(cnt, 1)[:, None], 0.0)
    st = np.stack([mass * (svv[:, q] - cnt * u[:, a] * u[:, b]) / steps for q, (a, b) in enumerate(PAIRS)], axis=1)
    return np.concatenate([u, st], axis=1)
