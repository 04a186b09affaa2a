"""Seeded synthetic workloads: parameter sets of the coupled LB-MPCD channel.

This module holds only problem definitions (geometry, physical parameters,
seeds).  It contains none of the method's arithmetic, imports neither the HIP
binding nor the oracle, and is the one piece both of them are driven from.

The paper's test problem is body-force driven Poiseuille flow between two
no-slip walls, periodic along the flow (Sec. 3, Table 1).  The presets below
are that channel at the sizes the throughput and parity work uses.
"""
from __future__ import annotations

import copy

import numpy as np

# Defaults shared by every preset (lattice units: dx = dt_LB = 1).
_BASE = dict(
    dim=2, n=(64, 32, 1), lb_fp=64, tau=1.0, rho0=1.0, g=(1e-6, 0.0, 0.0), walls_y=1,
    mpcd=1, ylo=12, yhi=20, buf_lo=2, buf_hi=2, refine=4, substeps=4, ppc=10,
    part_fp=64, mass=1.0, kT=1.0 / 3.0, alpha_deg=130.0, collision=0, grid_shift=1,
    feedback=1, init_flow=0, seed=1, instance=0,
    # exchange step: 0 Maxwell-Boltzmann, 1 Chapman-Enskog about the LB strain
    # rate with stress coefficient ce_nu (0: the post-collision kinetic stress
    # of the collision rule)
    reinject=0, ce_nu=0.0,
    # feedback: LB steps of the running mean of the node samples that is
    # projected onto the LB equilibria (0 = the library default, 50)
    fb_window=0,
    # 1: order-independent integer sums in the particle kernel (bit-identical runs)
    deterministic=0,
    # particle kernel's tile order: 0 XCD-blocked, 1 linear (launch shape, like tile_target)
    schedule=0,
    # launch configuration of the HIP path (tile shape in cells, tile slot
    # capacity over expected occupancy); 0 = library default
    tile=(0, 0, 0), capacity_factor=0.0, tile_target=0, wg_threads=0, closure=0,
)


def make(**kw) -> dict:
    """A full parameter dict: the defaults overridden by ``kw``."""
    p = copy.deepcopy(_BASE)
    for k, v in kw.items():
        if k not in p:
            raise KeyError(f"unknown parameter {k!r}")
        p[k] = v
    p["n"] = tuple(int(x) for x in p["n"])
    p["g"] = tuple(float(x) for x in p["g"])
    p["tile"] = tuple(int(x) for x in p["tile"])
    return p


# ---- the channel at full size -------------------------------------------------

def channel_2d() -> dict:
    """2D channel: D2Q9 64x32, tau 1, g 1e-6, slab y in [12,20) with 2-row
    buffers, r = 4 (256x32 cells), 10 particles/cell (81,920), SRD 130 deg,
    4 substeps, FP64 everywhere."""
    return make()


def channel_3d() -> dict:
    """3D channel: D3Q19 128x64x64, tau 0.8, slab y in [24,40) (16 rows) with
    2-row buffers, r = 4 (512x64x256 cells), 20 particles/cell (167,772,160),
    SRD 120 deg about a random axis, FP32 particles with FP64 cell sums."""
    return make(dim=3, n=(128, 64, 64), tau=0.8, ylo=24, yhi=40, buf_lo=2, buf_hi=2,
                ppc=20, part_fp=32, lb_fp=64, alpha_deg=120.0)


def thin_film_3d() -> dict:
    """Thin film: D3Q19 512x256x256 FP32 populations, tau 0.7, film
    y in [126,130) with 1-row buffers, r = 4, 10 particles/cell (335,544,320)."""
    return make(dim=3, n=(512, 256, 256), tau=0.7, ylo=126, yhi=130, buf_lo=1, buf_hi=1,
                ppc=10, part_fp=32, lb_fp=32, alpha_deg=120.0)


def channel_3d_scaled(fx: int = 1, fz: int = 1, ppc: int | None = None, **kw) -> dict:
    """The 3D channel with x and z cut by fx and fz (same per-node and
    per-particle work), used for bounded CPU timings and sampled parity."""
    p = channel_3d()
    n = (p["n"][0] // fx, p["n"][1], p["n"][2] // fz)
    q = make(**{**p, "n": n, **({"ppc": ppc} if ppc else {}), **kw})
    return q


# ---- the paper's coupled runs (Sec. 3, Table 1) ---------------------------------

def paper_centreline(N: int = 1000, **kw) -> dict:
    """The centre-line coupling of Sec. 3.2 (Table 1, second row): D2Q9 30x30,
    tau 1 (nu 1/6), g 5e-4, walls at y = 0 and 30; MPCD with Andersen
    thermostat on the lower half y in [0, 15), cell side a = 1, one MPCD step
    per LB step, kT 0.17, N particles per cell (60 to 1000 in the paper), a
    two-row buffer under the centre line.  Started from the exact Poiseuille
    profile."""
    base = dict(dim=2, n=(30, 30, 1), tau=1.0, g=(5e-4, 0.0, 0.0), walls_y=1, ylo=0, yhi=15, buf_lo=0, buf_hi=2,
                refine=1, substeps=1, ppc=N, kT=0.17, collision=1, feedback=0, init_flow=1, part_fp=64)
    base.update(kw)
    return make(**base)


def paper_near_wall(a: float = 1.0, **kw) -> dict:
    """The near-wall coupling of Sec. 3.3 (Table 1, third row): an MPCD slab on
    the bottom wall meets the LB through a two-row buffer, N = 1000 particles
    per cell, MPCD with Andersen thermostat, one MPCD step per LB step, g 5e-4,
    tau 1.  a = 1: LB 40x60, MPCD 40x14 cells, kT 0.17; a = 1/2: LB 20x30,
    MPCD 40x14 cells of side 1/2 (7 LB rows; the paper quotes 39x13), kT 0.3.
    Started from the exact Poiseuille profile."""
    if a == 1.0:
        base = dict(n=(40, 60, 1), yhi=14, refine=1, kT=0.17)
    elif a == 0.5:
        base = dict(n=(20, 30, 1), yhi=7, refine=2, kT=0.3)
    else:
        raise ValueError("the paper runs a = 1 and a = 1/2")
    base.update(dict(dim=2, tau=1.0, g=(5e-4, 0.0, 0.0), walls_y=1, ylo=0, buf_lo=0, buf_hi=2, substeps=1,
                     ppc=1000, collision=1, feedback=0, init_flow=1, part_fp=64))
    base.update(kw)
    return make(**base)


# ---- small cases for parity (the oracle finishes them in seconds) -------------

def small_2d(**kw) -> dict:
    """2D coupled channel, 40x24 nodes, slab [8,16), r 4, 6 ppc: 23,040 particles,
    several particle tiles and a ragged tail in x."""
    base = dict(n=(40, 24, 1), ylo=8, yhi=16, buf_lo=2, buf_hi=2, ppc=6)
    base.update(kw)
    return make(**base)


def small_3d(**kw) -> dict:
    """3D coupled channel, 12x16x10 nodes, slab [6,11), r 2, 5 ppc."""
    base = dict(dim=3, n=(12, 16, 10), tau=0.8, ylo=6, yhi=11, buf_lo=1, buf_hi=1,
                refine=2, ppc=5, alpha_deg=120.0)
    base.update(kw)
    return make(**base)


def walled_2d(**kw) -> dict:
    """Stand-alone MPCD Poiseuille channel: the slab is the whole channel, both
    faces are walls (bounce-back + virtual particles), no buffers."""
    base = dict(n=(16, 8, 1), ylo=0, buf_lo=0, buf_hi=0, refine=2, ppc=8, feedback=0)
    base.update(kw)
    base.setdefault("yhi", base["n"][1])
    return make(**base)


def periodic_2d(**kw) -> dict:
    """Fully periodic box (no walls, no buffers): equilibrium checks."""
    base = dict(n=(16, 16, 1), walls_y=0, ylo=0, buf_lo=0, buf_hi=0, refine=2,
                ppc=8, g=(0.0, 0.0, 0.0), feedback=0)
    base.update(kw)
    base.setdefault("yhi", base["n"][1])
    return make(**base)


# ---- derived sizes (pure bookkeeping) -----------------------------------------

def sizes(p: dict) -> dict:
    nx, ny, nz = p["n"]
    nodes = nx * ny * nz
    out = dict(nodes=nodes, Q=9 if p["dim"] == 2 else 19)
    if p["mpcd"]:
        r = p["refine"]
        R = (p["yhi"] - p["ylo"]) * r
        Cx = nx * r
        Cz = nz * r if p["dim"] == 3 else 1
        ywrap = (not p["walls_y"] and p["ylo"] == 0 and p["yhi"] == ny
                 and p["buf_lo"] == 0 and p["buf_hi"] == 0)
        CyB = R if ywrap else R + 1
        out.update(R=R, Cx=Cx, Cz=Cz, CyB=CyB, ncells=Cx * CyB * Cz,
                   particles=Cx * R * Cz * p["ppc"])
    else:
        out.update(particles=0)
    return out


def algorithmic_bytes_per_lb_step(p: dict) -> dict:
    """Bytes the method must move per LB step: one read and one write of the Q
    populations per node, and of each particle's position and velocity per
    MPCD step."""
    s = sizes(p)
    lbw = 8 if p["lb_fp"] == 64 else 4
    pw = 8 if p["part_fp"] == 64 else 4
    lb = 2 * s["Q"] * lbw * s["nodes"]
    part = 2 * 2 * p["dim"] * pw * s["particles"] * p["substeps"]
    return dict(lb=lb, mpcd=part, total=lb + part,
                per_node=2 * s["Q"] * lbw, per_particle_update=2 * 2 * p["dim"] * pw)


def closure_target(**kw) -> dict:
    """Channel the learned closure stands in for the MPCD slab of: D3Q19
    256x128x128 FP32 populations, walls at y = 0 and 128, slab of 16 rows
    y in [56, 72) with 1-row buffers, r 4, 10 particles per cell
    (335,544,320 FP32 particles), one-way coupling, exact Poiseuille start."""
    base = dict(dim=3, n=(256, 128, 128), tau=0.8, g=(1e-6, 0.0, 0.0), ylo=56, yhi=72, buf_lo=1, buf_hi=1,
                ppc=10, part_fp=32, lb_fp=32, alpha_deg=120.0, feedback=0, init_flow=1, closure=1)
    base.update(kw)
    return make(**base)


def closure_training_sections(n: int = 8, seed: int = 1) -> list[dict]:
    """Training channels for the closure of the target channel: sections of
    it 32 nodes long and 32 wide (same walls at y = 0 and 128, same slab
    y in [56, 72) with 1-row buffers, r 4, 10 particles per cell, one-way
    coupling, exact Poiseuille start, binary32 populations like the target),
    with body force log-uniform in [5e-7, 2e-6] and tau uniform in
    [0.7, 0.9], so that the target's g = 1e-6, tau = 0.8 lies inside the
    sampled range (centre-line velocities 0.008 to 0.06 against the
    target's 0.02).  The precision matters: the wall-normal velocity of this
    flow is zero up to rounding, so its feature columns are scaled by the
    rounding of the populations they were collected with, and binary64
    training data would read binary32 rounding as thousands of standard
    deviations."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        g = float(10.0 ** rng.uniform(np.log10(5e-7), np.log10(2e-6)))
        tau = float(rng.uniform(0.7, 0.9))
        out.append(make(dim=3, n=(32, 128, 32), tau=tau, g=(g, 0.0, 0.0), ylo=56, yhi=72, buf_lo=1, buf_hi=1,
                        ppc=10, part_fp=32, lb_fp=32, alpha_deg=120.0, feedback=0, init_flow=1, closure=1,
                        instance=i))
    return out


def ensemble(n_inst: int = 256, seed: int = 1) -> list[dict]:
    """Batched ensemble of independent 2D channels of uneven sizes: width
    W ~ U{16..128}, length L ~ U{32..256}, particles per cell U{5..20}; the
    slab is a centred strip of round(W/4) rows with 1-row buffers; every
    channel starts from the exact discrete Poiseuille profile (a 128-row
    channel would need some 10^5 LB steps to develop from rest)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_inst):
        W = int(rng.integers(16, 129))
        L = int(rng.integers(32, 257))
        ppc = int(rng.integers(5, 21))
        strip = max(4, int(round(W / 4)))
        ylo = (W - strip) // 2
        out.append(make(n=(L, W, 1), ylo=ylo, yhi=ylo + strip, buf_lo=1, buf_hi=1,
                        ppc=ppc, seed=seed, instance=i, init_flow=1))
    return out
