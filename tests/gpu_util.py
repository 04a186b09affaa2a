"""Helpers of the GPU parity tests: run a parameter set on the HIP path and on
the oracle and compare what both define uniquely."""
import sys

import numpy as np

RTOL64 = 1e-11   # FP64 path vs FP64 oracle, relative to each field's scale
RTOL32 = 2e-6    # binary32 stores vs the oracle's binary32 emulation


def banner(msg: str):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def scaled_err(a, b, scale=None):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if scale is None:
        scale = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / scale) if a.size else 0.0


def periodic_err(a, b, L):
    """Largest minimum-image distance between position arrays [d][n]."""
    d = np.abs(np.asarray(a) - np.asarray(b))
    out = 0.0
    for k in range(d.shape[0]):
        dk = d[k]
        if L[k] is not None:
            dk = np.minimum(dk, L[k] - dk)
        out = max(out, float(dk.max()) if dk.size else 0.0)
    return out


def compare_state(sim, orc, p, rtol, inst=0, check_cells=True, binning=None):
    """Element-wise comparison of every field both sides define.  `binning`
    is the HIP path's binning when it was read before (cell velocities exist
    only until the particles are read).

    Scales: each field's own magnitude; with binary32 populations the fields
    derived from them (u, Pi, the buffer velocities, the feedback's running
    mean) are compared in lattice units (at least rho0 c = 1), because the
    binary32 store bounds their error absolutely: Q populations of about
    rho/Q each, rounded to 2^-24 relative, give at most Q 2^-24 rho ~ 1.1e-6
    (D3Q19) in u, however small u is."""
    rep = {}
    floor = 1.0 if p.get("lb_fp", 64) == 32 else 1e-12
    f_g = sim.f(inst)
    f_o = orc.f()
    rep["pop"] = scaled_err(f_g, f_o)
    rho_g, u_g, pi_g = sim.fields(inst)
    rho_o, u_o, pi_o = orc.moments()
    rep["rho"] = scaled_err(rho_g, rho_o)
    uscale = max(np.abs(u_o).max(), floor)
    rep["u"] = scaled_err(u_g, u_o, uscale)
    rep["pi"] = scaled_err(pi_g, pi_o, max(np.abs(pi_o).max(), floor if floor > 1e-12 else 1e-300))
    if p["mpcd"]:
        vcm_g = None
        if check_cells:
            b_g = binning if binning is not None else sim.binning(inst)
            b_o = orc.binning()
            rep["cell_mismatch"] = int((b_g["cell"] != b_o["cell"]).sum())
            rep["count_mismatch"] = int((b_g["count"] != b_o["count"]).sum())
            occ = b_o["count"] > 0
            vscale = np.sqrt(p["kT"] / p["mass"])
            rep["vcm"] = scaled_err(b_g["vcm"][:, occ], b_o["vcm"][:, occ], vscale)
            vcm_g = b_g
        pos_g, vel_g = sim.particles(inst)
        pos_o, vel_o = orc.particles()
        nx, ny, nz = p["n"]
        L = [nx, None, nz][: p["dim"]]
        if not p["walls_y"] and p["ylo"] == 0 and p["yhi"] == ny:
            L[1] = ny
        rep["pos"] = periodic_err(pos_g, pos_o, L) / max(nx, ny)
        rep["vel"] = scaled_err(vel_g, vel_o, np.sqrt(p["kT"] / p["mass"]))
        if p["buf_lo"] + p["buf_hi"] > 0:
            uf_g = sim.ufine(inst)
            uf_o = orc.ufine()
            rep["ufine"] = scaled_err(uf_g, uf_o, max(np.abs(uf_o).max(), floor))
            if p.get("reinject", 0):
                tf_g = sim.tfine(inst)
                tf_o = orc.tfine()
                rep["tfine"] = scaled_err(tf_g, tf_o, max(np.abs(tf_o).max(), 1e-12))
        if p["feedback"] and hasattr(orc, "fb_u"):
            fb_g = sim.node_fb_u(inst)
            fb_o = orc.fb_u()[: p["dim"]]
            rep["fb_u"] = scaled_err(fb_g, fb_o, max(np.abs(fb_o).max(), floor))
        st = sim.stats(inst)
        rep["dropped"] = st["dropped"]
        rep["misplaced"] = st["misplaced"]
        rep["bad_state"] = st["bad_state"]
        del vcm_g
    return rep


def assert_parity(rep, rtol):
    bad = []
    for k, v in rep.items():
        if k in ("cell_mismatch", "count_mismatch", "dropped", "misplaced", "bad_state"):
            if v != 0:
                bad.append((k, v))
        elif v > rtol:
            bad.append((k, v))
    assert not bad, f"parity failures {bad} in {rep}"
