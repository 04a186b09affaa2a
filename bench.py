#!/usr/bin/env python3
"""Throughput of the coupled LB-MPCD time step on one MI355X.

Default workload: the thin film -- D3Q19 512x256x256 nodes with binary32
populations (tau 0.7, g 1e-6 along x, walls at y = 0 and 256, periodic x and
z) coupled to an MPCD film y in [126, 130) with 1-row buffers, cell side 1/4
(2048x16x1024 cells), 10 particles per cell (335,544,320 binary32 particles,
FP64 cell sums), SRD 120 deg about a random axis, 4 MPCD steps per LB step,
random grid shift, feedback on (window 50 LB steps).  The largest of the
single-GPU configurations.  Synthetic, seeded: positions uniform in cells,
Maxwell-Boltzmann velocities.

One "step" is one coupled LB step (LB collide-stream, feedback projection,
interpolation to the buffer cells, 4 fused MPCD steps).  Prints one JSON line:
the contract's fields; `roofline` for the fused particle kernel (algorithmic
bytes per launch over its HIP-event time, against 8 TB/s; `traffic` from the
committed rocprofv3 PMC summary of the workload while the sources of the
step's kernels are unchanged); `lb_roofline` for the LB collide-stream kernel;
`coupled_hbm_frac` (algorithmic) and `coupled_counter_frac` (counter-measured)
for the whole step; the timed steps in five chunks; the sample-window misses;
and `cpu_baseline`, the oracle timed on the host cores (one process per core,
up to 16) on a cut of the workload, taken before the GPU is touched.
Other workloads: --workload channel_3d | channel_3d_at | channel_3d_ce |
channel_2d | ensemble | closure.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
# every source the coupled step's kernels are compiled from, and the flags
KERNEL_SOURCES = ["paper_2004_00304_amd/csrc/particles.hpp", "paper_2004_00304_amd/csrc/kernels_mpcd.hip",
                  "paper_2004_00304_amd/csrc/kernels_mpcd_ce.hip", "paper_2004_00304_amd/csrc/common.hpp",
                  "paper_2004_00304_amd/csrc/fmath.hpp", "paper_2004_00304_amd/csrc/launch.hpp",
                  "paper_2004_00304_amd/csrc/kernels_lb.hip", "paper_2004_00304_amd/build.py"]
MAX_CPU_WORKERS = 16  # host cores the CPU baseline may use (the GPU machine's share)


def pmc_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"k_particles_{workload}_pmc.json")


def kernel_hash() -> str:
    """Hash of the sources the particle and LB kernels are built from.  In the
    C++ sources comments and white space are dropped first (none of them holds
    a comment marker inside a string), so that an edit of comments alone keeps
    the committed counter summaries valid; build.py, which holds the compiler
    flags, enters as it is."""
    import re
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        with open(os.path.join(ROOT, s), "rb") as f:
            text = f.read()
        if not s.endswith(".py"):
            t = text.decode()
            t = re.sub(r"/\*.*?\*/", " ", t, flags=re.S)
            t = re.sub(r"//[^\n]*", " ", t)
            text = " ".join(t.split()).encode()
        h.update(text)
    return h.hexdigest()[:16]


def workload_params(name: str) -> list:
    """Parameter dicts of the named workload (one per channel)."""
    from paper_2004_00304_amd import workloads as W
    if name == "ensemble":
        return W.ensemble(256)
    if name == "channel_3d_at":
        return [W.make(**{**W.channel_3d(), "collision": 1})]
    if name == "channel_3d_ce":
        return [W.make(**{**W.channel_3d(), "reinject": 1})]
    return [{"channel_3d": W.channel_3d, "channel_2d": W.channel_2d, "thin_film_3d": W.thin_film_3d}[name]()]


def totals(plist: list) -> dict:
    """Summed sizes and algorithmic bytes of a list of channels."""
    from paper_2004_00304_amd import workloads as W
    out = dict(nodes=0, particles=0, lb_bytes=0, mpcd_bytes=0, launch_bytes=0)
    for p in plist:
        sz, ab = W.sizes(p), W.algorithmic_bytes_per_lb_step(p)
        out["nodes"] += sz["nodes"]
        out["particles"] += sz["particles"]
        out["lb_bytes"] += ab["lb"]
        out["mpcd_bytes"] += ab["mpcd"]
        out["launch_bytes"] += ab["per_particle_update"] * sz["particles"]
    out["total_bytes"] = out["lb_bytes"] + out["mpcd_bytes"]
    return out


def _pmc(workload: str):
    """The committed rocprofv3 PMC summary of the workload (FETCH_SIZE,
    WRITE_SIZE scaled by a plain copy of known size), or None when it is
    absent or a source of the step's kernels changed since it was taken."""
    path = pmc_file(workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        pmc = json.load(f)
    if pmc.get("kernel_hash") != kernel_hash():
        return None
    return pmc


def measured_traffic(workload: str):
    """HBM bytes per launch of the particle kernel from the PMC summary."""
    pmc = _pmc(workload)
    return pmc.get("bytes_per_launch") if pmc else None


def measured_step_traffic(workload: str):
    """HBM bytes per coupled LB step (all its kernels) from the PMC summary."""
    pmc = _pmc(workload)
    return pmc.get("step_bytes_per_lb_step") if pmc else None


def _cut(p: dict) -> dict:
    """The bounded CPU sample of a workload: x and z cut (same per-node and
    per-particle work) by 8, or by 16 for the 512-node-long thin film."""
    from paper_2004_00304_amd import workloads as W
    if p["dim"] == 2:
        return W.make(**{**p, "n": (max(p["n"][0] // 8, 8), p["n"][1], 1)})
    f = 16 if p["n"][0] >= 512 else 8
    return W.make(**{**p, "n": (p["n"][0] // f, p["n"][1], p["n"][2] // f)})


def cpu_worker(workload: str, seconds: float, index: int, stride: int) -> None:
    """One CPU-baseline process: the oracle, single-threaded, on the cut of
    the workload (the ensemble: channels index, index + stride, ... one LB
    step each) until `seconds` have passed; prints its counts as JSON."""
    from oracle import oracle as O
    from paper_2004_00304_amd import workloads as W
    plist = workload_params(workload)
    particles = nodes = steps = 0
    t0 = time.perf_counter()
    if len(plist) > 1:
        k = index
        while time.perf_counter() - t0 < seconds and k < len(plist):
            O.Oracle(plist[k]).step(1)
            sz = W.sizes(plist[k])
            particles += sz["particles"]
            nodes += sz["nodes"]
            steps += 1
            k += stride
    else:
        q = _cut(plist[0])
        o = O.Oracle(q)
        sz = W.sizes(q)
        while True:
            o.step(1)
            steps += 1
            particles += sz["particles"]
            nodes += sz["nodes"]
            if time.perf_counter() - t0 > seconds or steps >= 200:
                break
    print(json.dumps(dict(steps=steps, particles=particles, nodes=nodes, dt=time.perf_counter() - t0)), flush=True)


def host_description() -> dict:
    """The host's CPU from lscpu (model, counts) and the cores this process may use."""
    import subprocess
    out = {"usable_cpus": len(os.sched_getaffinity(0))}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket", "Socket(s)",
                             "CPU max MHz"):
                out[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        out["lscpu"] = "unavailable"
    return out


def cpu_baseline(workload: str, seconds: float = 12.0) -> dict:
    """The oracle, as it stands, on a bounded sample of the workload: first
    one process (one core), then one process per usable core (at most 16)
    side by side; coupled LB steps/s of the whole workload scaled from the
    sample by the particle ratio.  Run before the GPU is initialised (the
    workers are child processes)."""
    import subprocess
    from oracle import oracle as O
    from paper_2004_00304_amd import workloads as W
    if not os.path.exists(O.LIB_PATH):
        O.build()
    plist = workload_params(workload)
    total_particles = sum(W.sizes(p)["particles"] for p in plist)
    substeps = plist[0]["substeps"]

    def run(nproc):
        procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", workload,
                                   str(seconds), str(i), str(nproc)], stdout=subprocess.PIPE, text=True)
                 for i in range(nproc)]
        res = [json.loads(pr.communicate()[0].strip().splitlines()[-1]) for pr in procs]
        rate = sum(r["particles"] / r["dt"] for r in res)  # particle-LB-steps per second
        lb = sum(r["nodes"] / r["dt"] for r in res)
        return rate, lb, res

    r1, lb1, res1 = run(1)
    nproc = max(1, min(len(os.sched_getaffinity(0)), MAX_CPU_WORKERS))
    rn, lbn, resn = run(nproc) if nproc > 1 else (r1, lb1, res1)
    if len(plist) > 1:
        sample = (f"one LB step of each of the first channels of the ensemble in turn, {seconds:.0f} s per "
                  f"process ({res1[0]['steps']} channels on one core; {sum(r['steps'] for r in resn)} on "
                  f"{nproc} cores), scaled by the particle ratio")
    else:
        q = _cut(plist[0])
        sample = (f"{q['n'][0]}x{q['n'][1]}x{q['n'][2]} nodes, {W.sizes(q)['particles']} particles (x and z "
                  f"cut like the workload's), {res1[0]['steps']} LB steps in {res1[0]['dt']:.1f} s on one core; "
                  f"{nproc} such processes side by side, {sum(r['steps'] for r in resn)} LB steps; scaled by "
                  f"the particle ratio {W.sizes(q)['particles'] / total_particles:.5f}")
    return dict(value=rn / total_particles, unit="coupled LB steps/s", cores=nproc, kind="oracle", sample=sample,
                one_core_value=r1 / total_particles,
                particle_updates_per_s=rn * substeps, particle_updates_per_s_one_core=r1 * substeps,
                lb_mlups=lbn / 1e6, lb_mlups_one_core=lb1 / 1e6, host=host_description())


def instance_profiles(sim, plist: list, steps: int, path: str | None) -> dict:
    """Time-averaged profiles of every channel of a batched context, after
    the timed region: `steps` sampled LB steps, then per channel the MPCD
    streamwise velocity of each interior slab row (the fine rows of an LB row
    pooled), the LB velocity of the same rows (mean over x) and the one-way
    Poiseuille parabola g y (H - y) / (2 nu) at the rows' centres.  The line
    carries the relative L2 difference of the MPCD profile from each, per
    channel (median, 90th percentile, largest); `path`, when given, receives
    every profile.  Narrow channels are dominated by thermal noise (a 16-row
    channel at g = 1e-6 peaks at 2e-4); the widest carries the flow."""
    import numpy as np
    sim.sample(1)
    sim.step(steps)
    sim.sync()
    devs, devp, rows = [], [], []
    for i, p in enumerate(plist):
        r, nsy = p["refine"], p["yhi"] - p["ylo"]
        prof = np.asarray(sim.profile(i)).reshape(nsy, r, 4).sum(axis=1)
        ys = range(p["buf_lo"], nsy - p["buf_hi"])
        u_m = np.array([prof[y, 1] / prof[y, 0] for y in ys])
        _, u, _ = sim.fields(i)
        u_lb = np.array([u[0, 0, p["ylo"] + y, :].mean() for y in ys])
        nu = (p["tau"] - 0.5) / 3.0
        yc = np.array([p["ylo"] + y + 0.5 for y in ys])
        u_par = p["g"][0] * yc * (p["n"][1] - yc) / (2.0 * nu)
        devs.append(float(np.linalg.norm(u_m - u_lb) / np.linalg.norm(u_lb)))
        devp.append(float(np.linalg.norm(u_m - u_par) / np.linalg.norm(u_par)))
        rows.append({"channel": i, "n": list(p["n"][:2]), "slab": [p["ylo"], p["yhi"]],
                     "mpcd_u": [round(float(x), 8) for x in u_m], "lb_u": [round(float(x), 8) for x in u_lb],
                     "parabola_u": [round(float(x), 8) for x in u_par]})
    sim.sample(0)
    if path:
        with open(path, "w") as fo:
            json.dump({"sampled_lb_steps": steps, "channels": rows}, fo)
    def summary(v):
        d = sorted(v)
        return {"median": d[len(d) // 2], "p90": d[int(0.9 * (len(d) - 1))], "max": d[-1]}
    return {"sampled_lb_steps": steps, "channels": len(plist),
            "rel_l2_mpcd_vs_lb": summary(devs), "rel_l2_mpcd_vs_parabola": summary(devp),
            "widest_channel": rows[int(np.argmax([q["n"][1] for q in plist]))], "file": path}


def one_by_one(lbmpcd, plist: list, batched_ms: float, sample: int = 16, steps: int = 8) -> dict:
    """The same channels advanced one context at a time (each alone on the
    GPU), for every len(plist)/sample-th channel; the summed time per coupled
    step is scaled to all channels and compared with the batched step."""
    import torch
    idx = list(range(0, len(plist), max(1, len(plist) // sample)))[:sample]
    total_ms = 0.0
    for i in idx:
        sim = lbmpcd.Sim(plist[i], device="cuda:0")
        sim.step(4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        total_ms += 1e3 * (time.perf_counter() - t0) / steps
        sim.close()
    est = total_ms * len(plist) / len(idx)
    return dict(channels_measured=len(idx), one_by_one_ms_per_step=est, batched_ms_per_step=batched_ms,
                speedup=est / batched_ms)


def closure_bench(lbmpcd, W, args):
    """The learned closure against the plain coupled step on the same channel
    (256x128x128 D3Q19, 16-row slab, 335.5M particles, one-way coupling).

    Training data come from eight 32x128x32 sections of the same channel
    (g log-uniform in [5e-7, 2e-6], tau in [0.7, 0.9], the target's 1e-6 and
    0.8 inside): per section 4 windows of 400 LB steps after 200 steps of
    warm-up, 524k samples, in consecutive pairs of windows
    so that the targets' noise can be measured (half the mean square
    difference of the two windows of a node, in the standardised units of the
    loss: the loss of a perfect predictor of the mean).  Training runs on the
    GPU with the library's kernels.  On the target channel, after 500 warm-up
    steps, the time-averaged profile of 100 plain steps is compared with the
    surrogate's (400 sampled steps each) and with the LB velocity itself
    (the network-free prediction); then plain and surrogate steps are timed, and surrogate steps
    with the periodic plain-MPCD check on."""
    import numpy as np
    import torch
    UC = 13 * 10 + 1  # the node's own LB velocity among the features
    t0 = time.perf_counter()
    X, Y = [], []
    for i, q in enumerate(W.closure_training_sections(8)):
        s = lbmpcd.Sim(q)
        s.step(200)
        for _ in range(4):
            x, y = s.closure_collect(400)
            X.append(x)
            Y.append(y)
        s.close()
        print(f"[closure] section {i}: g {q['g'][0]:.3g} tau {q['tau']:.3f} collected "
              f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    # noise of the targets from the pairs of consecutive windows
    Yr = [y.clone() for y in Y]
    for x, y in zip(X, Yr):
        y[:, :3] -= x[:, UC:UC + 3]
    allr = torch.cat(Yr).double()
    var = allr.var(dim=0)
    dsq = torch.stack([((Yr[i] - Yr[i + 1]).double() ** 2).mean(dim=0) for i in range(0, len(Yr), 2)]).mean(dim=0)
    floor_k = (0.5 * dsq / var).clamp(max=1.0)
    X = torch.cat(X)
    Y = torch.cat(Y)
    n_samples = X.shape[0]
    t_data = time.perf_counter() - t0
    trainer = lbmpcd.Sim(W.closure_training_sections(1)[0])
    t0 = time.perf_counter()
    first = trainer.closure_train(X, Y, epochs=1, batch=4096, lr=1e-30, seed=7)
    losses = list(trainer.closure_train(X, Y, epochs=30, batch=4096, lr=1e-3))
    print(f"[closure] 30 epochs at lr 1e-3 done ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    losses += list(trainer.closure_train(X, Y, epochs=20, batch=4096, lr=1e-4))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    block = trainer.closure_weights()
    trainer.close()
    del X, Y, Yr, allr
    torch.cuda.empty_cache()

    p = W.closure_target()
    sz = W.sizes(p)
    r, nsy = p["refine"], p["yhi"] - p["ylo"]
    rows = range(p["buf_lo"], nsy - p["buf_hi"])

    def profile_rows(sim):
        prof = np.asarray(sim.profile()).reshape(nsy, r, 4).sum(axis=1)
        return np.array([prof[y, 1] / prof[y, 0] for y in rows])

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    sim = lbmpcd.Sim(p, device="cuda:0")
    sim.step(500)
    sim.sample(1)
    sim.step(400)
    u_plain = profile_rows(sim)
    _, u, _ = sim.fields()
    u_lb = np.array([u[0, :, p["ylo"] + y, :].mean() for y in rows])
    sim.sample(0)

    def timed(n):
        torch.cuda.synchronize()
        t = time.perf_counter()
        sim.step(n)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / n

    sim.step(args.warmup)
    plain = timed(args.steps)
    sim.closure_weights(block)
    sim.closure_enable(True, tol=0.02, check_every=0)
    sim.sample(1)
    sim.step(400)
    u_sur = profile_rows(sim)
    sim.sample(0)
    sim.step(args.warmup)
    sim.timing(1)
    sur = timed(args.steps)
    sim.timing(0)
    kt = sim.timing_read()
    cl_ms = kt["closure"]["ms"] / max(1, kt["closure"]["launches"])
    # the surrogate with its periodic check: 40 plain steps every 400
    check_every, check_steps = 400, 40
    sim.closure_enable(True, tol=0.02, check_every=check_every, check_steps=check_steps)
    with_check = timed(2 * check_every)
    st = sim.closure_status()
    # network flops of one inference over every slab node (271 real inputs)
    nslab = p["n"][0] * (p["yhi"] - p["ylo"]) * p["n"][2]
    flops = 2.0 * nslab * (271 * 128 + 128 * 128 * 2 + 128 * 9)
    out = {
        "metric": "coupled steps/s: LB MLUPS + MPCD particle-updates/s, % HBM roofline",
        "value": 1.0 / sur, "unit": "coupled LB steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * sur, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 network (fp32 accumulate) / f32 LB",
        "data": "synthetic (seeded Poiseuille channels; training data from the coupled method itself)",
        "config": {"workload": (f"closure: D3Q19 {p['n'][0]}x{p['n'][1]}x{p['n'][2]} FP32, slab "
                                f"y[{p['ylo']},{p['yhi']}), {sz['particles']} particles replaced by the MLP "
                                f"271-128-128-128-9"), "lb_nodes": sz["nodes"], "particles": sz["particles"]},
        "plain_steps_per_s": 1.0 / plain, "plain_ms_per_step": 1e3 * plain,
        "surrogate_speedup": plain / sur,
        "profile_rel_err": rel(u_sur, u_plain),
        "profile_rel_err_lb_velocity_alone": rel(u_lb, u_plain),
        "profiles": {"plain": [round(float(x), 7) for x in u_plain], "surrogate": [round(float(x), 7) for x in u_sur],
                     "lb": [round(float(x), 7) for x in u_lb]},
        "with_check": {"check_every": check_every, "check_steps": check_steps, "ms_per_step": 1e3 * with_check,
                       "speedup": plain / with_check, "last_check_err": st["last_err"],
                       "fell_back": st["fell_back"]},
        "kernels_ms_per_launch": {k: v["ms"] / max(1, v["launches"]) for k, v in kt.items()},
        "roofline": {"bound": "mfma", "kernel": "closure inference (band moments + fused features/MLP)",
                     "achieved": flops / (cl_ms * 1e-3) / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": flops / (cl_ms * 1e-3) / 1e12 / 2500.0, "traffic": None,
                     "algorithmic_flops_per_launch": flops},
        "lb_mlups": sz["nodes"] / sur / 1e6,
        "training": {"samples": int(n_samples), "data_s": t_data, "train_s": t_train,
                     "initial_loss": float(first[0]), "epoch_loss": [float(x) for x in losses],
                     "loss_floor": float(floor_k.mean()),
                     "loss_floor_per_output": [round(float(x), 4) for x in floor_k],
                     # share of the reducible loss (initial loss less the noise floor)
                     # that training removed
                     "learned_fraction": float((first[0] - losses[-1]) / max(first[0] - floor_k.mean(), 1e-12))},
    }
    print(json.dumps(out), flush=True)


def calib_copy():
    """Plain device copy of known size, for scaling the PMC byte counters."""
    import torch
    n = 1 << 30
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": n}), flush=True)


def pmc_summary(workload: str, fetch_csv: str, write_csv: str, command: str) -> None:
    """Writes the committed PMC summary of the workload's particle kernel
    from two rocprofv3 --pmc runs of `bench.py --calib-copy` (FETCH_SIZE,
    WRITE_SIZE; KiB per dispatch).  Each counter is scaled by what it reads
    for the plain 1 GiB device copy in the same run; the same scales applied
    to k_lb_step, whose bytes are known exactly, check the calibration."""
    import csv
    from paper_2004_00304_amd import workloads as W

    def per_kernel(path, counter):
        out = {}
        for row in csv.DictReader(open(path)):
            if row["Counter_Name"] != counter:
                continue
            out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
        return out

    f = per_kernel(fetch_csv, "FETCH_SIZE")
    w = per_kernel(write_csv, "WRITE_SIZE")
    copy_f = [v for k, vs in f.items() if "copy" in k.lower() or "elementwise" in k.lower() for v in vs]
    copy_w = [v for k, vs in w.items() if "copy" in k.lower() or "elementwise" in k.lower() for v in vs]
    gib_kib = float(1 << 20)
    fscale = gib_kib / max(copy_f)  # the copy reads 1 GiB
    wscale = gib_kib / max(copy_w)  # and writes 1 GiB
    # the particle kernel of the fused step (mode 3), not its overflow pass
    is_fused = lambda k: "k_particles<" in k and ", 3>" in k
    fused = lambda d: [v for k, vs in d.items() if is_fused(k) for v in vs]
    pf, pw = fused(f), fused(w)
    names = sorted({k.split("(")[0].replace("void ", "").replace("lbmpcd::", "") for k in f if is_fused(k)})
    fetch_b = sum(pf) / len(pf) * 1024 * fscale
    write_b = sum(pw) / len(pw) * 1024 * wscale

    # the coupled step: S particle launches plus one LB step, band and
    # interpolation launch (the particle kernel's figures above, the others'
    # averages over their dispatches)
    def mean_bytes(tag):
        fk = [v for k, vs in f.items() if tag in k for v in vs]
        wk = [v for k, vs in w.items() if tag in k for v in vs]
        return (sum(fk) / len(fk) * fscale + sum(wk) / len(wk) * wscale) * 1024 if fk and wk else 0.0
    other = {t: mean_bytes(t) for t in ("k_lb_step", "k_band", "k_interp")}
    plist = workload_params(workload)
    p = plist[0]
    # the overflow pass after every particle launch of a two-pass step
    # (almost always an empty list)
    other["k_particles_ovf"] = p["substeps"] * mean_bytes("k_particles_ovf")
    alg = totals(plist)["launch_bytes"]
    lb_alg = totals(plist)["lb_bytes"]
    # a check of the copy calibration on another kernel: k_lb_step reads and
    # writes each population once, half of its algorithmic bytes each way
    lbf = [v for k, vs in f.items() if "k_lb_step" in k for v in vs]
    lbw = [v for k, vs in w.items() if "k_lb_step" in k for v in vs]
    lb_check = ({"fetch_over_algorithmic": sum(lbf) / len(lbf) * 1024 * fscale / (lb_alg / 2),
                 "write_over_algorithmic": sum(lbw) / len(lbw) * 1024 * wscale / (lb_alg / 2)}
                if lbf and lbw else None)
    out = {
        "kernel": f"{', '.join(names)} (fused MPCD step), {workload}",
        "kernel_hash": kernel_hash(),
        "command": command,
        "dispatches": len(pf),
        "fetch_kib_per_dispatch": sum(pf) / len(pf),
        "write_kib_per_dispatch": sum(pw) / len(pw),
        "copy_fetch_kib": max(copy_f), "copy_write_kib": max(copy_w),
        "fetch_scale": fscale, "write_scale": wscale,
        "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
        "bytes_per_launch": fetch_b + write_b,
        "algorithmic_bytes_per_launch": alg,
        "traffic_over_algorithmic": (fetch_b + write_b) / alg,
        "other_kernels_bytes_per_lb_step": other,
        "lb_step_algorithmic_bytes": lb_alg,
        "calibration_check_k_lb_step": lb_check,
        "step_bytes_per_lb_step": p["substeps"] * (fetch_b + write_b) + sum(other.values()),
    }
    with open(pmc_file(workload), "w") as fo:
        json.dump(out, fo, indent=1)
    print(json.dumps(out, indent=1))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="thin_film_3d",
                    choices=["channel_3d", "channel_3d_at", "channel_3d_ce", "channel_2d", "thin_film_3d",
                             "ensemble", "closure"])
    ap.add_argument("--autotune", action="store_true",
                    help="pick the launch shape with lbmpcd_autotune first (always on for the ensemble)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default launch shape for the ensemble too")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=1000,
                    help="batched workloads: LB steps sampled after the timed region for per-channel profiles")
    ap.add_argument("--profiles-out", default=None, help="batched workloads: file for every channel's profile")
    ap.add_argument("--calib-copy", action="store_true")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "COMMAND"),
                    help="write the workload's particle-kernel PMC summary from two rocprofv3 runs and exit")
    ap.add_argument("--cpu-worker", nargs=4, metavar=("WORKLOAD", "SECONDS", "INDEX", "STRIDE"),
                    help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        w, sec, i, st = args.cpu_worker
        cpu_worker(w, float(sec), int(i), int(st))
        return
    if args.pmc_summary:
        pmc_summary(args.workload, *args.pmc_summary)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the multi-GPU "
              "sharding of the coupled step is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2004_00304_amd import lbmpcd
    from paper_2004_00304_amd import workloads as W

    if args.workload == "closure":
        closure_bench(lbmpcd, W, args)
        return
    # the CPU baseline first: its worker processes start before this one
    # touches the GPU, and nothing else loads the host while the GPU is timed
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.workload)
    if args.calib_copy:
        calib_copy()
    plist = workload_params(args.workload)
    p = plist[0]
    tot = totals(plist)
    torch.cuda.set_device(0)
    tuning = None
    if args.autotune or (args.workload == "ensemble" and not args.no_autotune):
        tuning = lbmpcd.autotune(plist, lb_steps=5)
        plist = lbmpcd.with_tuning(plist, tuning)
        print(f"[bench] autotune: {tuning}", file=sys.stderr, flush=True)
    sim = lbmpcd.Sim(plist, device="cuda:0")
    print(f"[bench] {args.workload}: {len(plist)} channel(s), {tot['nodes']} nodes, {tot['particles']} "
          f"particles, workspace {sim.workspace_bytes / 2**30:.1f} GiB", file=sys.stderr, flush=True)
    sim.step(args.warmup)
    sim.sync()
    sim.timing(1)
    # the timed steps in five chunks, each bracketed by events on the library's
    # stream: the spread of the chunks shows how steady the rate is
    chunks = [args.steps // 5 + (1 if i < args.steps % 5 else 0) for i in range(5)]
    chunks = [n for n in chunks if n > 0]
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(chunks) + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(sim.stream)
    for i, n in enumerate(chunks):
        sim.step(n)
        evs[i + 1].record(sim.stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    chunk_ms = [evs[i].elapsed_time(evs[i + 1]) / n for i, n in enumerate(chunks)]
    sim.timing(0)
    kt = sim.timing_read()
    sim.sync()
    st = sim.stats()  # device counters shared by all channels of the context
    if st["dropped"] or st["misplaced"]:
        raise SystemExit(f"invalid run: {st}")
    dt = t1 - t0
    sps = args.steps / dt
    ms_per_step = 1e3 * dt / args.steps
    kp = kt["particles"]
    part_ms = kp["ms"] / max(kp["launches"], 1)
    per_launch = tot["launch_bytes"]
    achieved = per_launch / (part_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload)
    step_traffic = measured_step_traffic(args.workload)
    lb_ms = kt["lb_step"]["ms"] / max(kt["lb_step"]["launches"], 1)
    if args.workload == "ensemble":
        wl = (f"ensemble: 256 2D channels (D2Q9, widths 16-128, lengths 32-256, strip W/4 with 1-row "
              f"buffers, r 4, 5-20 ppc, FP64), {tot['nodes']} nodes, {tot['particles']} particles, "
              f"S {p['substeps']}, SRD {p['alpha_deg']} deg")
    else:
        lat = "D2Q9" if p["dim"] == 2 else "D3Q19"
        wl = (f"{args.workload}: {lat} {p['n'][0]}x{p['n'][1]}x{p['n'][2]} tau {p['tau']}, "
              f"slab y[{p['ylo']},{p['yhi']}) buffers {p['buf_lo']}/{p['buf_hi']}, r {p['refine']}, "
              f"{p['ppc']} ppc ({tot['particles']} particles), S {p['substeps']}, "
              f"{'MPCD-AT' if p.get('collision', 0) == 1 else 'SRD ' + str(p['alpha_deg']) + ' deg'}, "
              f"{'Chapman-Enskog' if p.get('reinject', 0) else 'Maxwell-Boltzmann'} exchange, "
              f"feedback {p['feedback']}")
    out = {
        "metric": "coupled steps/s: LB MLUPS + MPCD particle-updates/s, % HBM roofline",
        "value": sps,
        "unit": "coupled LB steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f64" if p["part_fp"] == 64 and p["lb_fp"] == 64 else
                  f"f32 particles, f{p['lb_fp']} LB populations, f64 cell sums and arithmetic"),
        "data": "synthetic (seeded Poiseuille channel; uniform-in-cell positions, Maxwellian velocities)",
        "config": {
            "workload": wl, "channels": len(plist),
            "lb_nodes": tot["nodes"], "particles": tot["particles"], "substeps": p["substeps"],
            "launch_shape": tuning if tuning else "default (tile_target 1280, 256 threads)",
        },
        "lb_mlups": tot["nodes"] * sps / 1e6,
        "mpcd_particle_updates_per_s": tot["particles"] * p["substeps"] * sps,
        "coupled_hbm_frac": tot["total_bytes"] * sps / 1e9 / HBM_PEAK_GBS,
        # counter-measured HBM traffic of the whole coupled step (rocprofv3
        # FETCH_SIZE + WRITE_SIZE of every kernel of an LB step) per second
        "coupled_counter_frac": (step_traffic * sps / 1e9 / HBM_PEAK_GBS) if step_traffic else None,
        "kernels_ms_per_launch": {k: v["ms"] / max(v["launches"], 1) for k, v in kt.items()},
        "chunk_ms_per_step": chunk_ms,
        "sample_window_misses": st["window_misses"],
        "median_chunk_ms_per_step": float(sorted(chunk_ms)[len(chunk_ms) // 2]),
        "roofline": {
            "bound": "hbm",
            "kernel": "k_particles (fused MPCD step)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": per_launch,
        },
        "lb_roofline": {
            "bound": "hbm", "kernel": "k_lb_step (collide and stream)",
            "achieved": tot["lb_bytes"] / (lb_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": tot["lb_bytes"] / (lb_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes_per_launch": tot["lb_bytes"],
        },
        "cpu_baseline": cpu,
    }
    if len(plist) > 1:
        out["per_instance_profiles"] = instance_profiles(sim, plist, args.profile_steps, args.profiles_out)
        del sim
        torch.cuda.empty_cache()
        out["batched_vs_one_by_one"] = one_by_one(lbmpcd, plist, ms_per_step)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
