"""Python binding of the HIP library ``liblbmpcd.so`` (C ABI in include/lbmpcd.h).

Argument marshalling only: every step of the coupled LB-MPCD method runs in the
library's gfx950 kernels.  PyTorch supplies the device memory (one workspace
tensor) and the HIP stream.  Importing this module loads the library and fails
loudly when it has not been built (``python -m paper_2004_00304_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# torch first: the library then binds to the HIP runtime torch carries.  Loaded
# the other way round the process would hold two HIP runtimes, and torch's
# device pointers and streams would mean nothing to the library's.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmpcd.so")

ABI_VERSION = 6

RHO, U, PI, POP, PART_POS, PART_VEL, CELL_ID, CELL_COUNT, CELL_VCM, PROFILE, UFINE, STATS, \
    PART_VEL_PENDING, CELL_START, NODE_MPCD_U, TFINE, NODE_FB_U = range(17)
FIELD_NAMES = dict(rho=RHO, u=U, pi=PI, pop=POP, pos=PART_POS, vel=PART_VEL, cell_id=CELL_ID,
                   cell_count=CELL_COUNT, cell_vcm=CELL_VCM, profile=PROFILE, ufine=UFINE, stats=STATS,
                   vel_pending=PART_VEL_PENDING, cell_start=CELL_START, node_mpcd_u=NODE_MPCD_U,
                   tfine=TFINE, node_fb_u=NODE_FB_U)
ERRORS = {1: "E_INVALID", 2: "E_NOMEM", 3: "E_DEVICE", 4: "E_OVERFLOW", 5: "E_STATE", 6: "E_UNSUPPORTED"}


class LbmpcdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("struct_size", C.c_uint32),
        ("dim", C.c_int32), ("n", C.c_int32 * 3), ("lb_fp", C.c_int32),
        ("tau", C.c_double), ("rho0", C.c_double), ("g", C.c_double * 3),
        ("walls_y", C.c_int32), ("mpcd", C.c_int32), ("ylo", C.c_int32), ("yhi", C.c_int32),
        ("buf_lo", C.c_int32), ("buf_hi", C.c_int32), ("refine", C.c_int32), ("substeps", C.c_int32),
        ("ppc", C.c_int32), ("part_fp", C.c_int32),
        ("mass", C.c_double), ("kT", C.c_double), ("alpha_deg", C.c_double),
        ("collision", C.c_int32), ("grid_shift", C.c_int32), ("feedback", C.c_int32),
        ("init_flow", C.c_int32), ("seed", C.c_uint64), ("instance", C.c_uint32),
        ("tile", C.c_int32 * 3), ("capacity_factor", C.c_double),
        ("tile_target", C.c_int32), ("wg_threads", C.c_int32), ("closure", C.c_int32),
        ("reinject", C.c_int32), ("ce_nu", C.c_double), ("fb_window", C.c_int32), ("deterministic", C.c_int32),
        ("schedule", C.c_int32),
    ]


class TrainOpts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_uint64)]


# the closure network's sizes (see include/lbmpcd.h)
CLOSURE_NF, CLOSURE_NOUT, CLOSURE_NPARAM, CLOSURE_NSTATS = 271, 9, 71177, 560


class Tuning(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("tile_target", C.c_int32), ("wg_threads", C.c_int32),
                ("tried", C.c_int32), ("ms_per_step", C.c_double), ("ms_default", C.c_double),
                ("schedule", C.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2004_00304_amd.build` "
                          "(the HIP library is the only compute path; there is no fallback)")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    L.lbmpcd_workspace_size.argtypes = [P, C.c_int32, C.POINTER(C.c_size_t)]
    L.lbmpcd_init.argtypes = [P, C.c_int32, P, C.c_size_t, P, C.POINTER(C.c_void_p)]
    L.lbmpcd_step.argtypes = [P, C.c_int32]
    L.lbmpcd_moments.argtypes = [P, C.c_int32, C.c_int32, P, C.c_size_t, C.c_int32]
    L.lbmpcd_field_bytes.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]
    L.lbmpcd_sample.argtypes = [P, C.c_int32]
    L.lbmpcd_get_state.argtypes = [P, C.c_int32, C.c_int32, P, C.c_size_t, C.c_int32]
    L.lbmpcd_set_state.argtypes = [P, C.c_int32, C.c_int32, P, C.c_size_t, C.c_int32]
    L.lbmpcd_sync.argtypes = [P]
    L.lbmpcd_destroy.argtypes = [P]
    L.lbmpcd_destroy.restype = None
    L.lbmpcd_timing.argtypes = [P, C.c_int32]
    L.lbmpcd_timing.restype = C.c_int
    L.lbmpcd_timing_read.argtypes = [P, P, C.c_int32]
    L.lbmpcd_timing_read.restype = C.c_int
    L.lbmpcd_graphs.argtypes = [P, C.c_int32]
    L.lbmpcd_graphs.restype = C.c_int
    L.lbmpcd_strerror.argtypes = [C.c_int]
    L.lbmpcd_strerror.restype = C.c_char_p
    L.lbmpcd_autotune.argtypes = [P, C.c_int32, P, C.c_size_t, P, C.c_int32, C.POINTER(Tuning)]
    L.lbmpcd_autotune.restype = C.c_int
    L.lbmpcd_closure_scratch_size.argtypes = [C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]
    L.lbmpcd_closure_collect.argtypes = [P, C.c_int32, P, P]
    L.lbmpcd_closure_train.argtypes = [P, P, P, C.c_int64, C.POINTER(TrainOpts), P, C.c_size_t, P]
    L.lbmpcd_closure_loss_grad.argtypes = [P, P, P, C.c_int64, P, C.c_size_t, P, P]
    L.lbmpcd_closure_forward.argtypes = [P, P, C.c_int64, P, P, C.c_size_t]
    L.lbmpcd_closure_features.argtypes = [P, P]
    L.lbmpcd_closure_predict.argtypes = [P, P]
    L.lbmpcd_closure_forward_noalloc.argtypes = [P, P, C.c_int64, P]
    L.lbmpcd_viscosity.argtypes = [C.POINTER(Params), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.lbmpcd_viscosity.restype = C.c_int
    L.lbmpcd_closure_weights.argtypes = [P, C.c_int32, P, C.c_size_t]
    L.lbmpcd_closure_enable.argtypes = [P, C.c_int32, C.c_double, C.c_int32, C.c_int32]
    L.lbmpcd_closure_check.argtypes = [P, C.c_int32, C.POINTER(C.c_double)]
    L.lbmpcd_closure_status.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    L.lbmpcd_closure_gemm_bf16.argtypes = [C.c_int64, C.c_int64, C.c_int64, P, P, P, P]
    for name in ("lbmpcd_closure_scratch_size", "lbmpcd_closure_collect", "lbmpcd_closure_train",
                 "lbmpcd_closure_loss_grad", "lbmpcd_closure_forward", "lbmpcd_closure_weights",
                 "lbmpcd_closure_enable", "lbmpcd_closure_check", "lbmpcd_closure_status",
                 "lbmpcd_closure_gemm_bf16", "lbmpcd_closure_features", "lbmpcd_closure_predict",
                 "lbmpcd_closure_forward_noalloc"):
        getattr(L, name).restype = C.c_int
    L.lbmpcd_last_error.argtypes = [P]
    L.lbmpcd_last_error.restype = C.c_char_p
    for name in ("lbmpcd_workspace_size", "lbmpcd_init", "lbmpcd_step", "lbmpcd_moments",
                 "lbmpcd_field_bytes", "lbmpcd_sample", "lbmpcd_get_state", "lbmpcd_set_state",
                 "lbmpcd_sync"):
        getattr(L, name).restype = C.c_int
    return L


_lib = _load()
EXPORTED = ("lbmpcd_workspace_size", "lbmpcd_init", "lbmpcd_step", "lbmpcd_moments",
            "lbmpcd_field_bytes", "lbmpcd_sample", "lbmpcd_get_state", "lbmpcd_set_state",
            "lbmpcd_sync", "lbmpcd_destroy", "lbmpcd_strerror", "lbmpcd_last_error", "lbmpcd_timing",
            "lbmpcd_timing_read", "lbmpcd_graphs", "lbmpcd_autotune", "lbmpcd_closure_scratch_size",
            "lbmpcd_closure_collect", "lbmpcd_closure_train", "lbmpcd_closure_loss_grad",
            "lbmpcd_closure_forward", "lbmpcd_closure_weights", "lbmpcd_closure_enable",
            "lbmpcd_closure_check", "lbmpcd_closure_status", "lbmpcd_closure_gemm_bf16",
            "lbmpcd_closure_features", "lbmpcd_closure_predict", "lbmpcd_viscosity",
            "lbmpcd_closure_forward_noalloc")

# rows of one lbmpcd_closure_forward_noalloc call
NOALLOC_MAX_ROWS = 8192

# candidate tile sizes of lbmpcd_autotune (expected particles per tile)
TUNE_TILE_TARGETS = (160, 320, 640, 1280)


def lib():
    return _lib


def params_struct(p: dict) -> Params:
    s = Params()
    s.abi_version = ABI_VERSION
    s.struct_size = C.sizeof(Params)
    s.dim = p["dim"]
    for k in range(3):
        s.n[k] = p["n"][k]
        s.g[k] = p["g"][k]
        s.tile[k] = p.get("tile", (0, 0, 0))[k]
    s.lb_fp = p["lb_fp"]
    s.tau, s.rho0 = p["tau"], p["rho0"]
    s.walls_y, s.mpcd = p["walls_y"], p["mpcd"]
    s.ylo, s.yhi, s.buf_lo, s.buf_hi = p["ylo"], p["yhi"], p["buf_lo"], p["buf_hi"]
    s.refine, s.substeps, s.ppc, s.part_fp = p["refine"], p["substeps"], p["ppc"], p["part_fp"]
    s.mass, s.kT, s.alpha_deg = p["mass"], p["kT"], p["alpha_deg"]
    s.collision, s.grid_shift, s.feedback, s.init_flow = (p["collision"], p["grid_shift"],
                                                          p["feedback"], p["init_flow"])
    s.seed, s.instance = p["seed"], p["instance"]
    s.capacity_factor = p.get("capacity_factor", 0.0)
    s.tile_target = p.get("tile_target", 0)
    s.wg_threads = p.get("wg_threads", 0)
    s.closure = p.get("closure", 0)
    s.reinject = p.get("reinject", 0)
    s.ce_nu = p.get("ce_nu", 0.0)
    s.fb_window = p.get("fb_window", 0)
    s.deterministic = p.get("deterministic", 0)
    s.schedule = p.get("schedule", 0)
    return s


def _check(rc: int, ctx=None):
    if rc != 0:
        raise LbmpcdError(rc, _lib.lbmpcd_last_error(ctx).decode())


def workspace_size(params) -> int:
    plist = params if isinstance(params, (list, tuple)) else [params]
    arr = (Params * len(plist))(*[params_struct(p) for p in plist])
    n = C.c_size_t()
    _check(_lib.lbmpcd_workspace_size(C.cast(arr, C.c_void_p), len(plist), C.byref(n)))
    return int(n.value)


def viscosity(params) -> tuple:
    """(nu_lb, nu_mpcd) of one parameter set (lbmpcd_viscosity; host only)."""
    ps = params_struct(params)
    nl, nm = C.c_double(), C.c_double()
    _check(_lib.lbmpcd_viscosity(C.byref(ps), C.byref(nl), C.byref(nm)))
    return float(nl.value), float(nm.value)


def autotune(params, lb_steps: int = 5, device="cuda", stream=None) -> dict:
    """Runs lbmpcd_autotune on a scratch workspace large enough for every
    candidate and returns the chosen launch shape (tile_target, wg_threads,
    schedule) with the timings."""
    import torch

    plist = list(params) if isinstance(params, (list, tuple)) else [params]
    need = 0
    for tt in TUNE_TILE_TARGETS:
        try:
            need = max(need, workspace_size([{**p, "tile_target": tt} for p in plist]))
        except LbmpcdError:
            pass
    arr = (Params * len(plist))(*[params_struct(p) for p in plist])
    dev = torch.device(device)
    if dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    out = Tuning()
    out.struct_size = C.sizeof(Tuning)
    with torch.cuda.device(dev):
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        rc = _lib.lbmpcd_autotune(C.cast(arr, C.c_void_p), len(plist), C.c_void_p(ws.data_ptr()), need,
                                  C.c_void_p(st.cuda_stream), int(lb_steps), C.byref(out))
        _check(rc, None)
        del ws
    return dict(tile_target=out.tile_target, wg_threads=out.wg_threads, schedule=out.schedule, tried=out.tried,
                ms_per_step=out.ms_per_step, ms_default=out.ms_default)


def gemm_bf16(A, B):
    """C = A B^T on the matrix cores (A: M x K, B: N x K, torch bfloat16 on
    the GPU, row-major) -> float32 M x N."""
    import torch
    A = A.contiguous()
    B = B.contiguous()
    M, K = A.shape
    N = B.shape[0]
    out = torch.empty(M, N, dtype=torch.float32, device=A.device)
    st = torch.cuda.current_stream(A.device)
    _check(_lib.lbmpcd_closure_gemm_bf16(M, N, K, C.c_void_p(A.data_ptr()), C.c_void_p(B.data_ptr()),
                                         C.c_void_p(out.data_ptr()), C.c_void_p(st.cuda_stream)))
    return out


def scratch_size(n: int, batch: int = 0) -> int:
    b = C.c_size_t()
    _check(_lib.lbmpcd_closure_scratch_size(int(n), int(batch), C.byref(b)))
    return int(b.value)


def with_tuning(params, tuning: dict):
    """The parameter dict(s) with the launch shape chosen by autotune."""
    upd = {"tile_target": tuning["tile_target"], "wg_threads": tuning["wg_threads"],
           "schedule": tuning.get("schedule", 0)}
    if isinstance(params, (list, tuple)):
        return [{**p, **upd} for p in params]
    return {**params, **upd}


class Sim:
    """One or more coupled channels advanced by the HIP library on one GPU."""

    def __init__(self, params, device="cuda", stream=None):
        import torch

        self.torch = torch
        self.plist = list(params) if isinstance(params, (list, tuple)) else [params]
        self.n_inst = len(self.plist)
        self.dim = self.plist[0]["dim"]
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self._arr = (Params * self.n_inst)(*[params_struct(p) for p in self.plist])
        nbytes = workspace_size(self.plist)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            h = C.c_void_p()
            rc = _lib.lbmpcd_init(C.cast(self._arr, C.c_void_p), self.n_inst,
                                  C.c_void_p(self.workspace.data_ptr()), nbytes,
                                  C.c_void_p(self.stream.cuda_stream), C.byref(h))
            _check(rc, None)
        self._h = h
        self.workspace_bytes = nbytes

    def close(self):
        """Wait for queued work and release the context (the workspace is torch's)."""
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            try:
                _lib.lbmpcd_sync(h)
            finally:
                _lib.lbmpcd_destroy(h)

    def __del__(self):
        if _lib is not None:  # module globals may already be gone at interpreter exit
            self.close()

    # -- stepping
    def step(self, n: int = 1):
        _check(_lib.lbmpcd_step(self._h, int(n)), self._h)

    def sync(self):
        _check(_lib.lbmpcd_sync(self._h), self._h)

    def sample(self, mode: int):
        _check(_lib.lbmpcd_sample(self._h, int(mode)), self._h)

    def graphs(self, enable: bool):
        """Replay steady-state steps from a captured HIP graph (default on)."""
        _check(_lib.lbmpcd_graphs(self._h, int(bool(enable))), self._h)

    # -- fields (device tensors)
    def field_bytes(self, field: int, inst: int = 0) -> int:
        n = C.c_size_t()
        _check(_lib.lbmpcd_field_bytes(self._h, field, inst, C.byref(n)), self._h)
        return int(n.value)

    def _alloc(self, field, inst, dtype):
        torch = self.torch
        nb = self.field_bytes(field, inst)
        item = torch.empty((), dtype=dtype).element_size()
        return torch.empty(nb // item, dtype=dtype, device=self.device)

    def moments(self, field, inst: int = 0):
        torch = self.torch
        field = FIELD_NAMES.get(field, field) if isinstance(field, str) else field
        if field == STATS:
            out = np.zeros(10, np.int64)
            _check(_lib.lbmpcd_moments(self._h, STATS, inst, out.ctypes.data_as(C.c_void_p), 80, 0),
                   self._h)
            keys = ("lb_steps", "sampled_steps", "dropped", "misplaced", "far_moves", "max_fill",
                    "particles", "cells", "window_misses", "bad_state")
            return dict(zip(keys, (int(x) for x in out)))
        dtype = torch.int32 if field in (CELL_ID, CELL_COUNT, CELL_START) else torch.float64
        if field == POP:
            dtype = torch.float64 if self.plist[inst]["lb_fp"] == 64 else torch.float32
        out = self._alloc(field, inst, dtype)
        with torch.cuda.device(self.device):
            _check(_lib.lbmpcd_moments(self._h, field, inst, C.c_void_p(out.data_ptr()),
                                       out.numel() * out.element_size(), 1), self._h)
        return out

    def get_state(self, field, inst: int = 0):
        field = FIELD_NAMES.get(field, field) if isinstance(field, str) else field
        return self.moments(field, inst)

    def set_state(self, field, src, inst: int = 0):
        torch = self.torch
        field = FIELD_NAMES.get(field, field) if isinstance(field, str) else field
        dtype = torch.float64
        if field == POP and self.plist[inst]["lb_fp"] == 32:
            dtype = torch.float32
        t = torch.as_tensor(src).to(device=self.device, dtype=dtype).contiguous()
        with torch.cuda.device(self.device):
            _check(_lib.lbmpcd_set_state(self._h, field, inst, C.c_void_p(t.data_ptr()),
                                         t.numel() * t.element_size(), 1), self._h)

    # -- numpy views in the oracle's layouts
    def shape(self, inst=0):
        nx, ny, nz = self.plist[inst]["n"]
        return (nz, ny, nx)

    def f(self, inst=0) -> np.ndarray:
        p = self.plist[inst]
        Q = 9 if p["dim"] == 2 else 19
        return self.get_state(POP, inst).cpu().numpy().reshape((Q,) + self.shape(inst)).astype(np.float64)

    def fields(self, inst=0):
        sh = self.shape(inst)
        rho = self.moments(RHO, inst).cpu().numpy().reshape(sh)
        u = self.moments(U, inst).cpu().numpy().reshape((3,) + sh)
        pi = self.moments(PI, inst).cpu().numpy().reshape((6,) + sh)
        return rho, u, pi

    def particles(self, inst=0):
        d = self.plist[inst]["dim"]
        pos = self.get_state(PART_POS, inst).cpu().numpy().reshape(d, -1)
        vel = self.get_state(PART_VEL, inst).cpu().numpy().reshape(d, -1)
        return pos, vel

    def binning(self, inst=0):
        """Cell of every particle (by id), cell counts and the cell centre-of-mass
        velocities of the last MPCD step (call right after step())."""
        d = self.plist[inst]["dim"]
        vcm = self.moments(CELL_VCM, inst).cpu().numpy().reshape(d, -1)
        cell = self.moments(CELL_ID, inst).cpu().numpy()
        count = self.moments(CELL_COUNT, inst).cpu().numpy()
        return dict(cell=cell, count=count, vcm=vcm)

    def cell_start(self, inst=0) -> np.ndarray:
        """Start of every cell of the last binning in a stable counting sort's order."""
        return self.moments(CELL_START, inst).cpu().numpy()

    def node_mpcd_u(self, inst=0) -> np.ndarray:
        """Mean sampled particle velocity per slab node in the last LB step, [dim][nz][ny_slab][nx]."""
        p = self.plist[inst]
        return self.moments(NODE_MPCD_U, inst).cpu().numpy().reshape(p["dim"], p["n"][2], p["yhi"] - p["ylo"],
                                                                      p["n"][0])

    def node_fb_u(self, inst=0) -> np.ndarray:
        """Running mean of the MPCD velocity per slab node that the feedback projects,
        [dim][nz][ny_slab][nx]."""
        p = self.plist[inst]
        return self.moments(NODE_FB_U, inst).cpu().numpy().reshape(p["dim"], p["n"][2], p["yhi"] - p["ylo"],
                                                                    p["n"][0])

    def profile(self, inst=0) -> np.ndarray:
        return self.moments(PROFILE, inst).cpu().numpy().reshape(-1, 4)

    def ufine(self, inst=0) -> np.ndarray:
        p = self.plist[inst]
        r = p["refine"]
        R = (p["yhi"] - p["ylo"]) * r
        Cz = p["n"][2] * r if p["dim"] == 3 else 1
        return self.moments(UFINE, inst).cpu().numpy().reshape(p["dim"], Cz, R, p["n"][0] * r)

    def tfine(self, inst=0) -> np.ndarray:
        """Chapman-Enskog tensor of the buffer cells of the last exchange step,
        [6][Cz][R][Cx] (xx, yy, zz, xy, xz, yz)."""
        p = self.plist[inst]
        r = p["refine"]
        R = (p["yhi"] - p["ylo"]) * r
        Cz = p["n"][2] * r if p["dim"] == 3 else 1
        return self.moments(TFINE, inst).cpu().numpy().reshape(6, Cz, R, p["n"][0] * r)

    def stats(self, inst=0) -> dict:
        return self.moments(STATS, inst)

    # -- learned closure
    def _scratch(self, n, batch=0):
        return self.torch.empty(scratch_size(n, batch), dtype=self.torch.uint8, device=self.device)

    def closure_collect(self, lb_steps: int):
        """(X, Y) device tensors: features and targets of every slab node
        averaged over lb_steps plain coupled steps."""
        t = self.torch
        p = self.plist[0]
        nslab = p["n"][0] * (p["yhi"] - p["ylo"]) * p["n"][2]
        X = t.empty(nslab, CLOSURE_NF, dtype=t.float32, device=self.device)
        Y = t.empty(nslab, CLOSURE_NOUT, dtype=t.float32, device=self.device)
        _check(_lib.lbmpcd_closure_collect(self._h, int(lb_steps), C.c_void_p(X.data_ptr()),
                                           C.c_void_p(Y.data_ptr())), self._h)
        return X, Y

    def closure_features(self):
        """Raw features of every slab node of the current populations."""
        t = self.torch
        p = self.plist[0]
        nslab = p["n"][0] * (p["yhi"] - p["ylo"]) * p["n"][2]
        X = t.empty(nslab, CLOSURE_NF, dtype=t.float32, device=self.device)
        _check(_lib.lbmpcd_closure_features(self._h, C.c_void_p(X.data_ptr())), self._h)
        return X

    def closure_train(self, X, Y, epochs=1, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=1):
        o = TrainOpts()
        o.struct_size = C.sizeof(TrainOpts)
        o.epochs, o.batch, o.lr, o.beta1, o.beta2, o.eps, o.seed = epochs, batch, lr, beta1, beta2, eps, seed
        X = X.contiguous()
        Y = Y.contiguous()
        n = X.shape[0]
        scr = self._scratch(n, batch)
        losses = np.zeros(epochs, np.float32)
        _check(_lib.lbmpcd_closure_train(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), n,
                                         C.byref(o), C.c_void_p(scr.data_ptr()), scr.numel(),
                                         losses.ctypes.data_as(C.c_void_p)), self._h)
        return losses

    def closure_loss_grad(self, X, Y):
        X = X.contiguous()
        Y = Y.contiguous()
        n = X.shape[0]
        scr = self._scratch(n, n)
        loss = C.c_double()
        g = np.zeros(CLOSURE_NPARAM, np.float32)
        _check(_lib.lbmpcd_closure_loss_grad(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), n,
                                             C.c_void_p(scr.data_ptr()), scr.numel(), C.byref(loss),
                                             g.ctypes.data_as(C.c_void_p)), self._h)
        return float(loss.value), g

    def closure_forward(self, X):
        X = X.contiguous()
        n = X.shape[0]
        scr = self._scratch(n, n)
        Y = self.torch.empty(n, CLOSURE_NOUT, dtype=self.torch.float32, device=self.device)
        _check(_lib.lbmpcd_closure_forward(self._h, C.c_void_p(X.data_ptr()), n, C.c_void_p(Y.data_ptr()),
                                           C.c_void_p(scr.data_ptr()), scr.numel()), self._h)
        return Y

    def closure_forward_noalloc(self, X):
        """lbmpcd_closure_forward_noalloc: the network on rows of raw features
        (at most NOALLOC_MAX_ROWS) with the library's own device array for the
        activations.  Only the output tensor is allocated here, by torch."""
        X = X.contiguous()
        n = X.shape[0]
        Y = self.torch.empty(n, CLOSURE_NOUT, dtype=self.torch.float32, device=self.device)
        _check(_lib.lbmpcd_closure_forward_noalloc(self._h, C.c_void_p(X.data_ptr()), n, C.c_void_p(Y.data_ptr())),
               self._h)
        return Y

    def closure_predict(self):
        """Network output in physical units for every slab node of the current
        populations (device tensor [nslab, 9]) through the fused inference
        kernel of the surrogate step."""
        p = self.plist[0]
        nslab = p["n"][0] * (p["yhi"] - p["ylo"]) * p["n"][2]
        Y = self.torch.empty(nslab, CLOSURE_NOUT, dtype=self.torch.float32, device=self.device)
        _check(_lib.lbmpcd_closure_predict(self._h, C.c_void_p(Y.data_ptr())), self._h)
        return Y

    def closure_weights(self, block=None):
        """Without argument: the FP32 parameter block (numpy); with one: load it."""
        if block is None:
            out = np.zeros(CLOSURE_NPARAM + CLOSURE_NSTATS, np.float32)
            _check(_lib.lbmpcd_closure_weights(self._h, 0, out.ctypes.data_as(C.c_void_p), out.nbytes), self._h)
            return out
        blk = np.ascontiguousarray(block, np.float32)
        _check(_lib.lbmpcd_closure_weights(self._h, 1, blk.ctypes.data_as(C.c_void_p), blk.nbytes), self._h)

    def closure_enable(self, on=True, tol=0.02, check_every=0, check_steps=40):
        _check(_lib.lbmpcd_closure_enable(self._h, int(on), float(tol), int(check_every), int(check_steps)),
               self._h)

    def closure_check(self, burst_steps=40) -> float:
        e = C.c_double()
        _check(_lib.lbmpcd_closure_check(self._h, int(burst_steps), C.byref(e)), self._h)
        return float(e.value)

    def closure_status(self) -> dict:
        on, fb, err = C.c_int32(), C.c_int32(), C.c_double()
        _check(_lib.lbmpcd_closure_status(self._h, C.byref(on), C.byref(fb), C.byref(err)), self._h)
        return dict(on=bool(on.value), fell_back=bool(fb.value), last_err=float(err.value))

    # -- kernel timing (HIP events on the context's stream)
    KERNEL_CLASSES = ("lb_step", "band", "interp", "particles", "closure")

    def timing(self, mode: int):
        _check(_lib.lbmpcd_timing(self._h, int(mode)), self._h)

    def timing_read(self) -> dict:
        out = np.zeros(10, np.float64)
        _check(_lib.lbmpcd_timing_read(self._h, out.ctypes.data_as(C.c_void_p), 5), self._h)
        return {k: dict(ms=float(out[2 * i]), launches=int(out[2 * i + 1]))
                for i, k in enumerate(self.KERNEL_CLASSES)}
