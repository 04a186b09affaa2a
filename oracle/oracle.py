"""ctypes wrapper of the plain FP64 CPU oracle (``liblbmpcd_oracle.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
CPU-baseline leg of the benchmark.  The product path never imports it.  It is
driven from the neutral parameter dicts of ``paper_2004_00304_amd.workloads``
and shares nothing else with the HIP binding.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmpcd_oracle.so")
SRC = os.path.join(_HERE, "lbmpcd_oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no fast-math, no FMA contraction."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("tau", C.c_double), ("rho0", C.c_double), ("g", C.c_double * 3),
        ("walls_y", C.c_int32), ("mpcd", C.c_int32), ("ylo", C.c_int32), ("yhi", C.c_int32),
        ("buf_lo", C.c_int32), ("buf_hi", C.c_int32), ("refine", C.c_int32),
        ("substeps", C.c_int32), ("ppc", C.c_int32), ("part_fp32", C.c_int32),
        ("mass", C.c_double), ("kT", C.c_double), ("alpha_deg", C.c_double),
        ("grid_shift", C.c_int32), ("feedback", C.c_int32), ("init_flow", C.c_int32),
        ("seed", C.c_uint64), ("instance", C.c_uint32), ("collision", C.c_int32),
        ("reinject", C.c_int32), ("ce_nu", C.c_double), ("fb_window", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_Params), C.POINTER(C.c_void_p)]
        L.orc_create.restype = C.c_int
        L.orc_destroy.argtypes = [P]
        L.orc_step.argtypes = [P, C.c_int32]
        L.orc_step.restype = C.c_int
        L.orc_sample.argtypes = [P, C.c_int32]
        for name in ("orc_num_particles", "orc_lb_step_count"):
            getattr(L, name).argtypes = [P]
            getattr(L, name).restype = C.c_int64
        for name in ("orc_num_cells", "orc_num_fine_rows"):
            getattr(L, name).argtypes = [P]
            getattr(L, name).restype = C.c_int32
        for name in ("orc_get_f", "orc_set_f", "orc_get_fstar", "orc_get_ufine", "orc_get_step_acc",
                     "orc_get_fb_u"):
            getattr(L, name).argtypes = [P, P]
        L.orc_get_moments.argtypes = [P, P, P, P]
        L.orc_get_shift.argtypes = [P, P]
        L.orc_refresh_ufine.argtypes = [P]
        L.orc_get_particles.argtypes = [P, P, P]
        L.orc_set_particles.argtypes = [P, P, P]
        L.orc_get_binning.argtypes = [P, P, P, P, P, P]
        L.orc_get_profile.argtypes = [P, P, P]
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_philox_stream.argtypes = [P, C.c_uint64, C.c_uint64, P]
        L.orc_u01.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_u01.restype = C.c_double
        L.orc_lattice.argtypes = [C.c_int32, P, P, P]
        L.orc_lattice.restype = C.c_int
        L.orc_feq.argtypes = [C.c_int32, C.c_double, P, P]
        L.orc_collide_node.argtypes = [C.c_int32, C.c_double, P, P]
        L.orc_box_muller.argtypes = [C.c_double, C.c_double, P, P]
        L.orc_ln32.argtypes = [C.c_float]
        L.orc_ln32.restype = C.c_float
        L.orc_sincos32.argtypes = [C.c_float, P, P]
        L.orc_normals32.argtypes = [P, C.c_int32, P]
        L.orc_normals32_n.argtypes = [P, C.c_int64, C.c_int32, P]
        L.orc_srd_rotate.argtypes = [C.c_int32, C.c_int32, P, C.c_double, C.c_double,
                                     C.c_double, P, P, C.c_double, P]
        L.orc_counting_sort.argtypes = [C.c_int32, P, C.c_int32, P, P, P]
        L.orc_at_collide.argtypes = [C.c_int32, C.c_int32, P, P, P, C.c_double, P]
        L.orc_nu_at.argtypes = [C.c_double] * 5
        L.orc_nu_at.restype = C.c_double
        L.orc_nu_kinetic.argtypes = [C.POINTER(_Params)]
        L.orc_nu_kinetic.restype = C.c_double
        L.orc_ce_nu.argtypes = [C.POINTER(_Params)]
        L.orc_ce_nu.restype = C.c_double
        L.orc_ce_tensor.argtypes = [P, P]
        L.orc_get_tfine.argtypes = [P, P]
        L.orc_ce_normals.argtypes = [C.POINTER(_Params), C.c_uint32, C.c_uint32, C.c_uint32, P, P]
        L.orc_ce_normals.restype = C.c_int32
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def params_struct(p: dict) -> _Params:
    s = _Params()
    s.dim = p["dim"]
    s.nx, s.ny, s.nz = p["n"]
    s.tau, s.rho0 = p["tau"], p["rho0"]
    for k in range(3):
        s.g[k] = p["g"][k]
    s.walls_y, s.mpcd = p["walls_y"], p["mpcd"]
    s.ylo, s.yhi, s.buf_lo, s.buf_hi = p["ylo"], p["yhi"], p["buf_lo"], p["buf_hi"]
    s.refine, s.substeps, s.ppc = p["refine"], p["substeps"], p["ppc"]
    s.part_fp32 = 1 if p["part_fp"] == 32 else 0
    s.mass, s.kT, s.alpha_deg = p["mass"], p["kT"], p["alpha_deg"]
    s.grid_shift, s.feedback, s.init_flow = p["grid_shift"], p["feedback"], p["init_flow"]
    s.seed, s.instance = p["seed"], p["instance"]
    s.collision = int(p.get("collision", 0))
    s.reinject = int(p.get("reinject", 0))
    s.ce_nu = float(p.get("ce_nu", 0.0))
    s.fb_window = int(p.get("fb_window", 0))
    return s


class Oracle:
    """One simulated channel held in host memory by the C oracle."""

    def __init__(self, p: dict):
        self.p = dict(p)
        self._L = lib()
        self._ps = params_struct(p)
        h = C.c_void_p()
        rc = self._L.orc_create(C.byref(self._ps), C.byref(h))
        if rc != 0:
            raise ValueError(f"orc_create failed ({rc}) for {p}")
        self._h = h
        self.dim = p["dim"]
        self.Q = 9 if p["dim"] == 2 else 19
        self.N = p["n"][0] * p["n"][1] * p["n"][2]
        self.Np = int(self._L.orc_num_particles(h))
        self.ncells = int(self._L.orc_num_cells(h)) if p["mpcd"] else 0
        self.R = int(self._L.orc_num_fine_rows(h)) if p["mpcd"] else 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.orc_destroy(h)
            self._h = None

    # -- stepping
    def step(self, n: int = 1):
        rc = self._L.orc_step(self._h, int(n))
        if rc != 0:
            raise RuntimeError(f"orc_step failed ({rc})")

    def sample(self, mode: int):
        self._L.orc_sample(self._h, int(mode))

    @property
    def t(self) -> int:
        return int(self._L.orc_lb_step_count(self._h))

    # -- state
    def shape(self):
        nx, ny, nz = self.p["n"]
        return (nz, ny, nx)

    def f(self) -> np.ndarray:
        out = np.empty((self.Q,) + self.shape(), np.float64)
        self._L.orc_get_f(self._h, _ptr(out))
        return out

    def set_f(self, f: np.ndarray):
        f = np.ascontiguousarray(f, np.float64)
        self._L.orc_set_f(self._h, _ptr(f))

    def fstar(self) -> np.ndarray:
        out = np.empty((self.Q,) + self.shape(), np.float64)
        self._L.orc_get_fstar(self._h, _ptr(out))
        return out

    def moments(self):
        rho = np.empty(self.shape(), np.float64)
        u = np.empty((3,) + self.shape(), np.float64)
        pi = np.empty((6,) + self.shape(), np.float64)
        self._L.orc_get_moments(self._h, _ptr(rho), _ptr(u), _ptr(pi))
        return rho, u, pi

    def particles(self):
        pos = np.zeros((self.dim, self.Np), np.float64)
        vel = np.zeros((self.dim, self.Np), np.float64)
        self._L.orc_get_particles(self._h, _ptr(pos), _ptr(vel))
        return pos, vel

    def set_particles(self, pos=None, vel=None):
        pa = np.ascontiguousarray(pos, np.float64) if pos is not None else None
        va = np.ascontiguousarray(vel, np.float64) if vel is not None else None
        self._L.orc_set_particles(self._h, _ptr(pa) if pa is not None else None,
                                  _ptr(va) if va is not None else None)

    def binning(self):
        cell = np.empty(self.Np, np.int32)
        count = np.empty(self.ncells, np.int32)
        start = np.empty(self.ncells, np.int32)
        order = np.empty(self.Np, np.int32)
        vcm = np.empty((3, self.ncells), np.float64)
        self._L.orc_get_binning(self._h, _ptr(cell), _ptr(count), _ptr(start), _ptr(order),
                                _ptr(vcm))
        return dict(cell=cell, count=count, start=start, order=order, vcm=vcm[: self.dim])

    def ufine(self) -> np.ndarray:
        p = self.p
        r = p["refine"]
        Cx = p["n"][0] * r
        Cz = p["n"][2] * r if self.dim == 3 else 1
        out = np.empty((3, Cz, self.R, Cx), np.float64)
        self._L.orc_get_ufine(self._h, _ptr(out))
        return out[: self.dim]

    def shift(self) -> np.ndarray:
        out = np.zeros(3, np.float64)
        self._L.orc_get_shift(self._h, _ptr(out))
        return out[: self.dim]

    def refresh_ufine(self):
        self._L.orc_refresh_ufine(self._h)

    def ce_tensor(self) -> np.ndarray:
        """Chapman-Enskog tensor of every node from the current populations,
        [6][nz][ny][nx] (xx, yy, zz, xy, xz, yz)."""
        out = np.empty((6,) + self.shape(), np.float64)
        self._L.orc_ce_tensor(self._h, _ptr(out))
        return out

    def tfine(self) -> np.ndarray:
        """Chapman-Enskog tensor of the buffer fine cells of the last exchange
        step, [6][Cz][R][Cx]."""
        p = self.p
        r = p["refine"]
        Cx = p["n"][0] * r
        Cz = p["n"][2] * r if self.dim == 3 else 1
        out = np.empty((6, Cz, self.R, Cx), np.float64)
        self._L.orc_get_tfine(self._h, _ptr(out))
        return out

    def profile(self):
        acc = np.empty((self.R, 4), np.float64)
        n = C.c_int64()
        self._L.orc_get_profile(self._h, _ptr(acc), C.byref(n))
        return acc, int(n.value)

    def fb_u(self) -> np.ndarray:
        """Running mean of the node samples that the feedback projects, [3][nz][yhi-ylo][nx]."""
        nx, _, nz = self.p["n"]
        out = np.empty((nz, self.p["yhi"] - self.p["ylo"], nx, 3), np.float64)
        self._L.orc_get_fb_u(self._h, _ptr(out))
        return np.moveaxis(out, -1, 0).copy()

    def step_acc(self) -> np.ndarray:
        nx, _, nz = self.p["n"]
        out = np.empty((nz, self.R, nx, 4), np.float64)
        self._L.orc_get_step_acc(self._h, _ptr(out))
        return out


# ---- building blocks -----------------------------------------------------------

def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, np.uint32)
    k = np.asarray(key, np.uint32)
    out = np.empty(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox_stream(key, first: int, n: int) -> np.ndarray:
    """Philox4x32-10 of the consecutive counters first .. first + n - 1: [n][4]."""
    k = np.asarray(key, np.uint32)
    out = np.empty((n, 4), np.uint32)
    lib().orc_philox_stream(_ptr(k), int(first), int(n), _ptr(out))
    return out


def u01(lo: int, hi: int) -> float:
    return float(lib().orc_u01(lo, hi))


def lattice(dim: int):
    c = np.empty((19, 3), np.int32)
    w = np.empty(19, np.float64)
    opp = np.empty(19, np.int32)
    Q = lib().orc_lattice(dim, _ptr(c), _ptr(w), _ptr(opp))
    return c[:Q].copy(), w[:Q].copy(), opp[:Q].copy()


def feq(dim: int, rho: float, u) -> np.ndarray:
    uu = np.zeros(3, np.float64)
    uu[: len(u)] = u
    out = np.empty(19, np.float64)
    lib().orc_feq(dim, float(rho), _ptr(uu), _ptr(out))
    return out[: (9 if dim == 2 else 19)].copy()


def collide_node(dim: int, tau: float, g, f) -> np.ndarray:
    gg = np.zeros(3, np.float64)
    gg[: len(g)] = g
    ff = np.zeros(19, np.float64)
    Q = 9 if dim == 2 else 19
    ff[:Q] = f
    lib().orc_collide_node(dim, float(tau), _ptr(gg), _ptr(ff))
    return ff[:Q].copy()


def box_muller(u0: float, u1: float):
    z0 = np.zeros(1)
    z1 = np.zeros(1)
    lib().orc_box_muller(float(u0), float(u1), _ptr(z0), _ptr(z1))
    return float(z0[0]), float(z1[0])


def ln32(x) -> np.ndarray:
    """The binary32 ln on (0, 1] of the binary32 normals, elementwise."""
    x = np.atleast_1d(np.asarray(x, np.float32))
    return np.array([lib().orc_ln32(float(v)) for v in x], np.float32)


def sincos32(u):
    """The binary32 sin and cos of 2 pi u, elementwise: (sin, cos)."""
    u = np.atleast_1d(np.asarray(u, np.float32))
    sn, cs = np.zeros(1, np.float32), np.zeros(1, np.float32)
    out = np.empty((2, u.size), np.float32)
    for i, v in enumerate(u):
        lib().orc_sincos32(float(v), _ptr(sn), _ptr(cs))
        out[0, i], out[1, i] = sn[0], cs[0]
    return out[0], out[1]


def normals32(w, dim: int = 3) -> np.ndarray:
    """The binary32 normals of Philox blocks w [n][4]: [n][3] (z2 = 0 in 2D)."""
    w = np.ascontiguousarray(np.asarray(w, np.uint32).reshape(-1, 4))
    z = np.empty((w.shape[0], 3), np.float32)
    lib().orc_normals32_n(_ptr(w), int(w.shape[0]), int(dim), _ptr(z))
    return z


def srd_rotate(dim, vel, alpha_deg, sign2d=1.0, axis=(0.0, 0.0, 1.0), p_virt=(0, 0, 0), m_virt=0.0):
    v = np.ascontiguousarray(vel, np.float64).copy()
    n = v.shape[1]
    a = np.radians(alpha_deg)
    ax = np.asarray(axis, np.float64)
    pv = np.asarray(p_virt, np.float64)
    vcm = np.zeros(3)
    lib().orc_srd_rotate(dim, n, _ptr(v), float(np.cos(a)), float(np.sin(a)), float(sign2d),
                         _ptr(ax), _ptr(pv), float(m_virt), _ptr(vcm))
    return v, vcm[:dim]


def at_collide(dim, vel, vran, p_virt=(0, 0, 0), m_virt=0.0):
    """MPCD-AT collision (Eq. 6) of vel [dim][n] with random velocities vran [dim][n]."""
    v = np.ascontiguousarray(vel, np.float64).copy()
    r = np.ascontiguousarray(vran, np.float64)
    pv = np.asarray(p_virt, np.float64)
    vcm = np.zeros(3)
    lib().orc_at_collide(dim, v.shape[1], _ptr(v), _ptr(r), _ptr(pv), float(m_virt), _ptr(vcm))
    return v, vcm[:dim]


def nu_at(kT, mass, dt, a, N):
    """Kinematic viscosity of MPCD-AT, Eq. 7."""
    return float(lib().orc_nu_at(float(kT), float(mass), float(dt), float(a), float(N)))


def nu_kinetic(p: dict) -> float:
    """Kinetic part of the MPCD viscosity of a parameter set."""
    ps = params_struct(p)
    return float(lib().orc_nu_kinetic(C.byref(ps)))


def ce_nu(p: dict) -> float:
    """Stress coefficient of the Chapman-Enskog exchange (ce_nu, or the
    post-collision kinetic stress nu_kin - kT dt / (2m))."""
    ps = params_struct(p)
    return float(lib().orc_ce_nu(C.byref(ps)))


def ce_normals(p: dict, ids, t: int, sub: int, T) -> tuple:
    """Chapman-Enskog exchange deviates (in units of sqrt(kT/m)) of the
    elements ids for the tensor T[6]: returns z [3][n] and the accepted
    attempt of each element."""
    ps = params_struct(p)
    T = np.ascontiguousarray(T, np.float64)
    ids = np.asarray(ids, np.uint32)
    z = np.empty((3, len(ids)))
    att = np.empty(len(ids), np.int32)
    zz = np.empty(3)
    L = lib()
    for i, e in enumerate(ids):
        att[i] = L.orc_ce_normals(C.byref(ps), int(e), int(t), int(sub), _ptr(T), _ptr(zz))
        z[:, i] = zz
    return z, att


def counting_sort(cell, nc):
    cell = np.ascontiguousarray(cell, np.int32)
    count = np.empty(nc, np.int32)
    start = np.empty(nc, np.int32)
    order = np.empty(len(cell), np.int32)
    lib().orc_counting_sort(len(cell), _ptr(cell), nc, _ptr(count), _ptr(start), _ptr(order))
    return count, start, order


class Probe:
    """Geometry-only oracle state: per-particle and per-cell steps of the
    method on caller arrays, for sampled checks of runs too large to run
    through the full oracle."""

    def __init__(self, p: dict):
        self.p = dict(p)
        L = lib()
        if not getattr(L, "_probe_types", False):
            P = C.c_void_p
            L.orc_create_geometry.argtypes = [C.POINTER(_Params), C.POINTER(C.c_void_p)]
            L.orc_create_geometry.restype = C.c_int
            L.orc_grid_shift.argtypes = [P, C.c_uint32, C.c_uint32, P]
            L.orc_bin_positions.argtypes = [P, P, C.c_int64, P, P]
            L.orc_exchange_stream.argtypes = [P, C.c_uint32, C.c_uint32, C.c_int64, P, P, P, P, P]
            L.orc_in_buffer.argtypes = [P, P]
            L.orc_in_buffer.restype = C.c_int32
            L.orc_collide_cell.argtypes = [P, C.c_int32, C.c_uint32, C.c_uint32, P, C.c_int32, P, P, P]
            L.orc_interpolate.argtypes = [P, P, P]
            L._probe_types = True
        self._L = L
        self._ps = params_struct(p)
        h = C.c_void_p()
        rc = L.orc_create_geometry(C.byref(self._ps), C.byref(h))
        if rc != 0:
            raise ValueError(f"orc_create_geometry failed ({rc})")
        self._h = h
        self.dim = p["dim"]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.orc_destroy(h)
            self._h = None

    def shift(self, t: int, sub: int) -> np.ndarray:
        out = np.zeros(3)
        self._L.orc_grid_shift(self._h, t, sub, _ptr(out))
        return out

    def bin(self, sh, pos) -> np.ndarray:
        pos = np.ascontiguousarray(pos, np.float64)
        sh = np.ascontiguousarray(sh, np.float64)
        n = pos.shape[1]
        out = np.empty(n, np.int32)
        self._L.orc_bin_positions(self._h, _ptr(sh), n, _ptr(pos), _ptr(out))
        return out

    def exchange_stream(self, t, sub, ids, pos, vel, u, tens=None):
        ids = np.ascontiguousarray(ids, np.uint32)
        pos = np.ascontiguousarray(pos, np.float64).copy()
        vel = np.ascontiguousarray(vel, np.float64).copy()
        u = np.ascontiguousarray(u, np.float64)
        tp = None
        if tens is not None:
            tens = np.ascontiguousarray(tens, np.float64)
            tp = _ptr(tens)
        self._L.orc_exchange_stream(self._h, t, sub, len(ids), _ptr(ids), _ptr(pos), _ptr(vel), _ptr(u), tp)
        return pos, vel

    def in_buffer(self, r) -> bool:
        rr = np.zeros(3)
        rr[: len(r)] = r
        return bool(self._L.orc_in_buffer(self._h, _ptr(rr)))

    def interpolate(self, unode) -> np.ndarray:
        """Buffer fine-cell velocities [dim][Cz][R][Cx] from node velocities [3][nz][ny][nx]."""
        p = self.p
        r = p["refine"]
        R = (p["yhi"] - p["ylo"]) * r
        Cx = p["n"][0] * r
        Cz = p["n"][2] * r if self.dim == 3 else 1
        u = np.ascontiguousarray(unode, np.float64)
        out = np.zeros((3, Cz, R, Cx))
        self._L.orc_interpolate(self._h, _ptr(u), _ptr(out))
        return out[: self.dim]

    def collide_cell(self, c, t, sub, sh, vel, ids=None):
        v = np.ascontiguousarray(vel, np.float64).copy()
        sh = np.ascontiguousarray(sh, np.float64)
        vcm = np.zeros(3)
        idp = None
        if ids is not None:
            ids = np.ascontiguousarray(ids, np.int32)
            idp = _ptr(ids)
        self._L.orc_collide_cell(self._h, int(c), t, sub, _ptr(sh), v.shape[1], idp, _ptr(v), _ptr(vcm))
        return v, vcm[: self.dim]
