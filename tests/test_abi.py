"""The C-ABI library loads on a CPU-only host, exports every entry point that
include/lbmpcd.h declares, sizes workspaces and rejects bad parameters
(host logic only; no compute call needs a GPU here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2004_00304_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def binding():
    from paper_2004_00304_amd import lbmpcd
    return lbmpcd


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbmpcd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbmpcd_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(binding):
    names = declared_functions()
    assert len(names) >= 12
    lib = ctypes.CDLL(binding.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(binding.EXPORTED)


def test_params_struct_matches_header(binding):
    """The ctypes mirror has the size the library checks (struct_size)."""
    p = binding.params_struct(W.channel_2d())
    assert p.struct_size == ctypes.sizeof(binding.Params)
    assert binding.workspace_size(W.channel_2d()) > 0


def test_workspace_sizes(binding):
    s1 = binding.workspace_size(W.channel_2d())
    s3 = binding.workspace_size(W.channel_3d())
    # the 3D channel holds 167,772,160 FP32 particles in two tile stores
    assert s3 > 2 * 167_772_160 * 28
    assert s3 < 40 * 2 ** 30
    assert s1 < s3
    big = binding.workspace_size(W.thin_film_3d())
    assert big < 200 * 2 ** 30  # fits one MI355X (288 GB)
    ens = binding.workspace_size(W.ensemble(8))
    assert ens > 0


@pytest.mark.parametrize("kw,code", [
    (dict(tau=0.5), 1), (dict(dim=4), 1), (dict(lb_fp=16), 1), (dict(ylo=20, yhi=10), 1),
    (dict(buf_lo=5, buf_hi=5), 1), (dict(walls_y=1, ylo=0, buf_lo=1), 1), (dict(collision=2), 6),
    (dict(part_fp=16), 1), (dict(refine=0), 1), (dict(n=(8, 8, 2)), 1),
    (dict(walls_y=0, ylo=0, yhi=8), 6), (dict(substeps=300), 1),
    (dict(reinject=2), 1), (dict(reinject=1, kT=0.0), 1), (dict(ce_nu=float("nan")), 1),
    (dict(ce_nu=float("inf")), 1), (dict(reinject=1, alpha_deg=0.0), 1),
    (dict(deterministic=2), 1), (dict(deterministic=1, reinject=1), 6), (dict(schedule=2), 1),
    (dict(dim=3, n=(16, 16, 8), ylo=4, yhi=12, buf_lo=1, buf_hi=1, closure=1, deterministic=1), 6),
])
def test_invalid_params(binding, kw, code):
    with pytest.raises(binding.LbmpcdError) as e:
        binding.workspace_size(W.make(**kw))
    assert e.value.code == code


def test_mixed_batch_rejected(binding):
    with pytest.raises(binding.LbmpcdError):
        binding.workspace_size([W.channel_2d(), W.small_3d()])
    with pytest.raises(binding.LbmpcdError):
        binding.workspace_size([W.channel_2d(), W.make(reinject=1)])
    with pytest.raises(binding.LbmpcdError):
        binding.workspace_size([W.channel_2d(), {**W.channel_2d(), "deterministic": 1, "instance": 1}])


def test_chapman_enskog_workspace(binding):
    """The Chapman-Enskog exchange adds six doubles per band node and per
    buffer cell, and nothing else."""
    p = W.channel_2d()
    base = binding.workspace_size(p)
    ce = binding.workspace_size(W.make(reinject=1))
    nx, ny, nz = p["n"]
    band_nodes = nx * (p["yhi"] - p["ylo"] + 2) * nz  # the slab rows and one more on each side
    buffer_cells = (p["buf_lo"] + p["buf_hi"]) * p["refine"] * nx * p["refine"]
    # both regions are 256-byte aligned; without the exchange each still takes 256 bytes
    assert ce - base == 6 * 8 * (buffer_cells + band_nodes) - 2 * 256


def test_abi_version_checked(binding):
    p = binding.params_struct(W.channel_2d())
    p.abi_version = 99
    n = ctypes.c_size_t()
    rc = binding.lib().lbmpcd_workspace_size(ctypes.byref(p), 1, ctypes.byref(n))
    assert rc == 1
    assert b"abi" in binding.lib().lbmpcd_last_error(None)


def test_strerror(binding):
    L = binding.lib()
    assert L.lbmpcd_strerror(0) == b"ok"
    assert L.lbmpcd_strerror(4) == b"particle tile overflow"
    assert L.lbmpcd_strerror(77) == b"unknown error"


def test_null_context_calls_fail_cleanly(binding):
    L = binding.lib()
    assert L.lbmpcd_step(None, 1) == 1
    assert L.lbmpcd_sync(None) == 1
    L.lbmpcd_destroy(None)


@pytest.mark.parametrize("kw", [dict(wg_threads=64), dict(tile_target=-1), dict(tile_target=1 << 20),
                                dict(tile=(3, 2, 1))])
def test_invalid_launch_shape(binding, kw):
    with pytest.raises(binding.LbmpcdError) as e:
        binding.workspace_size(W.make(**kw))
    assert e.value.code == 1


def test_mixed_workgroup_sizes_rejected(binding):
    with pytest.raises(binding.LbmpcdError):
        binding.workspace_size([W.channel_2d(), W.make(wg_threads=512)])


def test_tile_target_sets_the_tile(binding):
    """A smaller tile target gives smaller tiles, hence more tile metadata
    and a different workspace size; the same target reproduces the size."""
    a = binding.workspace_size(W.make(tile_target=160))
    b = binding.workspace_size(W.make(tile_target=1280))
    assert a != b
    assert a == binding.workspace_size(W.make(tile_target=160))


def test_autotune_argument_checks(binding):
    """Argument errors are reported before any device work."""
    lib = binding.lib()
    arr = (binding.Params * 1)(binding.params_struct(W.channel_2d()))
    out = binding.Tuning()
    out.struct_size = 3  # wrong
    rc = lib.lbmpcd_autotune(ctypes.cast(arr, ctypes.c_void_p), 1, None, 0, None, 1, ctypes.byref(out))
    assert rc == 1
    out.struct_size = ctypes.sizeof(binding.Tuning)
    arr[0].tile[0] = 4
    rc = lib.lbmpcd_autotune(ctypes.cast(arr, ctypes.c_void_p), 1, None, 0, None, 1, ctypes.byref(out))
    assert rc == 1
    assert b"tile" in lib.lbmpcd_last_error(None)


def test_viscosity_matches_eq7_and_the_oracle(binding):
    """lbmpcd_viscosity (host arithmetic of the library): the LB viscosity of
    BGK, and for MPCD-AT Eq. 7 at dt = 1/S as the oracle evaluates it; 2D
    SRD against the formula the long-run test uses; 3D SRD as the oracle's
    kinetic term plus the collisional term a^2 (1 - cos a)(N-1+e^-N)/(18 dt N)."""
    from oracle import oracle as O
    p = W.small_3d(collision=1, kT=0.3, mass=1.5)
    nl, nm = binding.viscosity(p)
    assert nl == pytest.approx((p["tau"] - 0.5) / 3.0, rel=1e-15)
    assert nm == pytest.approx(O.nu_at(p["kT"], p["mass"], 1.0 / p["substeps"], 1.0 / p["refine"], p["ppc"]),
                               rel=1e-13)
    q = W.small_2d()
    _, ns = binding.viscosity(q)
    a, dt, N, al = 1.0 / q["refine"], 1.0 / q["substeps"], q["ppc"], np.deg2rad(q["alpha_deg"])
    e = N - 1 + np.exp(-N)
    ref = q["kT"] * dt / q["mass"] * (N / (e * (1 - np.cos(2 * al))) - 0.5) + a * a * (1 - np.cos(al)) * e / (12 * dt * N)
    assert ns == pytest.approx(ref, rel=1e-13)
    r3 = W.small_3d()
    _, n3 = binding.viscosity(r3)
    a, dt, N, al = 1.0 / r3["refine"], 1.0 / r3["substeps"], r3["ppc"], np.deg2rad(r3["alpha_deg"])
    e = N - 1 + np.exp(-N)
    ref3 = O.nu_kinetic(r3) + a * a * (1 - np.cos(al)) * e / (18 * dt * N)
    assert n3 == pytest.approx(ref3, rel=1e-13)


def test_one_hip_runtime_whatever_the_import_order():
    """Importing the binding before torch must not load a second HIP runtime
    (torch's device memory and streams would be foreign to the library's)."""
    import subprocess
    import sys
    code = ("from paper_2004_00304_amd import lbmpcd\n"
            "import torch\n"
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, check=True,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert out.stdout.strip() == "1", out.stdout + out.stderr


def test_binding_fails_loudly_without_the_library(tmp_path):
    """The HIP library is the only compute path: a copy of the package
    without liblbmpcd.so refuses to import instead of falling back."""
    import shutil
    import subprocess
    import sys
    src = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2004_00304_amd")
    shutil.copytree(src, tmp_path / "paper_2004_00304_amd",
                    ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__", "csrc"))
    r = subprocess.run([sys.executable, "-c", "from paper_2004_00304_amd import lbmpcd"], cwd=tmp_path,
                       capture_output=True, text=True)
    assert r.returncode != 0 and "is not built" in r.stderr, r.stderr[-500:]


def test_product_never_touches_the_oracle():
    """The oracle is test infrastructure: no source of the package (Python,
    HIP, C++) imports, includes or loads it."""
    root = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2004_00304_amd")
    hits = []
    for dirpath, _, files in os.walk(root):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn), encoding="utf-8").read()
                if re.search(r"import\s+oracle|from\s+oracle|lbmpcd_oracle|orc_", text):
                    hits.append(fn)
    assert not hits, hits
