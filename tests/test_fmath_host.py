"""The FP64 elementary functions of the HIP path's Box-Muller transform
(paper_2004_00304_amd/csrc/fmath.hpp: ln on (0, 1], sin and cos of 2 pi u on
[0, 1)), compiled for the host with g++ and checked against x87 extended
precision references at the edges of their domains and on random inputs of
the uniform grid the generator produces (multiples of 2^-53).  The exchange
step (Sec. 2.3) and the rotation axes (Eq. 4) draw through them."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2004_00304_amd", "csrc")

DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include "fmath.hpp"
int main() {
    char buf[64];
    while (scanf("%63s", buf) == 1) {
        double u = strtod(buf, 0), s, c;
        lbmpcd::sincos_2pi(u, &s, &c);
        printf("%a %a %a\n", lbmpcd::ln_unit(1.0 - u), s, c);
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def run():
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    d = tempfile.mkdtemp()
    src, exe = os.path.join(d, "fm.cpp"), os.path.join(d, "fm")
    open(src, "w").write(DRIVER)
    subprocess.run([gxx, "-O2", "-ffp-contract=off", "-I", HDR, src, "-o", exe, "-lm"], check=True)

    def call(u):
        out = subprocess.run([exe], input="\n".join(float(x).hex() for x in u), capture_output=True,
                             text=True, check=True).stdout.split()
        v = np.array([float.fromhex(t) for t in out]).reshape(-1, 3)
        return v[:, 0], v[:, 1], v[:, 2]
    yield call
    shutil.rmtree(d, ignore_errors=True)


def inputs():
    g = 2.0 ** -53
    edges = [0.0, g, 2 * g, 1 - g, 1 - 2 * g, 0.5 - g, 0.5, 0.5 + g]
    for q in range(1, 8):  # octant boundaries and their neighbours
        edges += [q / 8 - g, q / 8, q / 8 + g]
    for k in range(1, 54):  # 1 - u across every binade of (0, 1]
        edges += [2.0 ** -k, 1 - 2.0 ** -k]
    rng = np.random.default_rng(11)
    rand = rng.integers(0, 2 ** 53, size=20000, dtype=np.int64).astype(np.float64) * g
    return np.concatenate([np.array(edges), rand])


def reference(u):
    L = np.longdouble
    pi = np.arccos(L(-1))
    x = (L(1) - u.astype(L))
    a = L(2) * pi * u.astype(L)
    return np.log(x), np.sin(a), np.cos(a)


def ulps(got, ref, floor=0.0):
    """Error in units of the last place of the reference; `floor` is the
    reference's own absolute error (its pi is exact to about 1e-19, which
    matters only at the zeros of sin and cos)."""
    ref64 = ref.astype(np.float64)
    scale = np.spacing(np.maximum(np.abs(ref64), np.finfo(np.float64).tiny))
    err = np.maximum(np.abs(got.astype(np.longdouble) - ref) - np.longdouble(floor), 0)
    return (err / scale.astype(np.longdouble)).astype(np.float64)


def test_ln_unit(run):
    u = inputs()
    ln, _, _ = run(u)
    ref, _, _ = reference(u)
    assert ln[0] == 0.0  # ln 1
    e = ulps(ln, ref)
    assert e.max() <= 3.0, (e.max(), u[e.argmax()])


def test_sincos_2pi(run):
    u = inputs()
    _, s, c = run(u)
    _, rs, rc = reference(u)
    assert s[0] == 0.0 and c[0] == 1.0
    # exact quadrant points: u = 1/4, 1/2, 3/4
    for uq, (sq, cq) in ((0.25, (1.0, 0.0)), (0.5, (0.0, -1.0)), (0.75, (-1.0, 0.0))):
        i = int(np.flatnonzero(u == uq)[0])
        assert abs(s[i] - sq) == 0.0 and abs(c[i] - cq) == 0.0
    es, ec = ulps(s, rs, 1e-18), ulps(c, rc, 1e-18)
    assert es.max() <= 3.0, (es.max(), u[es.argmax()])
    assert ec.max() <= 3.0, (ec.max(), u[ec.argmax()])
    # the pair lies on the unit circle
    assert np.abs(s * s + c * c - 1.0).max() <= 4e-16


DRIVER32 = r"""
#include <stdio.h>
#include <stdint.h>
#include <string.h>
#include "fmath.hpp"
extern "C" float orc_ln32(float x);
extern "C" void orc_sincos32(float u, float* sn, float* cs);
static uint32_t bits(float v) { uint32_t b; memcpy(&b, &v, 4); return b; }
int main() {
    // every argument the binary32 generator produces: a = k 2^-24, k < 2^24
    long bad_ln = 0, bad_sc = 0;
    for (uint32_t k = 0; k < (1u << 24); ++k) {
        const float a = (float)k * 0x1p-24f;
        if (bits(lbmpcd::ln_unit32(1.0f - a)) != bits(orc_ln32(1.0f - a))) ++bad_ln;
        float s0, c0, s1, c1;
        lbmpcd::sincos_2pi32(a, &s0, &c0);
        orc_sincos32(a, &s1, &c1);
        if (bits(s0) != bits(s1) || bits(c0) != bits(c1)) ++bad_sc;
    }
    printf("%ld %ld\n", bad_ln, bad_sc);
    return 0;
}
"""


def test_binary32_functions_equal_the_oracle_bit_for_bit(tmp_path):
    """The binary32 ln and sin/cos of the HIP path (fmath.hpp, compiled for
    the host) and of the oracle are written separately from one definition,
    every step an IEEE binary32 operation: they agree to the bit on all 2^24
    arguments the generator produces.  Their accuracy is pinned against
    extended precision in tests/test_oracle_normals32.py."""
    from oracle import oracle as O
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    so = O.build(force=False)
    src, exe = tmp_path / "fm32.cpp", tmp_path / "fm32"
    src.write_text(DRIVER32)
    subprocess.run([gxx, "-O2", "-ffp-contract=off", "-fno-fast-math", "-I", HDR, str(src), so, "-o", str(exe),
                    "-lm", f"-Wl,-rpath,{os.path.dirname(so)}"], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert out == ["0", "0"], out
