"""The closure network's GELU (paper_2004_00304_amd/csrc/gelu.hpp): erf by
Abramowitz and Stegun's formula 7.1.26, compiled for the host with g++ and
checked against the exact erf.  The formula's own bound is 1.5e-7; binary32
evaluation adds the cancellation near 0 (about 6e-7 in all).  GELU and its
derivative follow; the oracle's network (oracle/mlp.py) uses the exact erf,
and the difference stays orders of magnitude below the BF16 rounding of the
activations (2^-9 relative)."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy.special import erf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2004_00304_amd", "csrc")

DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include "gelu.hpp"
int main() {
    char buf[64];
    while (scanf("%63s", buf) == 1) {
        float x = strtof(buf, 0), e;
        float r = lbmpcd::erf_as(x, &e);
        printf("%a %a %a %a\n", (double)r, (double)e, (double)lbmpcd::gelu(x), (double)lbmpcd::gelu_grad(x));
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
    src, exe = os.path.join(d, "g.cpp"), os.path.join(d, "g")
    open(src, "w").write(DRIVER)
    subprocess.run([gxx, "-O2", "-ffp-contract=off", "-I", HDR, src, "-o", exe, "-lm"], check=True)

    def call(x):
        x = np.asarray(x, np.float32)
        out = subprocess.run([exe], input="\n".join(float(v).hex() for v in x), capture_output=True,
                             text=True, check=True).stdout.split()
        return np.array([float.fromhex(t) for t in out]).reshape(-1, 4).T
    yield call
    shutil.rmtree(d, ignore_errors=True)


def test_erf_within_the_formula_bound(run):
    y = np.concatenate([np.linspace(-6, 6, 60001), [0.0, -0.0, 1e-8, 10.0, -10.0, 30.0]]).astype(np.float32)
    r, e, _, _ = run(y)
    yd = y.astype(np.float64)
    err = np.abs(r - erf(yd))
    assert err.max() <= 7e-7, (err.max(), y[err.argmax()])
    # away from the cancellation near 0: the formula's 1.5e-7 plus binary32
    # rounding of its terms
    far = np.abs(yd) >= 0.5
    assert err[far].max() <= 3.5e-7, err[far].max()
    # odd, saturating, and the exponential it hands on is exp(-y^2)
    # (near 0 the cancellation may return 0 itself, within the bound above)
    assert np.all(r * yd >= 0) and abs(r[np.where(y == 0)[0][0]]) <= 1e-8
    assert r[np.where(y == 30.0)[0][0]] == 1.0
    # (y^2 rounded in binary32 moves exp(-y^2) by about y^2 * 6e-8 relative)
    assert np.allclose(e, np.exp(-yd * yd), rtol=1e-5, atol=1e-37)


def test_gelu_and_its_derivative(run):
    x = np.linspace(-8, 8, 40001).astype(np.float32)
    _, _, g, gg = run(x)
    xd = x.astype(np.float64)
    cdf = 0.5 * (1.0 + erf(xd / np.sqrt(2.0)))
    pdf = np.exp(-0.5 * xd * xd) / np.sqrt(2.0 * np.pi)
    want_g, want_gg = xd * cdf, cdf + xd * pdf
    # binary32 arithmetic plus the erf error: absolute (for x << 0 the value
    # 1 + erf cancels in binary32 whatever erf is used), and relative where
    # the activation is not negligible, far below a BF16 unit (2^-9)
    assert np.abs(g - want_g).max() <= 2e-6 * np.abs(xd).max()
    rel = np.abs(g - want_g) / np.maximum(np.abs(want_g), 0.1)
    assert rel.max() <= 1e-5, rel.max()
    assert np.abs(gg - want_gg).max() <= 2e-6
    # the derivative is the slope of GELU
    h = 1e-3
    xs = np.linspace(-4, 4, 801).astype(np.float64)
    _, _, gp, _ = run(xs + h)
    _, _, gm, _ = run(xs - h)
    _, _, _, d = run(xs)
    assert np.abs((gp - gm) / (2 * h) - d).max() <= 2e-3
