"""Pins of the oracle's MPCD-AT collision (Eq. 6) and of the MPCD-AT
viscosity (Eq. 7).

* Table 1 lists nu_MPCD = 0.167 for the three runs; Eq. 7 with their a, kT
  and N and a unit MPCD time step reproduces it to the precision kT is
  printed with (tests/golden/table1_mpcd_at.json).  A time step of 1/4 instead
  (kinetic part x 1/4, collisional part x 4) misses by more than 20 %, so
  the pin fixes the time-step scaling of both terms.
* Limits: N -> infinity gives kT dt / (2 m) + a^2 / (12 dt).
* The collision conserves the cell's momentum (with virtual wall particles:
  it sets the real particles' mean to the centre of mass that includes them),
  forgets the relative velocities it is given (two inputs with the same
  centre of mass give the same output), leaves a lone particle unchanged,
  and thermalises: relative velocities have variance (N - 1)/N kT/m per
  component over many cells."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def test_table1_viscosities():
    rows = json.load(open(os.path.join(HERE, "golden", "table1_mpcd_at.json")))["rows"]
    for r in rows:
        nu = O.nu_at(r["kT"], 1.0, 1.0, r["a"], r["N"])
        assert abs(nu - r["nu_mpcd"]) / r["nu_mpcd"] <= 0.03, (r, nu)
        wrong_dt = O.nu_at(r["kT"], 1.0, 0.25, r["a"], r["N"])
        assert abs(wrong_dt - r["nu_mpcd"]) / r["nu_mpcd"] > 0.2


def test_viscosity_limits_and_values():
    kT, m, dt, a = 0.3, 2.0, 0.25, 0.5
    big = O.nu_at(kT, m, dt, a, 1e6)
    assert big == pytest.approx(kT * dt / (2 * m) + a * a / (12 * dt), rel=1e-6)
    # N = 1: the kinetic bracket is 1/e^-1 - 1/2, the collisional one e^-1
    one = O.nu_at(kT, m, dt, a, 1.0)
    e = np.exp(-1.0)
    assert one == pytest.approx(kT * dt / m * (1 / e - 0.5) + a * a / (12 * dt) * e, rel=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_at_conserves_momentum_and_forgets_relative_velocities(dim):
    rng = np.random.default_rng(3)
    n = 17
    v = rng.normal(0.2, 1.0, (dim, n))
    vr = rng.normal(0.0, 0.6, (dim, n))
    out, vcm = O.at_collide(dim, v, vr)
    assert np.allclose(out.sum(axis=1), v.sum(axis=1), rtol=0, atol=1e-13)
    assert np.allclose(vcm, v.mean(axis=1), rtol=0, atol=1e-15)
    # same centre of mass, different relative velocities: same result
    w = v.mean(axis=1, keepdims=True) + rng.normal(0.0, 3.0, (dim, n))
    w += v.mean(axis=1, keepdims=True) - w.mean(axis=1, keepdims=True)
    out2, _ = O.at_collide(dim, w, vr)
    assert np.allclose(out2, out, rtol=0, atol=1e-13)
    # a lone particle keeps its velocity
    one, _ = O.at_collide(dim, v[:, :1], vr[:, :1])
    assert np.allclose(one, v[:, :1], rtol=0, atol=1e-15)


def test_at_virtual_wall_particles():
    rng = np.random.default_rng(4)
    v = rng.normal(0.0, 1.0, (2, 5))
    pv, mv = np.array([0.7, -0.3, 0.0]), 3.0
    out, vcm = O.at_collide(2, v, rng.normal(0.0, 0.5, (2, 5)), pv, mv)
    expect = (v.sum(axis=1) + pv[:2]) / (5 + mv)
    assert np.allclose(vcm, expect, rtol=0, atol=1e-15)
    assert np.allclose(out.mean(axis=1), expect, rtol=0, atol=1e-14)


def test_at_thermalises_cells():
    """Full oracle collision (its own random stream) of many cells of N
    particles: the velocity relative to the cell mean has variance
    (N - 1)/N kT/m per component, whatever the input."""
    from paper_2004_00304_amd import workloads as W
    p = W.small_3d(collision=1, kT=0.4, mass=1.3)
    orc = O.Probe(p)
    sh = np.zeros(3)
    n, cells = 6, 4000
    rel = []
    rng = np.random.default_rng(9)
    for c in range(cells):
        v = rng.normal(0.0, 5.0, (3, n))  # far from the target temperature
        out, _ = orc.collide_cell(c, 7, 1, sh, v, ids=np.arange(c * n, (c + 1) * n))
        rel.append(out - out.mean(axis=1, keepdims=True))
    rel = np.concatenate(rel, axis=1)
    var = (rel ** 2).mean()
    target = (n - 1) / n * p["kT"] / p["mass"]
    # sample variance of ~72k Gaussian values: relative standard error 0.5 %
    assert abs(var / target - 1) < 0.03, (var, target)
