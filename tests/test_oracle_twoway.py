"""Pins of the oracle's two-way coupling (feedback on): boundedness of the
windowed projection over 10^4 LB steps, against the instantaneous one.

The projection of MPCD averages onto the LB equilibria is not in the paper,
which couples one way (Sec. 2.3).  The paper averages its MPCD profiles over
many samples because a single sample is dominated by thermal noise
(Sec. 3.1); here a slab node of r^d cells holds about 160 particles, whose
mean carries a noise of 0.046 against a flow of 0.05.  The oracle projects a
running mean over LB steps (window 50 by default).  On the 2D channel of the
two-way long run (narrowed to 16 nodes along the flow so that 10^4 LB steps
take about a minute) the windowed run keeps rho within 2 % and |u| within
twice the flow; the instantaneous projection (window 1) drives rho beyond
10 % and |u| to five times the flow within 1000 LB steps.  The time-averaged
profile of the full-width channel against the two-way closed form is checked
on the GPU (100,000 LB steps): the oracle at this width is too noisy for it
in CPU time."""
import numpy as np
import pytest

from paper_2004_00304_amd import workloads as W


def _channel(**kw):
    return W.make(n=(16, 32, 1), tau=0.8, g=(4e-5, 0.0, 0.0), ylo=12, yhi=20, buf_lo=2, buf_hi=2, ppc=10,
                  feedback=1, init_flow=1, **kw)


def _excursion(o, steps, every):
    """Largest |rho - 1| and |u| seen every `every` LB steps over `steps`."""
    drho, umax = 0.0, 0.0
    for _ in range(steps // every):
        o.step(every)
        rho, u, _ = o.moments()
        drho = max(drho, float(np.abs(rho - 1.0).max()))
        umax = max(umax, float(np.abs(u).max()))
    return drho, umax


@pytest.mark.slow
def test_windowed_feedback_stays_bounded(oracle_lib):
    p = _channel()
    o = oracle_lib.Oracle(p)
    drho, umax = _excursion(o, 1000, 500)
    o.sample(1)
    d2, u2 = _excursion(o, 9000, 500)
    assert max(drho, d2) < 0.05 and max(umax, u2) < 0.12, (drho, umax, d2, u2)
    # the flow is carried: the time-averaged interior rows of the slab sit
    # near the two-way closed form's 0.0556 (at this width the mean flow
    # wanders by tens of percent over 10^4 steps; the GPU test checks 2 %)
    r = p["refine"]
    acc, _ = o.profile()
    J = np.arange(p["buf_lo"] * r, (p["yhi"] - p["ylo"] - p["buf_hi"]) * r)
    u_int = acc[J, 1].sum() / acc[J, 0].sum()
    assert 0.035 < u_int < 0.08, u_int


def test_instantaneous_feedback_is_not_bounded(oracle_lib):
    """The same channel with a window of one LB step leaves the bounds of the
    test above within 1000 LB steps."""
    o = oracle_lib.Oracle(_channel(fb_window=1))
    drho, umax = _excursion(o, 1000, 250)
    assert drho > 0.1 or umax > 0.2, (drho, umax)
