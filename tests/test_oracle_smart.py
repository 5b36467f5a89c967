"""Pins of the oracle's SMART face value (Gaskell & Lau normalised-variable
diagram: the convective scheme the paper names in Sec. 2 as a bounded
QUICK).  Expected values come from the published NVD characteristic and
from QUICK's quadratic interpolation, not from the oracle."""
import numpy as np
import pytest


@pytest.mark.parametrize("phat,expect", [
    (0.0, 0.0),          # lower end of the bounded region
    (1.0 / 12, 0.25),    # steep segment, slope 3
    (1.0 / 6, 0.5),      # first breakpoint
    (0.5, 0.75),         # QUICK segment 3/4 phat + 3/8
    (0.7, 0.9),
    (5.0 / 6, 1.0),      # second breakpoint
    (0.9, 1.0),          # capped
    (1.0, 1.0),
    (-0.5, -0.5),        # outside [0,1]: first-order upwind
    (1.5, 1.5),
])
def test_nvd_values(oracle, phat, expect):
    # U = 0, D = 1 makes the normalised variable equal to C
    assert oracle.smart(0.0, phat, 1.0) == pytest.approx(expect, abs=1e-15)


def test_continuous_at_breakpoints(oracle):
    for b in (0.0, 1.0 / 6, 5.0 / 6, 1.0):
        lo = oracle.smart(0.0, b - 1e-12, 1.0)
        hi = oracle.smart(0.0, b + 1e-12, 1.0)
        assert abs(lo - hi) < 1e-10


def test_quick_segment_is_quadratic_interpolation(oracle):
    """Inside the QUICK segment SMART equals the quadratic through U, C, D
    (at positions -1, 0, 1) evaluated at the face position 1/2."""
    rng = np.random.default_rng(1)
    n = 0
    while n < 200:
        U, C, D = rng.standard_normal(3)
        phat = (C - U) / (D - U)
        if not (1.0 / 6 + 1e-6 < phat < 5.0 / 6 - 1e-6):
            continue
        coef = np.polyfit([-1.0, 0.0, 1.0], [U, C, D], 2)
        assert oracle.smart(U, C, D) == pytest.approx(np.polyval(coef, 0.5), rel=1e-12, abs=1e-12)
        n += 1


def test_boundedness_and_affine_invariance(oracle):
    rng = np.random.default_rng(2)
    for _ in range(500):
        U, C, D = rng.standard_normal(3)
        f = oracle.smart(U, C, D)
        phat = (C - U) / (D - U)
        if 0.0 <= phat <= 1.0:
            # bounded: the face value lies between C and D
            assert min(C, D) - 1e-12 <= f <= max(C, D) + 1e-12
        else:
            assert f == pytest.approx(C, rel=1e-12, abs=1e-12)
        a, s = rng.standard_normal(), rng.standard_normal()
        g = oracle.smart(a + s * U, a + s * C, a + s * D)
        assert g == pytest.approx(a + s * f, rel=1e-9, abs=1e-9)


def test_tie_gives_central_value(oracle):
    assert oracle.smart(2.0, 5.0, 2.0) == 5.0
