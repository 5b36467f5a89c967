"""Pins of the oracle's Parareal iteration, Eq. (6):
y^{k+1}_{n+1} = G(y^{k+1}_n) + F(y^k_n) - G(y^k_n), and its fixed point
y_{n+1} = F(y_n), Eq. (7)."""
import math

import numpy as np
import pytest

from paper_1705_06149_amd import inputs


def test_dahlquist_closed_form(oracle):
    """For y' = lam y with Euler F and G, f and g are the one-slice
    amplification factors and the iterates have the closed form
    y^k_n = sum_{j<=k} C(n,j) (f-g)^j g^(n-j) y0."""
    lam, T, N, y0 = -1.3, 3.0, 6, 1.0
    nf, nc = 20, 2
    dtf, dtc = T / N / nf, T / N / nc
    f = (1 + lam * dtf) ** nf
    gg = (1 + lam * dtc) ** nc
    F = lambda y, n: y * (1 + lam * dtf) ** nf
    G = lambda y, n: y * (1 + lam * dtc) ** nc
    _, hist = oracle.parareal(y0, N, F, G, n_it=N)
    for rec in hist:
        k = rec["k"] + 1
        for n in range(N + 1):
            closed = sum(math.comb(n, j) * (f - gg) ** j * gg ** (n - j) for j in range(0, min(k, n) + 1)) * y0
            assert rec["Y"][n] == pytest.approx(closed, rel=1e-13, abs=1e-15)


def test_exact_after_k_iterations_navier_stokes(oracle):
    """After k iterations slices 0..k equal the serial fine solution, bit for
    bit; after N iterations every slice does."""
    n, N = 8, 3
    g = oracle.Grid(n, n, n, re=200.0)
    y0 = inputs.rest_state(n, n, n)
    F = lambda y, s: oracle.propagate(g, y, s * 0.004, (s + 1) * 0.004, 2e-3, rtol=1e-11)
    G = lambda y, s: oracle.propagate(g, y, s * 0.004, (s + 1) * 0.004, 4e-3, rtol=1e-11)
    serial = [y0]
    for s in range(N):
        serial.append(F(serial[-1], s))
    jn = lambda a, b: max(float(np.max(np.abs(x - y))) for x, y in zip(a[:3], b[:3]))
    _, hist = oracle.parareal(y0, N, F, G, n_it=N, jump_norm=jn)
    for rec in hist[1:]:
        k = rec["k"] + 1
        for m in range(min(k, N) + 1):
            for a, b in zip(rec["Y"][m], serial[m]):
                assert np.array_equal(a, b), (k, m)
    # the iteration converges: the last jump is far below the first
    assert hist[-1]["jump"] < 1e-3 * hist[1]["jump"]


def test_coarse_equal_fine_converges_in_one_iteration(oracle):
    n, N = 8, 3
    g = oracle.Grid(n, n, n, re=200.0)
    y0 = inputs.rest_state(n, n, n)
    F = lambda y, s: oracle.propagate(g, y, s * 0.004, (s + 1) * 0.004, 2e-3, rtol=1e-11)
    jn = lambda a, b: max(float(np.max(np.abs(x - y))) for x, y in zip(a[:3], b[:3]))
    _, hist = oracle.parareal(y0, N, F, F, n_it=2, jump_norm=jn)
    assert hist[1]["jump"] == 0.0 and hist[2]["jump"] == 0.0


def test_speedup_bound_eq8():
    """Eq. (8): s <= N_p_time / N_it, efficiency <= 1/N_it (reporting helper)."""
    for npt, nit in [(4, 1), (16, 3), (32, 5)]:
        assert npt / nit <= npt and 1.0 / nit <= 1.0
