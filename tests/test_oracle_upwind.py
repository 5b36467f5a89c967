"""Pins of the oracle's donor-cell (first-order upwind) convection, a coarse
propagator variant: the paper's G takes the fine scheme with a larger step
and leaves other coarse propagators to future work (Sec. 2.1.2).

What fixes it: the convective face value is the value at the node on the
face's upwind side (the C of the SMART triple), checked by hand for transport
in both directions; with a divergence-free transport field and a Courant
number below 1/2 the predictor is a convex combination of old values, so it
stays within their bounds; and Parareal with the donor-cell G still
reproduces the serial fine solution after N iterations on N slices."""
import numpy as np
import pytest

from paper_1705_06149_amd import inputs


def _rows_state(n, rows, V):
    u = np.zeros((n, n, n + 1))
    for j, a in enumerate(rows):
        u[:, j, 1:n] = a
    v = np.zeros((n, n + 1, n))
    v[:, 1:n, :] = V
    return u, v, np.zeros((n + 1, n, n))


@pytest.mark.parametrize("V", [0.4, -0.4])
def test_donor_cell_face_value_by_hand(oracle, V):
    """u uniform along x and z, varying along y; v = V on every open face.
    At an interior u face the x and z fluxes cancel and diffusion acts along
    y only; the y faces carry the upwind node's value."""
    n, re, dt = 10, 20.0, 1e-3
    h = 1.0 / n
    rows = [0.05 + 0.09 * j + 0.004 * j * j for j in range(n)]  # smooth: SMART takes its QUICK segment
    g = oracle.Grid(n, n, n, re=re, lid=np.zeros((n, n + 1)), upwind=True)
    Fu, _, _ = oracle.momentum(g, *_rows_state(n, rows, V), dt)
    j = 4
    a_m, a_0, a_p = rows[j - 1], rows[j], rows[j + 1]
    lap = (a_p - 2 * a_0 + a_m) / h ** 2
    fp = V * (a_0 if V > 0 else a_p)
    fm = V * (a_m if V > 0 else a_0)
    expect = a_0 + dt * (lap / re - (fp - fm) / h)
    assert Fu[5, j, 5] == pytest.approx(expect, rel=1e-13)
    # SMART takes other face values here
    gs = oracle.Grid(n, n, n, re=re, lid=np.zeros((n, n + 1)))
    Fs, _, _ = oracle.momentum(gs, *_rows_state(n, rows, V), dt)
    assert abs(Fs[5, j, 5] - expect) > 1e-7


def test_donor_cell_predictor_is_bounded(oracle):
    """A divergence-free transport field (a projected random field), Courant
    number <= 0.5 and negligible diffusion: the donor-cell predictor is a
    convex combination of neighbouring values, so on faces whose stencil
    meets no wall it stays within the old field's bounds."""
    n = 12
    g = oracle.Grid(n, n, n, re=1e9, lid=np.zeros((n, n + 1)), upwind=True)
    rng = np.random.default_rng(51)
    masks = oracle._open_masks(g)
    a = tuple(rng.standard_normal(m.shape) * m for m in masks)
    P, _ = oracle.project(g, a, rtol=1e-14)
    scale = max(np.abs(x).max() for x in P)
    P = tuple(x / scale for x in P)
    h = 1.0 / n
    dt = 0.5 * h / 3.0
    F = oracle.momentum(g, *P, dt)
    for c in range(3):
        inner = [slice(2, -2)] * 3
        got = F[c][tuple(inner)]
        lo, hi = P[c].min(), P[c].max()
        assert got.min() >= lo - 1e-12 and got.max() <= hi + 1e-12, c


def test_parareal_with_donor_cell_coarse_propagator_is_exact(oracle):
    n, N, dt, DT, T = 8, 3, 1e-3, 3e-3, 0.009
    fine = oracle.Grid(n, n, n, re=200.0)
    coarse = oracle.Grid(n, n, n, re=200.0, upwind=True)
    y0 = inputs.random_state(n, n, n, seed=8, scale=0.2, pscale=0.0)
    F = lambda y, k: oracle.propagate(fine, y, k * T / N, (k + 1) * T / N, dt, rtol=1e-12)
    G = lambda y, k: oracle.propagate(coarse, y, k * T / N, (k + 1) * T / N, DT, rtol=1e-12)
    Y, hist = oracle.parareal(y0, N, F, G)
    ys = y0
    for m in range(1, N + 1):
        ys = F(ys, m - 1)
        for c in range(4):
            assert np.array_equal(Y[m][c], ys[c]), (m, c)
    # the coarse propagator differs from the fine one with the same step
    gs = oracle.propagate(oracle.Grid(n, n, n, re=200.0), y0, 0.0, T / N, DT, rtol=1e-12)
    gu = G(y0, 0)
    assert max(np.abs(x - y).max() for x, y in zip(gs[:3], gu[:3])) > 1e-8
