"""Pins of the oracle's staggered-grid operators (Sec. 2: central
differences for the pressure gradient on a uniform staggered mesh, and the
projection's Poisson operator).

Dense matrices are assembled by applying the oracle's divergence, gradient
and Poisson operator to unit vectors on tiny grids, then checked against
what the mathematics fixes: D = -G^T, A = -D G, A symmetric positive
semi-definite with the constants as its kernel on a connected fluid region,
and the closed-form cosine eigenmode of the cell-centred Neumann Laplacian.
"""
import numpy as np
import pytest

from paper_1705_06149_amd import inputs


def _grids(oracle):
    rng = np.random.default_rng(4)
    solid = np.zeros((5, 6, 7), np.uint8)
    solid[1:3, 2:4, 2:5] = 1
    solid[3, 1, 5] = 1
    return [
        oracle.Grid(7, 6, 5, lx=1.4, ly=0.9, lz=1.1),
        oracle.Grid(7, 6, 5, lx=1.4, ly=0.9, lz=1.1, solid=solid),
    ]


def _dense(oracle, g):
    su, sv, sw, sp = g.shapes()
    nf = [int(np.prod(s)) for s in (su, sv, sw)]
    nc = int(np.prod(sp))
    D = np.zeros((nc, sum(nf)))
    col = 0
    for c, s in enumerate((su, sv, sw)):
        for m in range(nf[c]):
            a = [np.zeros(su), np.zeros(sv), np.zeros(sw)]
            a[c].flat[m] = 1.0
            D[:, col] = oracle.divergence(g, *a).ravel()
            col += 1
    G = np.zeros((sum(nf), nc))
    A = np.zeros((nc, nc))
    for m in range(nc):
        p = np.zeros(sp)
        p.flat[m] = 1.0
        G[:, m] = np.concatenate([x.ravel() for x in oracle.gradient(g, p)])
        A[:, m] = oracle.apply_A(g, p).ravel()
    return D, G, A


def test_divergence_is_minus_gradient_transpose(oracle):
    for g in _grids(oracle):
        D, G, A = _dense(oracle, g)
        assert np.array_equal(D, -G.T) or np.max(np.abs(D + G.T)) <= 1e-12 * np.max(np.abs(D))


def test_poisson_operator_is_minus_div_grad(oracle):
    for g in _grids(oracle):
        D, G, A = _dense(oracle, g)
        assert np.max(np.abs(A + D @ G)) <= 1e-12 * np.max(np.abs(A))
        assert np.max(np.abs(A - A.T)) <= 1e-12 * np.max(np.abs(A))
        fl = g.fluid().ravel()
        Af = A[np.ix_(fl, fl)]
        ones = np.ones(fl.sum())
        assert np.max(np.abs(Af @ ones)) <= 1e-10 * np.max(np.abs(A))
        ev = np.linalg.eigvalsh(Af)
        assert ev[0] > -1e-9 * ev[-1]
        # connected fluid: the kernel is one-dimensional
        assert ev[1] > 1e-6 * ev[-1]
        # solid cells are decoupled and zero
        assert np.all(A[~fl] == 0.0) and np.all(A[:, ~fl] == 0.0)


def test_neumann_cosine_eigenmode(oracle):
    """cos(a pi x/Lx) cos(b pi y/Ly) cos(c pi z/Lz) sampled at cell centres is an
    exact eigenvector of the cell-centred Neumann Laplacian, with eigenvalue
    sum_d (4/h_d^2) sin^2(a_d pi/(2 n_d))."""
    g = oracle.Grid(12, 10, 9, lx=1.5, ly=1.0, lz=0.7)
    hx, hy, hz = g.h
    x = (np.arange(12) + 0.5) * hx
    y = (np.arange(10) + 0.5) * hy
    z = (np.arange(9) + 0.5) * hz
    for a, b, c in [(1, 1, 1), (2, 3, 1), (0, 1, 4)]:
        p = (np.cos(a * np.pi * z / g.lz)[:, None, None] * np.cos(b * np.pi * y / g.ly)[None, :, None]
             * np.cos(c * np.pi * x / g.lx)[None, None, :])
        lam = (4 / hx ** 2 * np.sin(c * np.pi / 24) ** 2 + 4 / hy ** 2 * np.sin(b * np.pi / 20) ** 2
               + 4 / hz ** 2 * np.sin(a * np.pi / 18) ** 2)
        Ap = oracle.apply_A(g, p)
        assert np.max(np.abs(Ap - lam * p)) <= 1e-11 * lam * np.max(np.abs(p))


def test_gradient_of_linear_field(oracle):
    g = oracle.Grid(6, 5, 7, lx=1.2, ly=0.8, lz=1.4)
    hx, hy, hz = g.h
    x = (np.arange(6) + 0.5) * hx
    y = (np.arange(5) + 0.5) * hy
    z = (np.arange(7) + 0.5) * hz
    p = 2.0 * x[None, None, :] - 3.0 * y[None, :, None] + 0.5 * z[:, None, None]
    Gu, Gv, Gw = oracle.gradient(g, p)
    assert np.allclose(Gu[:, :, 1:-1], 2.0, rtol=1e-12) and np.all(Gu[:, :, [0, -1]] == 0.0)
    assert np.allclose(Gv[:, 1:-1, :], -3.0, rtol=1e-12) and np.all(Gv[:, [0, -1], :] == 0.0)
    assert np.allclose(Gw[1:-1], 0.5, rtol=1e-12) and np.all(Gw[[0, -1]] == 0.0)


def test_divergence_telescopes_to_zero(oracle):
    """Divergence theorem: with every boundary and obstacle face closed, the
    divergence summed over the fluid cells vanishes for any face field."""
    solid = inputs.obstacle_mask(12, seed=3, frac=0.1, smin=2, smax=4)
    g = oracle.Grid(12, 12, 12, solid=solid)
    u, v, w, _ = inputs.random_state(12, 12, 12, seed=5)
    d = oracle.divergence(g, u, v, w)
    assert abs(d[g.fluid()].sum()) <= 1e-11 * np.abs(d).sum()
    assert np.all(d[~g.fluid()] == 0.0)
