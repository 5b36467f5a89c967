"""Pins of the oracle's pressure Poisson solves (the projection step's
Poisson equation, Sec. 2; Jacobi-preconditioned CG in FP64 and the
FP32-inner / FP64-outer defect correction).

- closed form: the cell-centred Neumann Laplacian on a box is diagonalised
  by the type-II DCT (scipy.fft.dctn), any grid size and aspect;
- manufactured solution: second-order convergence;
- brute force: bordered dense solve [A 1; 1^T 0] with obstacles on 8^3.
"""
import numpy as np
import pytest
from scipy import fft

from paper_1705_06149_amd import inputs


def _dct_solve(b, h):
    nz, ny, nx = b.shape
    lam = (4 / h[0] ** 2 * np.sin(np.pi * np.arange(nx) / (2 * nx)) ** 2)[None, None, :] \
        + (4 / h[1] ** 2 * np.sin(np.pi * np.arange(ny) / (2 * ny)) ** 2)[None, :, None] \
        + (4 / h[2] ** 2 * np.sin(np.pi * np.arange(nz) / (2 * nz)) ** 2)[:, None, None]
    bh = fft.dctn(b, type=2, norm="ortho")
    lam[0, 0, 0] = 1.0
    ph = bh / lam
    ph[0, 0, 0] = 0.0
    return fft.idctn(ph, type=2, norm="ortho")


@pytest.mark.parametrize("shape,L", [((24, 16, 12), (1.5, 1.0, 0.75)), ((9, 13, 11), (1.0, 1.0, 1.0))])
def test_pcg_matches_dct_closed_form(oracle, shape, L):
    nx, ny, nz = shape
    g = oracle.Grid(nx, ny, nz, lx=L[0], ly=L[1], lz=L[2])
    rng = np.random.default_rng(7)
    b = rng.standard_normal((nz, ny, nx))
    b -= b.mean()
    p, info = oracle.pcg(g, b, rtol=1e-12)
    ref = _dct_solve(b, g.h)
    assert info["status"] == 0 and info["rel_res_true"] <= 2e-12
    assert np.linalg.norm(p - ref) / np.linalg.norm(ref) <= 1e-8
    assert abs(p.mean()) <= 1e-13 * np.abs(ref).max()


def test_mixed_matches_dct_closed_form(oracle):
    g = oracle.Grid(20, 14, 10, lx=1.0, ly=0.7, lz=0.5)
    rng = np.random.default_rng(8)
    b = rng.standard_normal((10, 14, 20))
    b -= b.mean()
    p, info = oracle.pcg_mixed(g, b, rtol=1e-10, eta=1e-5)
    ref = _dct_solve(b, g.h)
    assert info["status"] == 0 and info["rel_res_true"] <= 1e-10
    assert info["outer"] >= 2  # FP32 alone cannot reach 1e-10
    assert np.linalg.norm(p - ref) / np.linalg.norm(ref) <= 1e-8


def test_second_order_on_manufactured_solution(oracle):
    """p = cos(pi x) cos(pi y) cos(pi z) with -Lap p = 3 pi^2 p.  Sampled at
    cell centres p is a discrete eigenvector (eigenvalue lam_h), so the
    discrete solution is exactly (3 pi^2 / lam_h) p; its error converges at
    order 2."""
    errs = []
    for n in (16, 32, 64):
        g = oracle.Grid(n, n, n)
        h = 1.0 / n
        c = np.cos(np.pi * (np.arange(n) + 0.5) / n)
        pe = c[:, None, None] * c[None, :, None] * c[None, None, :]
        p, info = oracle.pcg(g, 3 * np.pi ** 2 * pe, rtol=1e-13)
        lam_h = 3 * (4 / h ** 2) * np.sin(np.pi * h / 2) ** 2
        assert np.max(np.abs(p - (3 * np.pi ** 2 / lam_h) * pe)) <= 1e-10 * np.max(np.abs(pe))
        errs.append(np.max(np.abs(p - pe)))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(o - 2.0) < 0.02 for o in orders), orders


def test_bordered_dense_solve_with_obstacles(oracle):
    n = 8
    solid = inputs.obstacle_mask(n, seed=12, frac=0.1, smin=2, smax=3)
    g = oracle.Grid(n, n, n, solid=solid)
    fl = g.fluid().ravel()
    nc = n ** 3
    A = np.zeros((nc, nc))
    for m in range(nc):
        e = np.zeros(nc)
        e[m] = 1.0
        A[:, m] = oracle.apply_A(g, e.reshape(n, n, n)).ravel()
    Af = A[np.ix_(fl, fl)]
    nf = fl.sum()
    rng = np.random.default_rng(9)
    bf = rng.standard_normal(nf)
    bf -= bf.mean()
    K = np.zeros((nf + 1, nf + 1))
    K[:nf, :nf] = Af
    K[:nf, nf] = 1.0
    K[nf, :nf] = 1.0
    sol = np.linalg.solve(K, np.concatenate([bf, [0.0]]))[:nf]
    b = np.zeros(nc)
    b[fl] = bf
    p, info = oracle.pcg(g, b.reshape(n, n, n), rtol=1e-12)
    assert info["status"] == 0
    assert np.linalg.norm(p.ravel()[fl] - sol) / np.linalg.norm(sol) <= 1e-8
    pm, im = oracle.pcg_mixed(g, b.reshape(n, n, n), rtol=1e-11)
    assert np.linalg.norm(pm.ravel()[fl] - sol) / np.linalg.norm(sol) <= 1e-8


def test_warm_start_and_status_codes(oracle):
    g = oracle.Grid(10, 10, 10)
    rng = np.random.default_rng(10)
    b = rng.standard_normal((10, 10, 10))
    b -= b.mean()
    p, info = oracle.pcg(g, b, rtol=1e-11)
    # exact warm start: no iteration
    p2, info2 = oracle.pcg(g, b, x0=p, rtol=1e-10)
    assert info2["iters"] == 0 and info2["status"] == 0
    # iteration limit: NOT_CONVERGED, iterate still written
    p3, info3 = oracle.pcg(g, b, rtol=1e-12, maxit=3)
    assert info3["status"] == 2 and info3["iters"] == 3 and np.abs(p3).max() > 0
    p4, info4 = oracle.pcg_mixed(g, b, rtol=1e-12, max_outer=1)
    assert info4["status"] == 2 and info4["outer"] == 1
    # zero right-hand side: p = 0
    p5, info5 = oracle.pcg(g, np.zeros_like(b), x0=rng.standard_normal(b.shape))
    assert info5["iters"] == 0 and np.all(p5 == 0.0)
    # non-finite input
    bn = b.copy()
    bn[2, 2, 2] = np.nan
    _, info6 = oracle.pcg(g, bn)
    assert info6["status"] == 3


def _periodic_closed_form(b, h):
    """Neumann in x, y and periodic in z: DCT-II in x, y and the DFT in z
    diagonalise A; the mean-free solution of A p = b."""
    nz, ny, nx = b.shape
    lam = ((4 / h[0] ** 2) * np.sin(np.pi * np.arange(nx) / (2 * nx)) ** 2)[None, None, :] \
        + ((4 / h[1] ** 2) * np.sin(np.pi * np.arange(ny) / (2 * ny)) ** 2)[None, :, None] \
        + ((4 / h[2] ** 2) * np.sin(np.pi * np.arange(nz) / nz) ** 2)[:, None, None]
    bh = np.fft.fft(fft.dctn(b, type=2, norm="ortho", axes=(1, 2)), axis=0)
    lam[0, 0, 0] = 1.0
    ph = bh / lam
    ph[0, 0, 0] = 0.0
    p = fft.idctn(np.fft.ifft(ph, axis=0).real, type=2, norm="ortho", axes=(1, 2))
    return p - p.mean()


@pytest.mark.parametrize("solver", ["pcg", "pcg_mixed", "bicgstab"])
def test_cold_start_on_rounding_level_rhs(oracle, solver):
    """A right-hand side at the rounding level (as after a step that left the
    flow uniform along periodic z) with a warm start of order 30: the warm
    start is worse than none (||b - A x0|| > ||b||), so the solve starts from
    x0 = 0 and converges to the closed-form solution.  Iterating from the
    warm start instead cannot meet ||r|| <= rtol ||b|| and breaks down."""
    g = oracle.Grid(6, 6, 6, periodic_z=True)
    rng = np.random.default_rng(21)
    b = rng.standard_normal((6, 6, 6)) * 1e-13
    b -= b.mean()
    x0 = rng.standard_normal((6, 6, 6)) * 30.0
    p, info = getattr(oracle, solver)(g, b, x0=x0, rtol=1e-10)
    ref = _periodic_closed_form(b, g.h)
    assert info["status"] == 0, info
    assert np.linalg.norm(p - ref) <= 1e-8 * np.linalg.norm(ref)


def test_cold_start_keeps_a_good_warm_start(oracle):
    """The rule fires only when the warm start is worse than none: a warm
    start near the solution is kept and saves iterations."""
    g = oracle.Grid(10, 10, 10)
    rng = np.random.default_rng(22)
    b = rng.standard_normal((10, 10, 10))
    b -= b.mean()
    ref = _dct_solve(b, g.h)
    _, cold = oracle.pcg(g, b, rtol=1e-10)
    near = ref + 1e-3 * np.abs(ref).max() * rng.standard_normal(b.shape)
    p, warm = oracle.pcg(g, b, x0=near, rtol=1e-10)
    assert warm["status"] == 0 and warm["iters"] < cold["iters"]
    assert np.linalg.norm(p - ref) <= 1e-8 * np.linalg.norm(ref)


def test_periodic_column_decays_in_closed_form(oracle):
    """A 1 x 1 x 4 column periodic in z: u and v sit on walls (zero), the
    projection leaves w uniform along z, and then each step multiplies it
    by 1 - 4 dt (1/hx^2 + 1/hy^2)/Re (no-slip images on the four side walls;
    a uniform w has equal fluxes through every z face).  From the second
    step on the right-hand side is rounding noise while the warm-started
    pressure is not: every step must still converge."""
    re, dt = 100.0, 1e-3
    g = oracle.Grid(1, 1, 4, lx=0.25, ly=0.25, lz=1.0, re=re, periodic_z=True)
    st = inputs.random_state(1, 1, 4, seed=3, scale=0.5, pscale=0.0)
    st = (st[0], st[1], np.concatenate([st[2][:-1], st[2][:1]], axis=0), st[3])
    hx, hy, _ = g.h
    fac = 1.0 - 4.0 * dt * (1.0 / hx ** 2 + 1.0 / hy ** 2) / re
    y1, _, _, s1 = oracle.fine_steps(g, st, 1, dt)
    y4, iters, rel, s4 = oracle.fine_steps(g, y1, 3, dt)
    assert s1 == 0 and s4 == 0
    assert np.all(y4[0] == 0.0) and np.all(y4[1] == 0.0)
    c1 = y1[2].mean()
    assert np.max(np.abs(y4[2] - c1 * fac ** 3)) <= 1e-9 * abs(c1)
    assert np.all(np.isfinite(y4[3]))
