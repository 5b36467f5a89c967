"""Pins of the oracle's mixed-precision Poisson solve with reliable updates
(FP32 Jacobi-PCG on the correction; the FP64 residual replaces the FP32 one
whenever it has fallen by delta, keeping the search direction).

What fixes it: the solution of the projection's Poisson equation (Sec. 2)
is unique up to the gauge, so it must equal the closed-form solves (DCT-II on
walls, DCT/DFT when periodic) and the bordered dense solve with obstacles to
the FP64 tolerance; the FP64 true residual it reports must be the one of the
iterate it returns; status codes at the update and iteration limits; and,
because the search direction survives the updates, its iteration count stays
within a few per cent of FP64 CG from the same warm start where restarting
the FP32 solve at each correction needs far more."""
import numpy as np
import pytest

from paper_1705_06149_amd import inputs
from test_oracle_poisson import _dct_solve, _periodic_closed_form


def test_ru_matches_dct_closed_form(oracle):
    g = oracle.Grid(20, 14, 10, lx=1.0, ly=0.7, lz=0.5)
    rng = np.random.default_rng(41)
    b = rng.standard_normal((10, 14, 20))
    b -= b.mean()
    p, info = oracle.pcg_mixed_ru(g, b, rtol=1e-10, delta=0.01)
    ref = _dct_solve(b, g.h)
    assert info["status"] == 0 and info["rel_res_true"] <= 1e-10
    assert info["outer"] >= 2  # FP32 alone cannot reach 1e-10
    assert np.linalg.norm(p - ref) <= 1e-8 * np.linalg.norm(ref)
    # the reported residual is the returned iterate's
    r = b - oracle.apply_A(g, p)
    assert np.linalg.norm(r) / np.linalg.norm(b) == pytest.approx(info["rel_res_true"], rel=1e-3)


def test_ru_matches_periodic_closed_form(oracle):
    g = oracle.Grid(12, 10, 8, lx=1.0, ly=0.8, lz=0.3, periodic_z=True)
    rng = np.random.default_rng(42)
    b = rng.standard_normal((8, 10, 12))
    b -= b.mean()
    p, info = oracle.pcg_mixed_ru(g, b, rtol=1e-11, delta=0.1)
    assert info["status"] == 0
    ref = _periodic_closed_form(b, g.h)
    assert np.linalg.norm(p - ref) <= 1e-9 * np.linalg.norm(ref)


def test_ru_bordered_dense_solve_with_obstacles(oracle):
    n = 8
    solid = inputs.obstacle_mask(n, seed=5, frac=0.08, smin=2, smax=3)
    g = oracle.Grid(n, n, n, solid=solid)
    fl = g.fluid().ravel()
    A = np.zeros((n ** 3, n ** 3))
    for m in range(n ** 3):
        e = np.zeros(n ** 3)
        e[m] = 1.0
        A[:, m] = oracle.apply_A(g, e.reshape(n, n, n)).ravel()
    A = A[np.ix_(fl, fl)]
    k = fl.sum()
    rng = np.random.default_rng(43)
    bf = rng.standard_normal(k)
    bf -= bf.mean()
    K = np.zeros((k + 1, k + 1))
    K[:k, :k] = A
    K[:k, k] = K[k, :k] = 1.0
    sol = np.linalg.solve(K, np.concatenate([bf, [0.0]]))[:k]
    b = np.zeros(n ** 3)
    b[fl] = bf
    p, info = oracle.pcg_mixed_ru(g, b.reshape(n, n, n), rtol=1e-11, delta=0.01)
    assert info["status"] == 0
    assert np.linalg.norm(p.ravel()[fl] - sol) <= 1e-8 * np.linalg.norm(sol)


def test_ru_keeps_the_krylov_space(oracle):
    """A 48^3 cavity step from a developed warm start: FP64 CG and the
    reliable-update solve take the same number of iterations to 1e-10 (within
    5 %), the restarting defect correction at least 20 % more."""
    n = 48
    g = oracle.Grid(n, n, n, re=1000.0)
    st, _, _, s = oracle.fine_steps(g, g.zeros_state(), 10, 5e-4)
    assert s == 0
    b = oracle.rhs(g, *oracle.momentum(g, *st[:3], 5e-4), 5e-4)
    _, i64 = oracle.pcg(g, b, st[3], rtol=1e-10)
    _, iru = oracle.pcg_mixed_ru(g, b, st[3], rtol=1e-10, delta=0.01)
    _, irs = oracle.pcg_mixed(g, b, st[3], rtol=1e-10, eta=1e-5)
    assert iru["status"] == 0 and iru["rel_res_true"] <= 1e-10
    assert abs(iru["iters"] - i64["iters"]) <= 0.05 * i64["iters"]
    assert irs["iters"] >= 1.2 * i64["iters"]


def test_ru_status_codes_and_cold_start(oracle):
    g = oracle.Grid(10, 10, 10)
    rng = np.random.default_rng(44)
    b = rng.standard_normal((10, 10, 10))
    b -= b.mean()
    _, i1 = oracle.pcg_mixed_ru(g, b, rtol=1e-12, delta=0.01, max_updates=1)
    assert i1["status"] == 2 and i1["outer"] == 1
    _, i2 = oracle.pcg_mixed_ru(g, b, rtol=1e-12, maxit=5)
    assert i2["status"] == 2 and i2["iters"] == 5
    p0, i0 = oracle.pcg_mixed_ru(g, np.zeros_like(b), x0=rng.standard_normal(b.shape))
    assert i0["iters"] == 0 and np.all(p0 == 0.0)
    gp = oracle.Grid(6, 6, 6, periodic_z=True)
    bt = rng.standard_normal((6, 6, 6)) * 1e-13
    bt -= bt.mean()
    p, info = oracle.pcg_mixed_ru(gp, bt, x0=rng.standard_normal(bt.shape) * 30.0, rtol=1e-10)
    assert info["status"] == 0
    ref = _periodic_closed_form(bt, gp.h)
    assert np.linalg.norm(p - ref) <= 1e-8 * np.linalg.norm(ref)


def test_ru_projection_step_agrees_with_fp64(oracle):
    n = 12
    solid = inputs.obstacle_mask(n, seed=4, frac=0.06, smin=2, smax=4)
    g = oracle.Grid(n, n, n, re=300.0, solid=solid)
    st = inputs.random_state(n, n, n, seed=2, scale=0.5, pscale=0.0)
    a, _, _, sa = oracle.fine_steps(g, st, 3, 2e-3, rtol=1e-11)
    b, _, _, sb = oracle.fine_steps(g, st, 3, 2e-3, rtol=1e-11, prec=2, eta=0.01, max_outer=64)
    assert sa == 0 and sb == 0
    num = np.sqrt(sum(np.sum((x - y) ** 2) for x, y in zip(a[:3], b[:3])))
    den = np.sqrt(sum(np.sum(x ** 2) for x in a[:3]))
    assert num <= 1e-9 * den
