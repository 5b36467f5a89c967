"""Pins of the oracle's single-reduction Jacobi-PCG (Chronopoulos & Gear's
rearrangement of CG: one merged inner-product stage per iteration), used for
the projection step's Poisson equation (Sec. 2).

What fixes it without retyping its recurrences:
  - it is the same Krylov method as textbook preconditioned CG, so its first
    iterates equal those of scipy.sparse.linalg.cg with the Jacobi
    preconditioner (a library routine) on the same matrix;
  - its solution equals the closed-form solve (DCT-II on walls; DCT-II in x,
    y and the DFT in z when periodic) and the bordered dense solve with
    obstacles;
  - a projection step with it agrees with the step using plain PCG."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from paper_1705_06149_amd import inputs
from test_oracle_poisson import _dct_solve, _periodic_closed_form


def _dense_A(oracle, g):
    n = g.nx * g.ny * g.nz
    A = np.zeros((n, n))
    for m in range(n):
        e = np.zeros(n)
        e[m] = 1.0
        A[:, m] = oracle.apply_A(g, e.reshape(g.nz, g.ny, g.nx)).ravel()
    return A


@pytest.mark.parametrize("solid", [False, True])
def test_first_iterates_equal_textbook_pcg(oracle, solid):
    nx, ny, nz = 7, 6, 5
    mask = None
    if solid:
        mask = np.zeros((nz, ny, nx), np.uint8)
        mask[1:3, 2:4, 2:5] = 1
    g = oracle.Grid(nx, ny, nz, lx=1.4, ly=0.9, lz=1.1, solid=mask)
    fl = g.fluid().ravel()
    A = _dense_A(oracle, g)[np.ix_(fl, fl)]
    Minv = np.diag(1.0 / np.diag(A))
    rng = np.random.default_rng(31)
    bf = rng.standard_normal(fl.sum())
    bf -= bf.mean()
    iterates = []
    spla.cg(A, bf, x0=np.zeros_like(bf), M=Minv, rtol=1e-30, atol=0.0, maxiter=8,
            callback=lambda xk: iterates.append(xk.copy()))
    assert len(iterates) == 8
    b = np.zeros(nx * ny * nz)
    b[fl] = bf
    b = b.reshape(nz, ny, nx)
    for k, ref in enumerate(iterates, start=1):
        x, info = oracle.pcg_sr(g, b, rtol=1e-30, maxit=k)
        assert info["iters"] == k and info["status"] == 2
        got = x.ravel()[fl]
        ref = ref - ref.mean()
        assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref), k


@pytest.mark.parametrize("shape,L", [((24, 16, 12), (1.5, 1.0, 0.75)), ((9, 13, 11), (1.0, 1.0, 1.0))])
def test_sr_matches_dct_closed_form(oracle, shape, L):
    nx, ny, nz = shape
    g = oracle.Grid(nx, ny, nz, lx=L[0], ly=L[1], lz=L[2])
    rng = np.random.default_rng(32)
    b = rng.standard_normal((nz, ny, nx))
    b -= b.mean()
    p, info = oracle.pcg_sr(g, b, rtol=1e-12)
    ref = _dct_solve(b, g.h)
    assert info["status"] == 0 and info["rel_res_true"] <= 2e-12
    assert np.linalg.norm(p - ref) <= 1e-8 * np.linalg.norm(ref)


def test_sr_matches_periodic_closed_form(oracle):
    g = oracle.Grid(12, 10, 8, lx=1.0, ly=0.8, lz=0.3, periodic_z=True)
    rng = np.random.default_rng(33)
    b = rng.standard_normal((8, 10, 12))
    b -= b.mean()
    p, info = oracle.pcg_sr(g, b, rtol=1e-12)
    ref = _periodic_closed_form(b, g.h)
    assert info["status"] == 0
    assert np.linalg.norm(p - ref) <= 1e-9 * np.linalg.norm(ref)


def test_sr_matches_bordered_dense_solve_with_obstacles(oracle):
    n = 8
    solid = inputs.obstacle_mask(n, seed=5, frac=0.08, smin=2, smax=3)
    g = oracle.Grid(n, n, n, solid=solid)
    fl = g.fluid().ravel()
    A = _dense_A(oracle, g)[np.ix_(fl, fl)]
    m = fl.sum()
    rng = np.random.default_rng(34)
    bf = rng.standard_normal(m)
    bf -= bf.mean()
    K = np.zeros((m + 1, m + 1))
    K[:m, :m] = A
    K[:m, m] = K[m, :m] = 1.0
    sol = np.linalg.solve(K, np.concatenate([bf, [0.0]]))[:m]
    b = np.zeros(n ** 3)
    b[fl] = bf
    p, info = oracle.pcg_sr(g, b.reshape(n, n, n), rtol=1e-11)
    assert info["status"] == 0
    assert np.linalg.norm(p.ravel()[fl] - sol) <= 1e-8 * np.linalg.norm(sol)


def test_sr_cold_start_and_status(oracle):
    g = oracle.Grid(6, 6, 6, periodic_z=True)
    rng = np.random.default_rng(35)
    b = rng.standard_normal((6, 6, 6)) * 1e-13
    b -= b.mean()
    p, info = oracle.pcg_sr(g, b, x0=rng.standard_normal(b.shape) * 30.0, rtol=1e-10)
    assert info["status"] == 0
    assert np.linalg.norm(p - _periodic_closed_form(b, g.h)) <= 1e-8 * np.linalg.norm(p)
    p0, info0 = oracle.pcg_sr(g, np.zeros_like(b), x0=rng.standard_normal(b.shape))
    assert info0["iters"] == 0 and np.all(p0 == 0.0)


def test_sr_projection_step_agrees_with_pcg(oracle):
    n = 12
    solid = inputs.obstacle_mask(n, seed=4, frac=0.06, smin=2, smax=4)
    g = oracle.Grid(n, n, n, re=300.0, solid=solid)
    st = inputs.random_state(n, n, n, seed=2, scale=0.5, pscale=0.0)
    a, ia, _, sa = oracle.fine_steps(g, st, 3, 2e-3, rtol=1e-12)
    b, ib, _, sb = oracle.fine_steps(g, st, 3, 2e-3, rtol=1e-12, solver=2)
    assert sa == 0 and sb == 0
    for x, y in zip(a[:3], b[:3]):
        assert np.max(np.abs(x - y)) <= 1e-10 * np.max(np.abs(x))
    assert abs(int(ia.sum()) - int(ib.sum())) <= 6
