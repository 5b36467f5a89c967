"""Degenerate grids on the GPU against the oracle: grids one cell wide in
one or two directions, a single cell, one plane periodic in z, a single
solid cell inside 3^3 and inside a periodic 4 x 3 x 2 box; Poisson solves
and projection steps in FP64 and mixed precision, batches of two different
slices.  Every neighbour of these cells is a wall, a periodic image or an
obstacle, so the image rule and the wrap handle every stencil position."""
import numpy as np
import pytest

from paper_1705_06149_amd import inputs

pytestmark = pytest.mark.gpu

CASES = [((1, 1, 1), False, None), ((1, 5, 3), False, None), ((4, 1, 2), False, None), ((3, 2, 1), False, None),
         ((2, 3, 1), True, None), ((3, 3, 3), False, (1, 1, 1)), ((4, 3, 2), True, (2, 1, 0))]


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def T(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def N(t):
    return t.detach().cpu().numpy()


def _close(got, ref, tol):
    """Relative L2 distance within tol; an all-zero reference must be met exactly."""
    den = np.sqrt(sum(np.sum(r ** 2) for r in ref))
    num = np.sqrt(sum(np.sum((g - r) ** 2) for g, r in zip(got, ref)))
    return num == 0.0 if den == 0.0 else num <= tol * den


def _setup(oracle, shape, periodic, hole):
    nx, ny, nz = shape
    solid = None
    if hole is not None:
        solid = np.zeros((nz, ny, nx), np.uint8)
        solid[hole[2], hole[1], hole[0]] = 1
    g = oracle.Grid(nx, ny, nz, re=50.0, solid=solid, periodic_z=periodic)
    return g, solid


def _state(shape, periodic, seed):
    st = inputs.random_state(*shape, seed=seed, scale=0.3, pscale=0.0)
    if periodic:  # the face at z = Lz is the face at z = 0
        st = (st[0], st[1], np.concatenate([st[2][:-1], st[2][:1]], axis=0), st[3])
    return st


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape,periodic,hole", CASES)
def test_degenerate_grid_parity(gpu, oracle, shape, periodic, hole, prec):
    nx, ny, nz = shape
    _say("degenerate grid", shape, "periodic" if periodic else "walls", "hole", hole, "prec", prec)
    g, solid = _setup(oracle, shape, periodic, hole)
    fluid = g.fluid()
    h = gpu.Handle(nx, ny, nz, re=50.0, solid=solid, periodic_z=periodic, max_batch=2)
    # Poisson: two mean-free right-hand sides
    rng = np.random.default_rng(7)
    bs = []
    for _ in range(2):
        b = rng.standard_normal((nz, ny, nx))
        b[~fluid] = 0.0
        b[fluid] -= b[fluid].mean()
        bs.append(b)
    pt = T(np.zeros((2, nz, ny, nx)))
    info = h.poisson_solve(T(np.stack(bs)), pt, gpu.PoissonOpts(rtol=1e-12, prec=prec))
    for i in range(2):
        ref, oinfo = oracle.pcg(g, bs[i], rtol=1e-12) if prec == 0 else oracle.pcg_mixed(g, bs[i], rtol=1e-12)
        assert oinfo["status"] == 0 and info[i]["status"] == 0
        _say("  poisson slice", i, "iters gpu", info[i]["iters"], "oracle", oinfo["iters"])
        assert _close([N(pt)[i]], [ref], 1e-9)
    # projection steps from two different random states
    sts = [_state(shape, periodic, seed) for seed in (3, 4)]
    y = tuple(T(np.stack([s[c] for s in sts])) for c in range(4))
    h.fine_step(y, 0.0, 0.003, 1e-3, gpu.PoissonOpts(rtol=1e-11, prec=prec))
    for i, st in enumerate(sts):
        ref, _, _, s = oracle.fine_steps(g, st, 3, 1e-3, prec=prec, rtol=1e-11)
        assert s == 0
        assert _close([N(a)[i] for a in y[:3]], ref[:3], 1e-10 if prec == 0 else 1e-8), i
    h.close()


@pytest.mark.parametrize("prec,solver", [(0, 0), (1, 0), (0, 1)])
def test_cold_start_on_rounding_level_rhs(gpu, oracle, prec, solver):
    """A warm start worse than none is dropped (p = 0) before the solve, as in
    the oracle.  A 1 x 1 x 4 column periodic in z is uniform along z after one
    step, so every later right-hand side is rounding noise while the
    warm-started pressure is not; and a Poisson solve with b ~ 1e-13 from a
    warm start of order 30 on a periodic 6^3 box.  Both converge, as the
    oracle does, and match it."""
    _say("cold start, prec", prec, "solver", solver)
    opts = gpu.PoissonOpts(rtol=1e-10, prec=prec, solver=solver)
    g = oracle.Grid(1, 1, 4, lx=0.25, ly=0.25, re=100.0, periodic_z=True)
    st = _state((1, 1, 4), True, 3)
    h = gpu.Handle(1, 1, 4, lx=0.25, ly=0.25, re=100.0, periodic_z=True, max_batch=1)
    y = tuple(T(a[None]) for a in st)
    info = h.fine_step(y, 0.0, 0.004, 1e-3, opts)
    ref, _, _, s = oracle.fine_steps(g, st, 4, 1e-3, prec=prec, solver=solver, rtol=1e-10)
    assert s == 0 and info[0]["status"] == 0
    assert _close([N(a)[0] for a in y[:3]], ref[:3], 1e-10 if prec == 0 else 1e-8)
    h.close()
    g6 = oracle.Grid(6, 6, 6, periodic_z=True)
    rng = np.random.default_rng(21)
    b = rng.standard_normal((6, 6, 6)) * 1e-13
    b -= b.mean()
    x0 = rng.standard_normal((6, 6, 6)) * 30.0
    solve = oracle.bicgstab if solver == 1 else (oracle.pcg_mixed if prec == 1 else oracle.pcg)
    ref, oinfo = solve(g6, b, x0=x0, rtol=1e-10)
    h6 = gpu.Handle(6, 6, 6, periodic_z=True, max_batch=1)
    pt = T(x0[None])
    info = h6.poisson_solve(T(b[None]), pt, opts)
    assert oinfo["status"] == 0 and info[0]["status"] == 0
    assert _close([N(pt)[0]], [ref], 1e-8)
    h6.close()
