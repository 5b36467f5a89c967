"""Pins of the oracle's coarser-grid coarse propagator G~ = P(G_c(R(y))) (a
coarse propagator of the kind the paper leaves to future work, Sec. 2.1.2):
the coarse grid has half the cells of the fine one in every direction.

What the definitions fix, checked here without retyping them: R(P(y)) = y
exactly; P(R(y)) = y for fields that are linear along each face normal and
constant across it; R commutes with the divergence (the flux through a coarse
face is the sum of the fluxes through its four fine faces) and P keeps a
divergence-free field divergence-free; both keep the mean pressure; and
Parareal, Eq. (6), with G~ still reproduces the serial fine solution after
N iterations on N slices."""
import numpy as np
import pytest

from paper_1705_06149_amd import inputs


def _pairs(oracle):
    return [
        (oracle.Grid(8, 6, 4, lx=1.2, ly=0.9, lz=0.6), oracle.Grid(4, 3, 2, lx=1.2, ly=0.9, lz=0.6)),
        (oracle.Grid(8, 8, 6, lz=0.5, periodic_z=True), oracle.Grid(4, 4, 3, lz=0.5, periodic_z=True)),
    ]


def _periodic_w(g, st):
    u, v, w, p = st
    if g.periodic_z:
        w = w.copy()
        w[-1] = w[0]
    return u, v, w, p


def test_restrict_of_prolong_is_identity(oracle):
    rng = np.random.default_rng(1)
    for g, gc in _pairs(oracle):
        sc = _periodic_w(gc, tuple(rng.standard_normal(s) for s in gc.shapes()))
        f = oracle.prolong(g, gc, sc)
        assert [a.shape for a in f] == list(g.shapes())
        r = oracle.restrict(g, gc, f)
        for a, b in zip(r, sc):
            assert np.array_equal(a, b)
        if g.periodic_z:
            assert np.array_equal(f[2][-1], f[2][0])


def test_prolong_of_restrict_keeps_piecewise_linear_fields(oracle):
    """u = a(j, k) + b(j, k) * i for i along x, constant over each 2 x 2 block
    of fine faces across the normal (likewise v, w); p constant on coarse
    cells.  R then P must give the field back exactly (values chosen as small
    integers, so every sum is exact)."""
    rng = np.random.default_rng(2)
    for g, gc in _pairs(oracle):
        nx, ny, nz = g.nx, g.ny, g.nz
        a = np.repeat(np.repeat(rng.integers(-8, 8, (gc.nz, gc.ny)), 2, 0), 2, 1).astype(float)
        b = np.repeat(np.repeat(rng.integers(-8, 8, (gc.nz, gc.ny)), 2, 0), 2, 1).astype(float)
        u = a[:, :, None] + b[:, :, None] * np.arange(nx + 1)[None, None, :]
        a = np.repeat(np.repeat(rng.integers(-8, 8, (gc.nz, gc.nx)), 2, 0), 2, 1).astype(float)
        b = np.repeat(np.repeat(rng.integers(-8, 8, (gc.nz, gc.nx)), 2, 0), 2, 1).astype(float)
        v = a[:, None, :] + b[:, None, :] * np.arange(ny + 1)[None, :, None]
        a = np.repeat(np.repeat(rng.integers(-8, 8, (gc.ny, gc.nx)), 2, 0), 2, 1).astype(float)
        b = np.repeat(np.repeat(rng.integers(-8, 8, (gc.ny, gc.nx)), 2, 0), 2, 1).astype(float)
        if g.periodic_z:
            b[:] = 0.0   # a periodic w must repeat its first plane
        w = a[None, :, :] + b[None, :, :] * np.arange(nz + 1)[:, None, None]
        pc = rng.integers(-8, 8, (gc.nz, gc.ny, gc.nx)).astype(float)
        p = np.repeat(np.repeat(np.repeat(pc, 2, 0), 2, 1), 2, 2)
        back = oracle.prolong(g, gc, oracle.restrict(g, gc, (u, v, w, p)))
        for x, y in zip(back, (u, v, w, p)):
            assert np.array_equal(x, y)


def _close_walls(g, st):
    """Zero normal velocity on the wall faces, as every state of the method
    carries (closed faces hold 0)."""
    u, v, w = (a.copy() for a in st[:3])
    u[:, :, 0] = u[:, :, -1] = 0.0
    v[:, 0, :] = v[:, -1, :] = 0.0
    if not g.periodic_z:
        w[0] = w[-1] = 0.0
    return (u, v, w) + tuple(st[3:])


def _restrict_cells(p):
    return 0.125 * sum(p[a::2, b::2, c::2] for a in (0, 1) for b in (0, 1) for c in (0, 1))


def test_restriction_commutes_with_divergence(oracle):
    """div_c(R u) = mean of div_f(u) over the eight fine cells of a coarse
    cell: a coarse face carries the summed flux of its four fine faces."""
    rng = np.random.default_rng(3)
    for g, gc in _pairs(oracle):
        st = _periodic_w(g, tuple(rng.standard_normal(s) for s in g.shapes()))
        dc = oracle.divergence(gc, *oracle.restrict(g, gc, st)[:3])
        df = _restrict_cells(oracle.divergence(g, *st[:3]))
        assert np.max(np.abs(dc - df)) <= 1e-12 * np.max(np.abs(df))


def test_prolongation_keeps_divergence_free(oracle):
    """A coarse field projected to zero divergence stays divergence-free on
    the fine grid after P, and in general (zero normal velocity on the walls)
    div_f(P U) is div_c(U) copied to the eight fine cells."""
    rng = np.random.default_rng(4)
    for g, gc in _pairs(oracle):
        F = _close_walls(gc, _periodic_w(gc, tuple(rng.standard_normal(s) for s in gc.shapes()))[:3])
        dcoarse = oracle.divergence(gc, *F)
        f = oracle.prolong(g, gc, F + (np.zeros(gc.shapes()[3]),))
        dfine = oracle.divergence(g, *f[:3])
        rep = np.repeat(np.repeat(np.repeat(dcoarse, 2, 0), 2, 1), 2, 2)
        assert np.max(np.abs(dfine - rep)) <= 1e-12 * np.max(np.abs(rep))
        U, _ = oracle.project(gc, F, rtol=1e-13)
        f = oracle.prolong(g, gc, tuple(U) + (np.zeros(gc.shapes()[3]),))
        scale = max(np.max(np.abs(a)) for a in U) / min(g.h)
        assert np.max(np.abs(oracle.divergence(g, *f[:3]))) <= 1e-10 * scale


def test_transfers_keep_the_mean_pressure(oracle):
    rng = np.random.default_rng(5)
    for g, gc in _pairs(oracle):
        st = tuple(rng.standard_normal(s) for s in g.shapes())
        pc = oracle.restrict(g, gc, st)[3]
        assert abs(pc.mean() - st[3].mean()) <= 1e-14
        pf = oracle.prolong(g, gc, oracle.restrict(g, gc, st))[3]
        assert abs(pf.mean() - st[3].mean()) <= 1e-14


@pytest.mark.parametrize("periodic", [False, True])
def test_parareal_with_coarse_grid_G_is_exact_after_n_iterations(oracle, periodic):
    nx, N, dt, DT, T = 8, 3, 2e-3, 4e-3, 0.024
    g = oracle.Grid(nx, nx, nx, re=200.0, periodic_z=periodic)
    gc = oracle.Grid(nx // 2, nx // 2, nx // 2, re=200.0, periodic_z=periodic)
    y0 = inputs.random_state(nx, nx, nx, seed=11, scale=0.1, pscale=0.0)
    if periodic:
        y0 = _periodic_w(g, y0)
    L = T / N
    Gt = oracle.coarse_grid_propagator(g, gc, DT, rtol=1e-12)

    def F(y, n):
        return oracle.propagate(g, y, n * L, (n + 1) * L, dt, rtol=1e-12)

    def G(y, n):
        return Gt(y, n * L, (n + 1) * L)

    Y, hist = oracle.parareal(y0, N, F, G)
    assert len(hist) == N + 1
    ys = y0
    for n in range(N):
        ys = F(ys, n)
        for a, b in zip(Y[n + 1], ys):
            assert np.array_equal(a, b), n
    # the first coarse sweep is a fine-grid state that differs from F
    assert hist[0]["Y"][1][0].shape == g.shapes()[0]
    assert np.max(np.abs(hist[0]["Y"][1][0] - F(y0, 0)[0])) > 0


def test_coarse_grid_rules(oracle):
    g = oracle.Grid(8, 8, 8)
    with pytest.raises(ValueError):
        oracle.restrict(g, oracle.Grid(4, 4, 3), g.zeros_state())
    with pytest.raises(ValueError):
        oracle.restrict(g, oracle.Grid(4, 4, 4, lx=2.0), g.zeros_state())
    solid = np.zeros((8, 8, 8), np.uint8)
    solid[3:5, 3:5, 3:5] = 1
    with pytest.raises(NotImplementedError):
        oracle.restrict(oracle.Grid(8, 8, 8, solid=solid), oracle.Grid(4, 4, 4), g.zeros_state())
