"""Pins of the oracle with the domain periodic in z (the boundary condition
of the paper's test runs, Sec. 3): the cell at k = 0 neighbours the cell at
k = nz - 1, the w face at z = Lz is the face at z = 0 (stored twice, equal).

What the mathematics fixes: D = -G^T and A = -D G over the distinct faces,
A symmetric positive semi-definite with a one-dimensional kernel; the
closed-form solve of the Neumann-x/y, periodic-z Laplacian (DCT-II in x and
y, DFT in z); equivariance of a projection step under a shift in z; a
z-uniform state staying z-uniform with w = 0 (the quasi-2D reduction), and
matching the one-plane run."""
import numpy as np
import pytest
import scipy.fft as sfft

from paper_1705_06149_amd import inputs


def _grids(oracle):
    solid = np.zeros((5, 6, 7), np.uint8)
    solid[1:3, 2:4, 2:5] = 1
    solid[0, 1, 5] = solid[4, 1, 5] = 1   # touches the periodic seam
    return [
        oracle.Grid(7, 6, 5, lx=1.4, ly=0.9, lz=1.1, periodic_z=True),
        oracle.Grid(7, 6, 5, lx=1.4, ly=0.9, lz=1.1, solid=solid, periodic_z=True),
    ]


def _distinct_faces(g):
    """Shapes and masks of the distinct faces: the w plane at z = Lz repeats z = 0."""
    su, sv, sw, sp = g.shapes()
    keep_w = np.ones(sw, bool)
    keep_w[-1] = False
    return (su, sv, sw, sp), [np.ones(su, bool), np.ones(sv, bool), keep_w]


def _dense(oracle, g):
    (su, sv, sw, sp), keep = _distinct_faces(g)
    cols = []
    for c, s in enumerate((su, sv, sw)):
        for m in np.flatnonzero(keep[c].ravel()):
            a = [np.zeros(su), np.zeros(sv), np.zeros(sw)]
            a[c].flat[m] = 1.0
            cols.append(oracle.divergence(g, *a).ravel())
    D = np.stack(cols, axis=1)
    nc = int(np.prod(sp))
    G = np.zeros((D.shape[1], nc))
    A = np.zeros((nc, nc))
    for m in range(nc):
        p = np.zeros(sp)
        p.flat[m] = 1.0
        gu, gv, gw = oracle.gradient(g, p)
        # the duplicate plane carries the same gradient as z = 0
        assert np.array_equal(gw[-1], gw[0])
        G[:, m] = np.concatenate([x.ravel()[k.ravel()] for x, k in zip((gu, gv, gw), keep)])
        A[:, m] = oracle.apply_A(g, p).ravel()
    return D, G, A


def test_periodic_div_grad_and_poisson_operator(oracle):
    for g in _grids(oracle):
        D, G, A = _dense(oracle, g)
        assert np.max(np.abs(D + G.T)) <= 1e-12 * np.max(np.abs(D))
        assert np.max(np.abs(A + D @ G)) <= 1e-12 * np.max(np.abs(A))
        assert np.max(np.abs(A - A.T)) <= 1e-12 * np.max(np.abs(A))
        fl = g.fluid().ravel()
        Af = A[np.ix_(fl, fl)]
        ev = np.linalg.eigvalsh(Af)
        assert np.max(np.abs(Af @ np.ones(fl.sum()))) <= 1e-10 * ev[-1]
        assert ev[0] > -1e-9 * ev[-1] and ev[1] > 1e-6 * ev[-1]
        # the seam is a real connection: cell (i,j,0) couples to (i,j,nz-1)
        nx, ny, nz = g.nx, g.ny, g.nz
        a, b = 0, (nz - 1) * ny * nx
        if fl[a] and fl[b]:
            assert A[a, b] == -1.0 / g.h[2] ** 2


def test_periodic_poisson_closed_form(oracle):
    """Neumann in x and y, periodic in z: DCT-II in x, y and the DFT in z
    diagonalise A, with eigenvalues (4/hx^2) sin^2(pi a/2nx) +
    (4/hy^2) sin^2(pi b/2ny) + (4/hz^2) sin^2(pi c/nz)."""
    nx, ny, nz = 12, 10, 8
    g = oracle.Grid(nx, ny, nz, lx=1.0, ly=0.8, lz=0.3, periodic_z=True)
    hx, hy, hz = g.h
    rng = np.random.default_rng(5)
    b = rng.standard_normal((nz, ny, nx))
    b -= b.mean()
    lam = ((4 / hx ** 2) * np.sin(np.pi * np.arange(nx) / (2 * nx)) ** 2)[None, None, :] \
        + ((4 / hy ** 2) * np.sin(np.pi * np.arange(ny) / (2 * ny)) ** 2)[None, :, None] \
        + ((4 / hz ** 2) * np.sin(np.pi * np.arange(nz) / nz) ** 2)[:, None, None]
    bh = np.fft.fft(sfft.dctn(b, type=2, norm="ortho", axes=(1, 2)), axis=0)
    lam[0, 0, 0] = 1.0
    ph = bh / lam
    ph[0, 0, 0] = 0.0
    p_ref = sfft.idctn(np.fft.ifft(ph, axis=0).real, type=2, norm="ortho", axes=(1, 2))
    p_ref -= p_ref.mean()
    p, info = oracle.pcg(g, b, rtol=1e-12)[:2]
    p = p - p.mean()
    assert np.linalg.norm(p - p_ref) <= 1e-9 * np.linalg.norm(p_ref)


def _roll_state(st, m):
    """Shift a state by m cells in z (the duplicate w plane follows plane 0)."""
    u, v, w, p = st
    wc = np.roll(w[:-1], m, axis=0)
    return (np.roll(u, m, axis=0), np.roll(v, m, axis=0), np.concatenate([wc, wc[:1]], axis=0),
            np.roll(p, m, axis=0))


def test_periodic_step_is_shift_equivariant(oracle):
    nx, ny, nz, m = 10, 9, 8, 3
    solid = inputs.obstacle_mask(10, 2, frac=0.06, smin=2, smax=3)[:nz, :ny, :nx]
    solid = np.ascontiguousarray(solid)
    g = oracle.Grid(nx, ny, nz, re=300.0, solid=solid, periodic_z=True)
    gs = oracle.Grid(nx, ny, nz, re=300.0, solid=np.ascontiguousarray(np.roll(solid, m, axis=0)), periodic_z=True)
    st = inputs.random_state(nx, ny, nz, seed=3, scale=0.3, pscale=0.0)
    st = (st[0], st[1], np.concatenate([st[2][:-1], st[2][:1]], axis=0), st[3])
    a, _, _, s1 = oracle.fine_steps(g, st, 3, 2e-3, rtol=1e-12)
    b, _, _, s2 = oracle.fine_steps(gs, _roll_state(st, m), 3, 2e-3, rtol=1e-12)
    assert s1 == 0 and s2 == 0
    b = _roll_state(b, -m)
    for x, y in zip(a[:3], b[:3]):
        assert np.max(np.abs(x - y)) <= 1e-11 * np.max(np.abs(x))
    # the duplicate w plane stays equal to plane 0
    assert np.array_equal(a[2][-1], a[2][0])


def test_periodic_quasi_2d_reduction(oracle):
    """A z-uniform state with w = 0 stays z-uniform (bitwise, every plane sees
    the same values and the same global scalars) with w exactly 0, and
    matches the run on a one-plane periodic grid."""
    nx, ny, lz = 12, 10, 0.1
    rng = np.random.default_rng(8)
    u1 = rng.standard_normal((1, ny, nx + 1)) * 0.2
    v1 = rng.standard_normal((1, ny + 1, nx)) * 0.2
    res = {}
    for nz in (1, 4):
        g = oracle.Grid(nx, ny, nz, lz=lz * nz / 4, re=500.0, periodic_z=True)
        st = (np.repeat(u1, nz, 0), np.repeat(v1, nz, 0), np.zeros((nz + 1, ny, nx)), np.zeros((nz, ny, nx)))
        out, _, _, s = oracle.fine_steps(g, st, 4, 1e-3, rtol=1e-12)
        assert s == 0
        assert np.all(out[2] == 0.0)
        for c in (0, 1, 3):
            assert all(np.array_equal(out[c][k], out[c][0]) for k in range(nz))
        res[nz] = out
    for c in (0, 1):
        assert np.max(np.abs(res[4][c][0] - res[1][c][0])) <= 1e-11 * np.max(np.abs(res[1][c]))


def test_periodic_adjoint_is_refused(oracle):
    g = oracle.Grid(6, 6, 4, periodic_z=True)
    with pytest.raises(NotImplementedError):
        oracle.adjoint_gradient(g, g.zeros_state(), 1, 1e-3)
