"""Pins of the oracle's BiCGStab, the paper's pressure solver (Sec. 2):
the closed-form DCT-II solve of the Neumann Laplacian (walls) and the
DCT/DFT solve (periodic z), the bordered dense solve with obstacles, and a
projection step that agrees with the one made with Jacobi-PCG (both solve
the same equation to the same tolerance)."""
import numpy as np
import scipy.fft as sfft

from paper_1705_06149_amd import inputs


def _closed_form(b, h, periodic_z):
    nz, ny, nx = b.shape
    hx, hy, hz = h
    lx = ((4 / hx ** 2) * np.sin(np.pi * np.arange(nx) / (2 * nx)) ** 2)[None, None, :]
    ly = ((4 / hy ** 2) * np.sin(np.pi * np.arange(ny) / (2 * ny)) ** 2)[None, :, None]
    if periodic_z:
        lz = ((4 / hz ** 2) * np.sin(np.pi * np.arange(nz) / nz) ** 2)[:, None, None]
        bh = np.fft.fft(sfft.dctn(b, type=2, norm="ortho", axes=(1, 2)), axis=0)
    else:
        lz = ((4 / hz ** 2) * np.sin(np.pi * np.arange(nz) / (2 * nz)) ** 2)[:, None, None]
        bh = sfft.dctn(b, type=2, norm="ortho")
    lam = lx + ly + lz
    lam[0, 0, 0] = 1.0
    ph = bh / lam
    ph[0, 0, 0] = 0.0
    if periodic_z:
        p = sfft.idctn(np.fft.ifft(ph, axis=0).real, type=2, norm="ortho", axes=(1, 2))
    else:
        p = sfft.idctn(ph, type=2, norm="ortho")
    return p - p.mean()


def test_bicgstab_closed_form(oracle):
    rng = np.random.default_rng(12)
    for periodic in (False, True):
        g = oracle.Grid(14, 11, 9, lx=1.0, ly=0.8, lz=0.6, periodic_z=periodic)
        b = rng.standard_normal((9, 11, 14))
        b -= b.mean()
        p, info = oracle.bicgstab(g, b, rtol=1e-12)
        assert info["status"] == 0 and info["rel_res_true"] <= 2e-12
        ref = _closed_form(b, g.h, periodic)
        assert np.linalg.norm(p - p.mean() - ref) <= 1e-9 * np.linalg.norm(ref)


def test_bicgstab_bordered_dense_with_obstacles(oracle):
    n = 8
    solid = inputs.obstacle_mask(n, 3, frac=0.08, smin=2, smax=3)
    g = oracle.Grid(n, n, n, solid=solid)
    fl = g.fluid()
    rng = np.random.default_rng(2)
    b = rng.standard_normal((n, n, n))
    b[fl] -= b[fl].mean()
    b[~fl] = 0.0
    # dense A on the fluid cells, bordered by the constraint sum(p) = 0
    idx = np.flatnonzero(fl.ravel())
    A = np.zeros((idx.size, idx.size))
    for j, c in enumerate(idx):
        e = np.zeros(n ** 3)
        e[c] = 1.0
        A[:, j] = oracle.apply_A(g, e.reshape(n, n, n)).ravel()[idx]
    K = np.block([[A, np.ones((idx.size, 1))], [np.ones((1, idx.size)), np.zeros((1, 1))]])
    sol = np.linalg.solve(K, np.concatenate([b.ravel()[idx], [0.0]]))[:-1]
    p, info = oracle.bicgstab(g, b, rtol=1e-12)
    assert info["status"] == 0
    got = p.ravel()[idx]
    got -= got.mean()
    assert np.linalg.norm(got - sol) <= 1e-9 * np.linalg.norm(sol)


def test_bicgstab_step_agrees_with_pcg_step(oracle):
    n = 12
    g = oracle.Grid(n, n, n, re=300.0, solid=inputs.obstacle_mask(n, 5, frac=0.05, smin=2, smax=3))
    st = inputs.random_state(n, n, n, seed=6, scale=0.2, pscale=0.0)
    a, ia, _, sa = oracle.fine_steps(g, st, 3, 2e-3, rtol=1e-12, solver=0)
    b, ib, _, sb = oracle.fine_steps(g, st, 3, 2e-3, rtol=1e-12, solver=1)
    assert sa == 0 and sb == 0
    for x, y in zip(a[:3], b[:3]):
        assert np.max(np.abs(x - y)) <= 1e-9 * np.max(np.abs(x))
    # BiCGStab takes two products with A per iteration: fewer iterations
    assert ib.sum() < ia.sum()
