"""Pins of the oracle's projection step (Sec. 2: forward Euler, central
diffusion, SMART convection, Chorin-Temam projection; Sec. 3: lid-driven
cavity, no-slip walls, start from rest).

Hand-derived values at chosen faces pin the image rule at walls and the lid;
structural properties pin the step as a whole.
"""
import numpy as np
import pytest

from paper_1705_06149_amd import inputs


def test_zero_lid_zero_start_stays_zero(oracle):
    g = oracle.Grid(8, 8, 8, lid=np.zeros((8, 9)))
    out, iters, _, st = oracle.fine_steps(g, g.zeros_state(), 3, 1e-3)
    assert st == 0 and all(np.all(a == 0.0) for a in out) and np.all(iters == 0)


def test_linear_shear_is_reproduced_exactly(oracle):
    """u = y (cell-centre heights) with the lid at u = 1 and the bottom at 0:
    tangential images continue the linear profile through both walls, there
    is no transport across x or z away from the side walls, so F = u there."""
    n = 8
    g = oracle.Grid(n, n, n, re=7.0)
    y = (np.arange(n) + 0.5) / n
    u = np.broadcast_to(y[None, :, None], (n, n, n + 1)).copy()
    u[:, :, 0] = u[:, :, -1] = 0.0
    v = np.zeros((n, n + 1, n))
    w = np.zeros((n + 1, n, n))
    Fu, Fv, Fw = oracle.momentum(g, u, v, w, 0.01)
    sel = (slice(1, n - 1), slice(None), slice(3, n - 2))
    assert np.max(np.abs(Fu[sel] - u[sel])) <= 1e-14
    assert np.all(Fv == 0.0) and np.all(Fw == 0.0)


def _smart_hand(U, C, D):
    # the NVD characteristic written out for the hand computations below
    ph = (C - U) / (D - U)
    if 0 < ph < 1 / 6:
        f = 3 * ph
    elif 1 / 6 <= ph < 5 / 6:
        f = 0.75 * ph + 0.375
    elif 5 / 6 <= ph < 1:
        f = 1.0
    else:
        f = ph
    return U + f * (D - U)


def test_normal_wall_reflection_by_hand(oracle):
    """u = sin(pi x) uniform in y, z, lid 0: at the first interior face next
    to the x = 0 wall the stencil sees 0 at the wall face and -u1 beyond it."""
    n, Re, dt = 8, 3.0, 1e-3
    h = 1.0 / n
    g = oracle.Grid(n, n, n, re=Re, lid=np.zeros((n, n + 1)))
    s = np.sin(np.pi * np.arange(n + 1) * h)
    s[0] = s[-1] = 0.0
    u = np.broadcast_to(s[None, None, :], (n, n, n + 1)).copy()
    v = np.zeros((n, n + 1, n))
    w = np.zeros((n + 1, n, n))
    Fu, _, _ = oracle.momentum(g, u, v, w, dt)
    u1, u2 = s[1], s[2]
    lap = (u2 - 2 * u1 + 0.0) / h ** 2
    ap, am = 0.5 * (u1 + u2), 0.5 * (0.0 + u1)
    fp = ap * _smart_hand(0.0, u1, u2)       # upwind triple (face 0, 1, 2)
    fm = am * _smart_hand(-u1, 0.0, u1)      # (odd image, wall face, face 1)
    expect = u1 + dt * (lap / Re - (fp - fm) / h)
    for j in range(1, n - 1):
        for k in range(1, n - 1):
            assert Fu[k, j, 1] == pytest.approx(expect, rel=1e-13)


def test_one_cell_gap_tangential_images(oracle):
    """u in a one-cell-high slot between solid layers: both y-neighbours are
    images 2*0 - u, so the y-diffusion is -4u/h^2 and nothing else acts."""
    n, Re, dt = 10, 5.0, 1e-3
    solid = np.zeros((n, n, n), np.uint8)
    solid[:, 3, 1:n - 1] = 1
    solid[:, 5, 1:n - 1] = 1
    g = oracle.Grid(n, n, n, re=Re, solid=solid, lid=np.zeros((n, n + 1)))
    u = np.zeros((n, n, n + 1))
    u[:, 4, :] = 0.3
    u[:, :, 0] = u[:, :, -1] = 0.0
    v = np.zeros((n, n + 1, n))
    w = np.zeros((n + 1, n, n))
    Fu, _, _ = oracle.momentum(g, u, v, w, dt)
    h = 1.0 / n
    expect = 0.3 + dt * (-4 * 0.3 / h ** 2) / Re
    assert Fu[4, 4, 5] == pytest.approx(expect, rel=1e-13)


def test_projection_identity(oracle):
    """After the correction D u = -dt (b - A p) on fluid cells (up to the
    rounding mean of the right-hand side): the divergence left by the
    projection is the solver's residual."""
    n = 12
    solid = inputs.obstacle_mask(n, seed=4, frac=0.06, smin=2, smax=4)
    g = oracle.Grid(n, n, n, re=300.0, solid=solid)
    u, v, w, _ = inputs.random_state(n, n, n, seed=2, scale=0.5)
    dt = 2e-3
    F = oracle.momentum(g, u, v, w, dt)
    b = oracle.rhs(g, *F, dt)
    p, info = oracle.pcg(g, b, rtol=1e-6)
    un = oracle.correct(g, *F, p, dt)
    div = oracle.divergence(g, *un)
    r = b - oracle.apply_A(g, p)
    fl = g.fluid()
    assert np.max(np.abs(div + dt * r)[fl]) <= 1e-9 * np.max(np.abs(dt * b))
    # the true residual is within the solver's bound (2 rtol after a restart)
    assert np.linalg.norm(div) <= dt * 2e-6 * np.linalg.norm(b)
    assert np.linalg.norm(div) == pytest.approx(dt * info["rel_res_true"] * np.linalg.norm(b), rel=1e-6)


def test_projection_is_an_orthogonal_projector(oracle):
    """The projection of Sec. 2, P F = F - G phi with A phi = -D F (dt = 1),
    on open-face fields: P(P a) = P a, <P a, b> = <a, P b> (every face
    carries the same weight hx hy hz, so the plain sum is the inner
    product), P G q = 0 for any cell field q, and D P a = 0.  The adjoint's
    mu = P lam' relies on the symmetry."""
    rng = np.random.default_rng(12)
    solid = inputs.obstacle_mask(10, seed=6, frac=0.06, smin=2, smax=4)[:8, :9, :10]
    solid = np.ascontiguousarray(solid)
    for sol in (None, solid):
        g = oracle.Grid(10, 9, 8, lx=1.0, ly=0.9, lz=0.7, solid=sol)
        masks = oracle._open_masks(g)
        a = tuple(rng.standard_normal(m.shape) * m for m in masks)
        b = tuple(rng.standard_normal(m.shape) * m for m in masks)
        Pa, _ = oracle.project(g, a, rtol=1e-14)
        Pb, _ = oracle.project(g, b, rtol=1e-14)
        PPa, _ = oracle.project(g, Pa, rtol=1e-14)
        na = np.sqrt(sum(np.sum(x * x) for x in a))
        nb = np.sqrt(sum(np.sum(x * x) for x in b))
        assert max(np.max(np.abs(x - y)) for x, y in zip(PPa, Pa)) <= 1e-11 * na
        lhs = sum(np.sum(x * y) for x, y in zip(Pa, b))
        rhs_ = sum(np.sum(x * y) for x, y in zip(a, Pb))
        assert abs(lhs - rhs_) <= 1e-11 * na * nb
        assert np.max(np.abs(oracle.divergence(g, *Pa))) <= 1e-9 * na / min(g.h)
        q = rng.standard_normal((g.nz, g.ny, g.nx))
        Gq = tuple(x * m for x, m in zip(oracle.gradient(g, q), masks))
        PGq, _ = oracle.project(g, Gq, rtol=1e-14)
        nq = np.sqrt(sum(np.sum(x * x) for x in Gq))
        assert max(np.max(np.abs(x)) for x in PGq) <= 1e-10 * nq


def test_z_mirror_symmetry(oracle):
    """Walls and lid symmetric under z -> Lz - z: u, v, p stay even, w odd."""
    n = 10
    g = oracle.Grid(n, n, n, re=400.0)
    (u, v, w, p), _, _, st = oracle.fine_steps(g, g.zeros_state(), 8, 2e-3, rtol=1e-12)
    s = max(np.abs(u).max(), np.abs(v).max())
    assert np.max(np.abs(u - u[::-1])) <= 1e-12 * s
    assert np.max(np.abs(v - v[::-1])) <= 1e-12 * s
    assert np.max(np.abs(w + w[::-1])) <= 1e-12 * s
    assert np.max(np.abs(p - p[::-1])) <= 1e-10 * np.abs(p).max()


def test_first_order_in_time(oracle):
    """Forward Euler: halving dt at fixed end time halves the error."""
    n, T = 10, 0.016
    g = oracle.Grid(n, n, n, re=100.0)
    sols = []
    for dt in (4e-3, 2e-3, 1e-3, 5e-4):
        (u, v, w, p), _, _, st = oracle.fine_steps(g, g.zeros_state(), int(round(T / dt)), dt, rtol=1e-12)
        sols.append(np.concatenate([u.ravel(), v.ravel(), w.ravel()]))
    e = [np.linalg.norm(sols[i] - sols[i + 1]) for i in range(3)]
    ratios = [e[0] / e[1], e[1] / e[2]]
    assert all(1.7 < r < 2.3 for r in ratios), ratios


def test_closed_faces_written_zero_and_ignored(oracle):
    """Values stored at closed faces never influence the step."""
    n = 9
    solid = np.zeros((n, n, n), np.uint8)
    solid[3:5, 3:6, 2:4] = 1
    g = oracle.Grid(n, n, n, solid=solid)
    st0 = inputs.random_state(n, n, n, seed=1, scale=0.2, pscale=0.0)
    a, _, _, _ = oracle.fine_steps(g, st0, 2, 1e-3)
    # perturb every closed face
    from_open = [x.copy() for x in st0]
    Gu, Gv, Gw = oracle.gradient(g, np.arange(n ** 3, dtype=float).reshape(n, n, n) + 1.0)
    for x, gg in zip(from_open[:3], (Gu, Gv, Gw)):
        x[gg == 0.0] += 123.0
    b, _, _, _ = oracle.fine_steps(g, tuple(from_open), 2, 1e-3)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)


def _layered_state(n, rows, V, solid_rows=()):
    """u = rows[j] on every interior u face of row j (uniform in x and z),
    v = V on every open v face, w = 0; rows listed in solid_rows are solid."""
    u = np.zeros((n, n, n + 1))
    for j, a in enumerate(rows):
        u[:, j, 1:n] = a
    v = np.zeros((n, n + 1, n))
    v[:, 1:n, :] = V
    for j in solid_rows:
        u[:, j, :] = 0.0
        v[:, j:j + 2, :] = 0.0
    return u, v, np.zeros((n + 1, n, n))


def _hand_F(a_m1, a_0, a_p1, a_p2, img_m2, V, h, dt, re):
    """F at a u face with row values a(-1), a(0), a(+1), a(+2) along y and the
    image img_m2 at offset -2, uniform along x and z (so only the y terms
    act), transport V > 0 through both y control-volume faces."""
    lap = (a_p1 - 2 * a_0 + a_m1) / h ** 2
    fp = V * _smart_hand(a_m1, a_0, a_p1)     # upwind triple (f-1, f, f+1)
    fm = V * _smart_hand(img_m2, a_m1, a_0)   # upwind triple (f-2, f-1, f)
    return a_0 + dt * (lap / re - (fp - fm) / h)


def test_tangential_no_slip_image_two_rows_above_the_bottom_wall(oracle):
    """u face one row above the bottom row, flow upward: the upwind triple
    of the lower control-volume face reaches two rows down, behind the
    no-slip wall at y = 0, whose image is 2*0 - u(row 0) (the wall sits
    half a cell below row 0, so row 0 is the mirror)."""
    n, re, dt, V = 8, 10.0, 1e-3, 0.3
    h = 1.0 / n
    rows = [0.2, 0.5, 0.65, 0.7, 0.72, 0.74, 0.76, 0.78]
    g = oracle.Grid(n, n, n, re=re, lid=np.zeros((n, n + 1)))
    Fu, _, _ = oracle.momentum(g, *_layered_state(n, rows, V), dt)
    expect = _hand_F(rows[0], rows[1], rows[2], None, -rows[0], V, h, dt, re)
    assert Fu[4, 1, 4] == pytest.approx(expect, rel=1e-13)
    # the image differs from the one a wall beside row 1 would give
    assert abs(expect - _hand_F(rows[0], rows[1], rows[2], None, -rows[1], V, h, dt, re)) > 1e-6


def test_tangential_no_slip_image_two_rows_above_an_obstacle_top(oracle):
    """The same branch at an obstacle: a solid slab fills row 2; the u face
    of row 4 looks two rows down at the closed row 2, image -u(row 3)."""
    n, re, dt, V = 8, 10.0, 1e-3, 0.3
    h = 1.0 / n
    rows = [0.1, 0.15, 0.0, 0.25, 0.55, 0.6, 0.62, 0.64]
    solid = np.zeros((n, n, n), np.uint8)
    solid[:, 2, :] = 1
    g = oracle.Grid(n, n, n, re=re, solid=solid, lid=np.zeros((n, n + 1)))
    Fu, _, _ = oracle.momentum(g, *_layered_state(n, rows, V, solid_rows=(2,)), dt)
    expect = _hand_F(rows[3], rows[4], rows[5], None, -rows[3], V, h, dt, re)
    assert Fu[4, 4, 4] == pytest.approx(expect, rel=1e-13)
