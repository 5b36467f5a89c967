"""Pins of the oracle's free-slip obstacle walls (slip boundaries are an
extension the paper leaves open; its obstacles are no-slip, Sec. 3).

Free slip on an obstacle face means zero normal velocity and zero tangential
stress.  What that fixes, checked here without retyping the image rule:
  * mirror equivalence: a cavity whose left columns are a free-slip obstacle
    evolves exactly like the right half of the mirror-doubled cavity without
    the obstacle (normal velocity odd, tangential velocity and pressure even
    about the obstacle face);
  * plug flow along a periodic channel walled by free-slip obstacles stays
    exactly uniform (no stress anywhere), and decays near no-slip walls;
  * the domain walls and the lid are not obstacles: without obstacles the
    flag changes nothing.
"""
import numpy as np
import pytest

from paper_1705_06149_amd import inputs


def _mirror_pair(oracle, periodic, slip=True):
    """A: 8 x 6 x 4 cells, columns i = 0, 1 solid; B: 12 x 6 x 4 cells, no
    obstacle, mirrored about x = 6 h (B cell i >= 6 is A cell i - 4)."""
    h = 0.125
    ny, nz = 6, 4
    solid = np.zeros((nz, ny, 8), np.uint8)
    solid[:, :, :2] = 1
    kw = dict(ly=ny * h, lz=nz * h, re=50.0, periodic_z=periodic)
    A = oracle.Grid(8, ny, nz, lx=8 * h, solid=solid, slip_obstacles=slip, lid=np.zeros((nz, 9)), **kw)
    B = oracle.Grid(12, ny, nz, lx=12 * h, lid=np.zeros((nz, 13)), **kw)
    return A, B


def _a_state(A, seed):
    rng = np.random.default_rng(seed)
    u, v, w, p = (rng.standard_normal(s) * 0.3 for s in A.shapes())
    # closed faces hold 0: the obstacle (u faces 0..2), the walls
    u[:, :, :3] = 0.0
    u[:, :, -1] = 0.0
    v[:, :, :2] = 0.0
    v[:, 0, :] = v[:, -1, :] = 0.0
    w[:, :, :2] = 0.0
    if A.periodic_z:
        w[-1] = w[0]
    else:
        w[0] = w[-1] = 0.0
    p[:, :, :2] = 0.0
    return u, v, w, p


def _mirror(st):
    """A state (fluid in i >= 2) -> the mirror-symmetric B state."""
    u, v, w, p = st

    def even(a):   # cell-centred in x: B cells 6..11 = A cells 2..7, cells 0..5 mirrored
        right = a[:, :, 2:]
        return np.concatenate([right[:, :, ::-1], right], axis=2)

    right = u[:, :, 2:]                      # A faces 2..8 -> B faces 6..12
    ub = np.concatenate([-right[:, :, :0:-1], right], axis=2)
    return ub, even(v), even(w), even(p)


@pytest.mark.parametrize("periodic", [False, True])
def test_slip_obstacle_equals_mirror_doubled_cavity(oracle, periodic):
    A, B = _mirror_pair(oracle, periodic)
    sa = _a_state(A, 3)
    sb = _mirror(sa)
    ra, _, _, s1 = oracle.fine_steps(A, sa, 3, 2e-3, rtol=1e-13)
    rb, _, _, s2 = oracle.fine_steps(B, sb, 3, 2e-3, rtol=1e-13)
    assert s1 == 0 and s2 == 0
    mb = _mirror(ra)
    for c in range(4):
        scale = np.max(np.abs(rb[c]))
        assert np.max(np.abs(mb[c] - rb[c])) <= 1e-10 * scale, c
    # the same obstacle with no-slip walls is a different flow
    An, _ = _mirror_pair(oracle, periodic, slip=False)
    rn, _, _, _ = oracle.fine_steps(An, sa, 3, 2e-3, rtol=1e-13)
    assert np.max(np.abs(_mirror(rn)[2] - rb[2])) > 1e-3 * np.max(np.abs(rb[2]))


def test_plug_flow_in_a_slip_channel_is_steady(oracle):
    n, nz, W0 = 8, 6, 0.7
    solid = np.zeros((nz, n, n), np.uint8)
    solid[:, :, 0] = solid[:, :, -1] = 1
    solid[:, 0, :] = solid[:, -1, :] = 1
    out = {}
    for slip in (True, False):
        g = oracle.Grid(n, n, nz, lz=0.75, re=100.0, solid=solid, periodic_z=True, slip_obstacles=slip)
        u, v, w, p = g.zeros_state()
        fl = g.fluid()
        w[:nz][fl] = W0
        w[nz] = w[0]
        res, _, _, st = oracle.fine_steps(g, (u, v, w, p), 5, 2e-3, rtol=1e-12)
        assert st == 0
        out[slip] = (res, fl)
    (u, v, w, p), fl = out[True]
    assert np.all(u == 0.0) and np.all(v == 0.0) and np.all(p == 0.0)
    assert np.all(w[:nz][fl] == W0)
    (u, v, w, p), fl = out[False]
    assert np.max(np.abs(w[:nz][fl] - W0)) > 1e-2


def test_slip_flag_without_obstacles_changes_nothing(oracle):
    n = 8
    st = inputs.random_state(n, n, n, seed=4, scale=0.2, pscale=0.0)
    a = oracle.fine_steps(oracle.Grid(n, n, n, re=300.0), st, 3, 2e-3, rtol=1e-12)[0]
    b = oracle.fine_steps(oracle.Grid(n, n, n, re=300.0, slip_obstacles=True), st, 3, 2e-3, rtol=1e-12)[0]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_slip_adjoint_is_refused(oracle):
    solid = np.zeros((6, 6, 6), np.uint8)
    solid[2:4, 2:4, 2:4] = 1
    g = oracle.Grid(6, 6, 6, solid=solid, slip_obstacles=True)
    with pytest.raises(NotImplementedError):
        oracle.adjoint_gradient(g, g.zeros_state(), 1, 1e-3)


def _smart_hand(U, C, D):
    # the NVD characteristic written out for the hand computation below
    if D == U:
        return C
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


@pytest.mark.parametrize("slip", [True, False])
def test_image_two_rows_above_an_obstacle_top_by_hand(oracle, slip):
    """A solid slab fills row 2; u is uniform along x and z in every row and
    v = V > 0 on the open v faces.  At the u face of row 4 the upwind triple
    of the lower control-volume face is (row 2, row 3, row 4), and row 2 is
    closed by the obstacle, half a cell beyond row 3: the image is u(row 3)
    itself with a free-slip obstacle (zero tangential stress mirrors it) and
    -u(row 3) with a no-slip one.  Hand value of F at that face."""
    n, re, dt, V = 8, 10.0, 1e-3, 0.3
    h = 1.0 / n
    rows = [0.1, 0.15, 0.0, 0.25, 0.55, 0.6, 0.62, 0.64]
    solid = np.zeros((n, n, n), np.uint8)
    solid[:, 2, :] = 1
    u = np.zeros((n, n, n + 1))
    for j, a in enumerate(rows):
        u[:, j, 1:n] = a
    u[:, 2, :] = 0.0
    v = np.zeros((n, n + 1, n))
    v[:, 1:n, :] = V
    v[:, 2:4, :] = 0.0
    w = np.zeros((n + 1, n, n))
    g = oracle.Grid(n, n, n, re=re, solid=solid, slip_obstacles=slip, lid=np.zeros((n, n + 1)))
    Fu, _, _ = oracle.momentum(g, u, v, w, dt)
    img = rows[3] if slip else -rows[3]
    lap = (rows[5] - 2 * rows[4] + rows[3]) / h ** 2
    fp = V * _smart_hand(rows[3], rows[4], rows[5])
    fm = V * _smart_hand(img, rows[3], rows[4])
    expect = rows[4] + dt * (lap / re - (fp - fm) / h)
    assert Fu[4, 4, 4] == pytest.approx(expect, rel=1e-13)
