"""Parity of the HIP path with the oracle on grids periodic in z (the
boundary condition of the paper's runs, Sec. 3): Poisson solves on flat and
column-tiled grids with and without obstacles, projection steps on the
paper's quasi-2D geometry (32 x 32 x 5 cells on [0,1]^2 x [0,0.1]), random
states with obstacles across the seam, Parareal exactness, and the duplicate
w plane.  Tolerances as for walls: 1e-9 on Poisson solutions, 1e-10 on
velocity (relative L2) for FP64."""
import numpy as np
import pytest

from paper_1705_06149_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def T(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def N(t):
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    num = np.sqrt(sum(np.sum((x - y) ** 2) for x, y in zip(a, b)))
    den = np.sqrt(sum(np.sum(y ** 2) for y in b))
    return num / den


def mean_free(b, fluid):
    b = b.copy()
    b[fluid] -= b[fluid].mean()
    b[~fluid] = 0.0
    return b


def seam_mask(n, nz, seed):
    """Cuboid obstacles that cross the periodic seam, fluid kept connected."""
    from scipy import ndimage
    rng = np.random.default_rng(seed)
    solid = np.zeros((nz, n, n), np.uint8)
    for _ in range(3):
        sx, sy, sz = rng.integers(2, 4, 3)
        x0, y0 = rng.integers(1, n - sx - 1), rng.integers(1, n - sy - 2)
        z0 = rng.integers(0, nz)
        for k in range(sz):
            solid[(z0 + k) % nz, y0:y0 + sy, x0:x0 + sx] = 1
    lab, nlab = ndimage.label(solid == 0, structure=ndimage.generate_binary_structure(3, 1))
    # regions touching through the seam are one region: union-find on labels
    root = list(range(nlab + 1))

    def find(a):
        while root[a] != a:
            root[a] = root[root[a]]
            a = root[a]
        return a
    for a, b in set(zip(lab[0].ravel().tolist(), lab[-1].ravel().tolist())):
        if a and b:
            ra, rb = find(a), find(b)
            if ra != rb:
                root[rb] = ra
    rep = np.array([find(a) for a in range(nlab + 1)])
    lab = rep[lab]
    top = np.unique(lab[:, n - 1, :])
    solid[~np.isin(lab, top[top > 0])] = 1
    return solid


def periodic_state(nx, ny, nz, seed, scale):
    u, v, w, p = inputs.random_state(nx, ny, nz, seed=seed, scale=scale, pscale=0.0)
    w[-1] = w[0]
    return u, v, w, p


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape,obst", [((24, 20, 16), False), ((16, 16, 12), True), ((64, 64, 64), False),
                                        ((64, 64, 72), True)])
def test_periodic_poisson_parity(gpu, oracle, shape, obst, prec):
    nx, ny, nz = shape
    _say("periodic poisson", shape, "obstacles" if obst else "", "prec", prec)
    solid = seam_mask(nx, nz, 7) if obst else None
    g = oracle.Grid(nx, ny, nz, lx=1.0, ly=1.3, lz=0.7, solid=solid, periodic_z=True)
    fluid = g.fluid()
    rng = np.random.default_rng(6)
    B = 2
    bs = [mean_free(rng.standard_normal((nz, ny, nx)), fluid) for _ in range(B)]
    h = gpu.Handle(nx, ny, nz, lx=1.0, ly=1.3, lz=0.7, solid=solid, max_batch=B, periodic_z=True)
    pt = T(np.zeros((B, nz, ny, nx)))
    info = h.poisson_solve(T(np.stack(bs)), pt, gpu.PoissonOpts(rtol=1e-12, prec=prec, inner_rtol=1e-5))
    p = N(pt)
    for i in range(B):
        if prec == 0:
            ref, oinfo = oracle.pcg(g, bs[i], rtol=1e-12)
        else:
            ref, oinfo = oracle.pcg_mixed(g, bs[i], rtol=1e-12, eta=1e-5)
        err = np.linalg.norm(p[i] - ref) / np.linalg.norm(ref)
        _say("  slice", i, "rel err", err, "iters gpu", info[i]["iters"], "oracle", oinfo["iters"])
        assert oinfo["status"] == 0 and info[i]["status"] == 0
        assert err < 1e-9
    h.close()


def test_paper_sim1_geometry_fine_steps(gpu, oracle):
    """32 x 32 x 5 cells on [0,1]^2 x [0,0.1], periodic in z, Re 1000, lid
    u = 1, dt 1e-3, 30 steps from rest (the quasi-2D setup of Sec. 3)."""
    nx, ny, nz, lz = 32, 32, 5, 0.1
    _say("sim1 geometry", nx, ny, nz)
    g = oracle.Grid(nx, ny, nz, lz=lz, re=1000.0, periodic_z=True)
    ref, iters, _, st = oracle.fine_steps(g, g.zeros_state(), 30, 1e-3, rtol=1e-10)
    assert st == 0
    h = gpu.Handle(nx, ny, nz, lz=lz, re=1000.0, max_batch=1, periodic_z=True)
    y = h.zeros_state(1)
    info = h.fine_step(y, 0.0, 0.03, 1e-3, gpu.PoissonOpts(rtol=1e-10))
    out = [N(a)[0] for a in y]
    e = rel_l2(out[:3], ref[:3])
    _say("  velocity rel L2", e, "CG iters gpu", info[0]["iters"], "oracle", int(iters.sum()))
    assert e <= 1e-10
    assert np.array_equal(out[2][-1], out[2][0])
    # from rest, the lid drives a flow that stays z-uniform with w = 0
    assert np.max(np.abs(out[2])) == 0.0
    assert all(np.array_equal(out[0][k], out[0][0]) for k in range(nz))
    h.close()


def test_paper_sim2_geometry_fine_steps(gpu, oracle):
    """32^3 cells on [0,1]^3, periodic in z, 49 seeded cubes along the median
    plane (the stand-in for the paper's fully 3D case, Sec. 3), Re 1000, lid
    u = 1, dt 1e-3: 25 steps from rest and, in a batch of 2, 5 more steps
    from a random state, against the oracle."""
    n = 32
    _say("sim2 geometry", n)
    solid = inputs.median_plane_cubes(n, seed=49)
    g = oracle.Grid(n, n, n, re=1000.0, solid=solid, periodic_z=True)
    ref, iters, _, st = oracle.fine_steps(g, g.zeros_state(), 25, 1e-3, rtol=1e-10)
    assert st == 0
    h = gpu.Handle(n, n, n, re=1000.0, solid=solid, max_batch=2, periodic_z=True)
    y = h.zeros_state(1)
    info = h.fine_step(y, 0.0, 0.025, 1e-3, gpu.PoissonOpts(rtol=1e-10))
    out = [N(a)[0] for a in y]
    e = rel_l2(out[:3], ref[:3])
    _say("  from rest: velocity rel L2", e, "CG iters gpu", info[0]["iters"], "oracle", int(iters.sum()))
    assert e <= 1e-10
    assert np.array_equal(out[2][-1], out[2][0])
    st0 = periodic_state(n, n, n, 12, 0.3)
    ref, _, _, s = oracle.fine_steps(g, st0, 5, 1e-3, rtol=1e-11)
    assert s == 0
    yb = tuple(T(np.stack([a, a])) for a in st0)
    h.fine_step(yb, 0.0, 0.005, 1e-3, gpu.PoissonOpts(rtol=1e-11))
    for b in range(2):
        e = rel_l2([N(a)[b] for a in yb[:3]], ref[:3])
        _say("  random state, slice", b, "velocity rel L2", e)
        assert e <= 1e-10
    h.close()


@pytest.mark.parametrize("shape", [(20, 20, 16), (64, 64, 64)])
def test_periodic_random_state_with_obstacles(gpu, oracle, shape):
    nx, ny, nz = shape
    _say("periodic random state + obstacles", shape)
    solid = seam_mask(nx, nz, 9)
    g = oracle.Grid(nx, ny, nz, re=400.0, solid=solid, periodic_z=True)
    st = periodic_state(nx, ny, nz, 4, 0.2)
    nsteps = 3
    ref, iters, _, s = oracle.fine_steps(g, st, nsteps, 1e-3, rtol=1e-11)
    assert s == 0
    h = gpu.Handle(nx, ny, nz, re=400.0, solid=solid, max_batch=2, periodic_z=True)
    y = tuple(T(np.stack([a, a])) for a in st)
    h.fine_step(y, 0.0, nsteps * 1e-3, 1e-3, gpu.PoissonOpts(rtol=1e-11))
    for b in range(2):
        out = [N(a)[b] for a in y]
        e = rel_l2(out[:3], ref[:3])
        _say("  slice", b, "velocity rel L2", e)
        assert e <= 1e-10
        assert np.array_equal(out[2][-1], out[2][0])
    assert all(np.array_equal(N(a)[0], N(a)[1]) for a in y)
    h.close()


def test_periodic_parareal_exact(gpu, oracle):
    nx, ny, nz, Ns = 12, 12, 6, 3
    dt, DT, T_end = 1e-3, 2e-3, 0.012
    _say("periodic parareal", nx, ny, nz, Ns)
    solid = seam_mask(nx, nz, 3)
    h = gpu.Handle(nx, ny, nz, lz=0.5, re=300.0, solid=solid, max_batch=Ns, periodic_z=True)
    y0 = periodic_state(nx, ny, nz, 8, 0.1)
    opts = gpu.PoissonOpts(rtol=1e-11)
    ys = tuple(T(a[None]) for a in y0)
    serial = [tuple(N(t)[0] for t in ys)]
    for s in range(Ns):
        h.fine_step(ys, s * T_end / Ns, (s + 1) * T_end / Ns, dt, opts)
        serial.append(tuple(N(t)[0] for t in ys))
    Y = tuple(T(np.stack([a] * (Ns + 1))) for a in y0)
    Fk = tuple(T(np.zeros((Ns,) + a.shape)) for a in y0)
    Gk = tuple(T(np.zeros((Ns,) + a.shape)) for a in y0)
    h.parareal_start(Y, Gk, Ns, 0.0, T_end, DT, opts)
    for k in range(Ns):
        h.parareal_iterate(Y, Fk, Gk, Ns, k, 0.0, T_end, dt, DT, opts, opts)
        for m in range(k + 2):
            for c in range(4):
                assert np.array_equal(N(Y[c])[m], serial[m][c]), (k, m, c)
    g = oracle.Grid(nx, ny, nz, lz=0.5, re=300.0, solid=solid, periodic_z=True)
    ref, _, _, st = oracle.fine_steps(g, y0, int(round(T_end / dt)), dt, rtol=1e-11)
    assert rel_l2([N(t)[Ns] for t in Y[:3]], ref[:3]) <= 1e-10
    h.close()


def test_periodic_adjoint_refused(gpu):
    h = gpu.Handle(8, 8, 4, max_batch=1, periodic_z=True)
    y0 = h.zeros_state(1)
    with pytest.raises(gpu.NSPError) as ex:
        h.fine_solve_adjoint(y0, 2, 1e-3)
    assert ex.value.status == gpu.NSP_ERR_UNSUPPORTED
    h.close()
