"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every case prints its name and sizes before touching the GPU.  Tolerances:
velocity relative L2 <= 1e-10 for the FP64 path (the oracle and the kernels
stop CG at the same 1e-10 relative residual but sum in different orders;
perturbing the oracle's stopping tolerance moves the c1 velocity by ~5e-13),
<= 1e-8 for the mixed-precision path against the FP64 oracle.
"""
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


def connected_mask(n, seed, frac=0.08):
    return inputs.obstacle_mask(n, seed, frac=frac, smin=2, smax=4)


def mean_free(b, fluid):
    b = b.copy()
    b[fluid] -= b[fluid].mean()
    b[~fluid] = 0.0
    return b


@pytest.mark.parametrize("shape,obst", [((24, 20, 16), False), ((16, 16, 16), True), ((40, 33, 7), False)])
@pytest.mark.parametrize("prec", [0, 1])
def test_poisson_parity(gpu, oracle, shape, obst, prec):
    nx, ny, nz = shape
    _say("poisson", shape, "obstacles" if obst else "", "prec", prec)
    solid = connected_mask(nx, 11) if (obst and nx == ny == nz) else None
    g = oracle.Grid(nx, ny, nz, lx=1.0, ly=1.3, lz=0.7, solid=solid)
    fluid = g.fluid()
    rng = np.random.default_rng(5)
    B = 3
    bs = [mean_free(rng.standard_normal((nz, ny, nx)), fluid) for _ in range(B)]
    x0 = [mean_free(rng.standard_normal((nz, ny, nx)), fluid) * (0.1 * i) for i in range(B)]
    h = gpu.Handle(nx, ny, nz, lx=1.0, ly=1.3, lz=0.7, solid=solid, max_batch=B)
    bt = T(np.stack(bs))
    pt = T(np.stack(x0))
    opts = gpu.PoissonOpts(rtol=1e-12, prec=prec, inner_rtol=1e-5)
    info = h.poisson_solve(bt, pt, opts)
    p = N(pt)
    for i in range(B):
        if prec == 0:
            ref, oinfo = oracle.pcg(g, bs[i], x0[i], rtol=1e-12)
        else:
            ref, oinfo = oracle.pcg_mixed(g, bs[i], x0[i], rtol=1e-12, eta=1e-5)
        assert oinfo["status"] == 0
        err = np.linalg.norm(p[i] - ref) / np.linalg.norm(ref)
        _say("  slice", i, "rel err", err, "iters gpu", info[i]["iters"], "oracle", oinfo["iters"])
        assert err < 1e-9
        assert info[i]["status"] == 0
        assert info[i]["rel_res_true"] <= 2e-12
        assert abs(p[i][fluid].mean()) < 1e-12 * np.abs(ref).max()
        if prec == 0:
            assert abs(info[i]["iters"] - oinfo["iters"]) <= 2
    h.close()


def test_fine_step_cavity32_fp64(gpu, oracle):
    """32^3 cavity, Re 100, dt 1e-3, 50 steps, FP64 Jacobi-PCG to 1e-10."""
    _say("fine_step cavity32 Re100 50 steps fp64")
    n = 32
    g = oracle.Grid(n, n, n, re=100.0)
    y0 = g.zeros_state()
    ref, oit, orel, st = oracle.fine_steps(g, y0, 50, 1e-3, rtol=1e-10)
    assert st == 0
    h = gpu.Handle(n, n, n, re=100.0, max_batch=1)
    y = tuple(T(a[None]) for a in y0)
    info = h.fine_step(y, 0.0, 0.05, 1e-3, gpu.PoissonOpts(rtol=1e-10))
    out = [N(t)[0] for t in y]
    e_vel = rel_l2(out[:3], ref[:3])
    e_p = np.linalg.norm(out[3] - ref[3]) / np.linalg.norm(ref[3])
    _say("  vel rel L2", e_vel, "p rel L2", e_p, "iters gpu", info[0]["iters"], "oracle", int(oit.sum()))
    assert e_vel <= 1e-10
    assert e_p <= 1e-9
    assert abs(info[0]["iters"] - int(oit.sum())) <= 50
    assert info[0]["rel_res_true"] <= 2e-10
    h.close()


def test_fine_step_mixed_vs_fp64_oracle(gpu, oracle):
    _say("fine_step cavity32 mixed 20 steps")
    n = 32
    g = oracle.Grid(n, n, n, re=1000.0)
    y0 = g.zeros_state()
    ref, _, _, st = oracle.fine_steps(g, y0, 20, 5e-4, rtol=1e-10)
    h = gpu.Handle(n, n, n, re=1000.0, max_batch=1)
    y = tuple(T(a[None]) for a in y0)
    info = h.fine_step(y, 0.0, 0.01, 5e-4, gpu.PoissonOpts(rtol=1e-10, prec=gpu.MIXED, inner_rtol=1e-5))
    out = [N(t)[0] for t in y]
    e_vel = rel_l2(out[:3], ref[:3])
    _say("  mixed vs fp64 oracle: vel", e_vel, "info", info[0])
    assert e_vel <= 1e-8
    assert info[0]["rel_res_true"] <= 1e-10
    h.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_fine_step_obstacles_ragged(gpu, oracle, prec):
    """Ragged grid with obstacles, random start (closed faces hold garbage)."""
    nx, ny, nz = 22, 19, 17
    _say("fine_step obstacles ragged", (nx, ny, nz), "prec", prec)
    rng = np.random.default_rng(3)
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[4:9, 5:8, 6:12] = 1
    solid[10:12, 2:6, 3:5] = 1
    solid[12, 10, 10] = 1           # single-cell obstacle
    solid[5:7, 12:14, 15] = 1       # thin slab
    g = oracle.Grid(nx, ny, nz, lx=1.1, ly=1.0, lz=0.9, re=400.0, solid=solid)
    g.lid = 1.0 + 0.3 * rng.standard_normal((nz, nx + 1))
    y0 = inputs.random_state(nx, ny, nz, seed=9, scale=0.3, pscale=0.0)
    ref, oit, _, st = oracle.fine_steps(g, y0, 6, 2e-3, prec=0, rtol=1e-11)
    assert st == 0
    h = gpu.Handle(nx, ny, nz, lx=1.1, ly=1.0, lz=0.9, re=400.0, solid=solid, max_batch=1)
    h.set_lid(T(g.lid))
    y = tuple(T(a[None]) for a in y0)
    h.fine_step(y, 0.0, 0.012, 2e-3, gpu.PoissonOpts(rtol=1e-11, prec=prec))
    out = [N(t)[0] for t in y]
    e_vel = rel_l2(out[:3], ref[:3])
    _say("  vel rel L2", e_vel)
    assert e_vel <= (1e-10 if prec == 0 else 1e-8)
    # closed faces are written as exact zeros
    for a, b in zip(out[:3], ref[:3]):
        assert np.array_equal(a == 0.0, b == 0.0) or np.all(np.abs(a[b == 0.0]) == 0.0)
    h.close()


def test_batched_equals_unbatched(gpu):
    """A batch of slices gives bit-identical results to one-slice launches."""
    n = 20
    _say("batched == unbatched", n)
    B = 4
    states = [inputs.random_state(n, n, n, seed=100 + i, scale=0.2, pscale=0.0) for i in range(B)]
    h = gpu.Handle(n, n, n, re=500.0, max_batch=B)
    for prec in (0, 1):
        opts = gpu.PoissonOpts(rtol=1e-10, prec=prec)
        yb = tuple(T(np.stack([s[c] for s in states])) for c in range(4))
        h.fine_step(yb, 0.0, 0.006, 2e-3, opts)
        for i in range(B):
            yi = tuple(T(states[i][c][None]) for c in range(4))
            h.fine_step(yi, 0.0, 0.006, 2e-3, opts)
            for c in range(4):
                assert np.array_equal(N(yb[c])[i], N(yi[c])[0]), (prec, i, c)
    h.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_column_depth_does_not_change_results(gpu, prec):
    """128 x ny x nz Poisson solves: a batch of 8 runs with deeper column
    tiles (and, in FP32 inner solves, two rows per thread), a batch of 1 with
    the shallowest tiles and one row per thread; partial sums are kept per row
    block and 8 planes (128^3) or 4 planes (the two smaller grids, whose slice
    has fewer 8-plane tiles than workgroups), so the slices must agree bitwise
    (with obstacles, a ragged last row block, an odd number of row blocks, nz
    not a multiple of 16)."""
    for shape, obst in [((128, 128, 128), False), ((128, 92, 112), True), ((128, 88, 120), False)]:
        nx, ny, nz = shape
        _say("column depth independence", shape, "obstacles", obst, "prec", prec)
        solid = inputs.obstacle_mask(nx, 4)[:nz, :ny, :nx] if obst else None
        if obst:
            solid = np.ascontiguousarray(solid)
            from scipy import ndimage
            lab, _ = ndimage.label(solid == 0)
            top = np.unique(lab[:, ny - 1, :])
            solid[~np.isin(lab, top[top > 0])] = 1
        fluid = np.ones((nz, ny, nx), bool) if solid is None else solid == 0
        rng = np.random.default_rng(11)
        B = 8
        bs = [mean_free(rng.standard_normal((nz, ny, nx)), fluid) for _ in range(B)]
        h = gpu.Handle(nx, ny, nz, re=100.0, solid=solid, max_batch=B)
        opts = gpu.PoissonOpts(rtol=1e-10, prec=prec)
        pb = T(np.zeros((B, nz, ny, nx)))
        h.poisson_solve(T(np.stack(bs)), pb, opts)
        for i in (0, 5):
            p1 = T(np.zeros((1, nz, ny, nx)))
            h.poisson_solve(T(bs[i][None]), p1, opts)
            assert np.array_equal(N(pb)[i], N(p1)[0]), (shape, i)
        h.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_autotune_keeps_results(gpu, prec):
    """nsp_autotune picks a workgroup count, a column depth and (FP32 inner
    solves) the rows per thread; the solution computed before and after
    tuning is bitwise the same."""
    n, B = 128, 4
    _say("autotune", n, B, "prec", prec)
    rng = np.random.default_rng(3)
    fluid = np.ones((n, n, n), bool)
    b = T(np.stack([mean_free(rng.standard_normal((n, n, n)), fluid) for _ in range(B)]))
    h = gpu.Handle(n, n, n, re=100.0, max_batch=B)
    opts = gpu.PoissonOpts(rtol=1e-10, prec=prec)
    p0 = T(np.zeros((B, n, n, n)))
    h.poisson_solve(b, p0, opts)
    wg, planes, items = h.autotune(B, prec)
    _say("  chose", wg, "workgroups,", planes, "planes,", items, "rows per thread")
    assert wg >= 1 and planes in (4, 8, 16, 32) and items in ((1,) if prec == 0 else (1, 2))
    p1 = T(np.zeros((B, n, n, n)))
    h.poisson_solve(b, p1, opts)
    assert np.array_equal(N(p0), N(p1))
    h.close()


def test_group_launch_equals_single(gpu):
    """Two grids in one launch (uneven batch) equal separate launches bitwise."""
    _say("group launch == single launches")
    sizes = [(16, 16, 16), (24, 20, 18)]
    hs = [gpu.Handle(*s, re=300.0, max_batch=2) for s in sizes]
    st = [tuple(T(np.stack([inputs.random_state(*s, seed=7 + j, scale=0.2, pscale=0.0)[c] for j in range(2)]))
                for c in range(4)) for s in sizes]
    ref = [tuple(t.clone() for t in y) for y in st]
    opts = gpu.PoissonOpts(rtol=1e-10)
    gpu.group_fine_step(hs, st, 0.0, 0.004, 2e-3, opts)
    for h, y in zip(hs, ref):
        h.fine_step(y, 0.0, 0.004, 2e-3, opts)
    for y, r in zip(st, ref):
        for a, b in zip(y, r):
            assert np.array_equal(N(a), N(b))
    for h in hs:
        h.close()


def test_parareal_exact_after_n_iterations(gpu, oracle):
    """Eq. (6): after k iterations slices 0..k equal the serial fine solution;
    after N iterations on N slices every slice does (bitwise, GPU vs GPU), and
    the slice ends match the oracle's serial fine solution."""
    n, N_s = 12, 4
    dt, DT, T_end = 1e-3, 3e-3, 0.012
    _say("parareal exactness", n, "slices", N_s)
    h = gpu.Handle(n, n, n, re=200.0, max_batch=N_s)
    y0 = inputs.rest_state(n, n, n)
    opts = gpu.PoissonOpts(rtol=1e-11)
    # serial fine on the GPU, slice by slice
    ys = tuple(T(a[None]) for a in y0)
    serial = [tuple(N(t)[0] for t in ys)]
    for s in range(N_s):
        h.fine_step(ys, s * 0.003, (s + 1) * 0.003, dt, opts)
        serial.append(tuple(N(t)[0] for t in ys))
    Y = tuple(T(np.stack([a] * (N_s + 1))) for a in y0)
    Fk = tuple(T(np.zeros((N_s,) + a.shape)) for a in y0)
    Gk = tuple(T(np.zeros((N_s,) + a.shape)) for a in y0)
    h.parareal_start(Y, Gk, N_s, 0.0, T_end, DT, opts)
    for k in range(N_s):
        jv, jp = h.parareal_iterate(Y, Fk, Gk, N_s, k, 0.0, T_end, dt, DT, opts, opts)
        _say("  k", k, "jump", jv, jp)
        for m in range(k + 2):
            for c in range(4):
                assert np.array_equal(N(Y[c])[m], serial[m][c]), (k, m, c)
    g = oracle.Grid(n, n, n, re=200.0)
    ref, _, _, st = oracle.fine_steps(g, y0, 12, dt, rtol=1e-11)
    out = [N(t)[N_s] for t in Y]
    assert rel_l2(out[:3], ref[:3]) <= 1e-10
    h.close()


def test_parareal_matches_oracle_iterates(gpu, oracle):
    """Each Parareal iterate (not only the converged one) matches the
    oracle's Eq. (6) iterates."""
    n, N_s = 10, 3
    dt, DT = 1e-3, 2e-3
    T_end = 0.006
    _say("parareal iterates vs oracle", n, N_s)
    g = oracle.Grid(n, n, n, re=150.0)
    y0 = inputs.rest_state(n, n, n)

    def F(y, s):
        return oracle.propagate(g, y, s * 0.002, (s + 1) * 0.002, dt, rtol=1e-11)

    def G(y, s):
        return oracle.propagate(g, y, s * 0.002, (s + 1) * 0.002, DT, rtol=1e-11)

    def jn(a, b):
        return max(float(np.max(np.abs(x - y))) for x, y in zip(a[:3], b[:3]))

    _, hist = oracle.parareal(y0, N_s, F, G, n_it=2, jump_norm=jn)
    h = gpu.Handle(n, n, n, re=150.0, max_batch=N_s)
    opts = gpu.PoissonOpts(rtol=1e-11)
    Y = tuple(T(np.stack([a] * (N_s + 1))) for a in y0)
    Fk = tuple(T(np.zeros((N_s,) + a.shape)) for a in y0)
    Gk = tuple(T(np.zeros((N_s,) + a.shape)) for a in y0)
    h.parareal_start(Y, Gk, N_s, 0.0, T_end, DT, opts)
    for m in range(N_s + 1):
        assert rel_l2([N(t)[m] for t in Y[:3]], hist[0]["Y"][m][:3]) <= 1e-10 if m else True
    for k in range(2):
        jv, jp = h.parareal_iterate(Y, Fk, Gk, N_s, k, 0.0, T_end, dt, DT, opts, opts)
        ref_Y = hist[k + 1]["Y"]
        for m in range(1, N_s + 1):
            e = rel_l2([N(t)[m] for t in Y[:3]], ref_Y[m][:3])
            assert e <= 1e-10, (k, m, e)
        assert abs(jv - hist[k + 1]["jump"]) <= 1e-10 * max(1.0, hist[k + 1]["jump"]) + 1e-13
    h.close()


def test_parareal_reports_a_solve_at_its_limit(gpu):
    """A fine solve capped at one CG iteration: the Parareal iteration still
    completes (Eq. (6) takes the solve's best iterate, the jumps are written)
    and reports NSP_ERR_NOT_CONVERGED instead of NSP_OK."""
    _say("parareal with maxit = 1")
    n, N_s = 16, 2
    h = gpu.Handle(n, n, n, re=100.0, max_batch=N_s)
    y0 = h.zeros_state(1)
    Y = tuple(t.repeat((N_s + 1,) + (1,) * (t.dim() - 1)).contiguous() for t in y0)
    Fk = h.zeros_state(N_s)
    Gk = h.zeros_state(N_s)
    good = gpu.PoissonOpts(rtol=1e-10)
    h.parareal_start(Y, Gk, N_s, 0.0, 0.004, 2e-3, good)
    capped = gpu.PoissonOpts(rtol=1e-10, maxit=1)
    with pytest.raises(gpu.NSPError) as e:
        h.parareal_iterate(Y, Fk, Gk, N_s, 0, 0.0, 0.004, 1e-3, 2e-3, capped, good)
    assert e.value.status == gpu.NSP_ERR_NOT_CONVERGED
    jv, jp = h.parareal_iterate(Y, Fk, Gk, N_s, 0, 0.0, 0.004, 1e-3, 2e-3, capped, good, check=False)
    assert h.last_status == gpu.NSP_ERR_NOT_CONVERGED
    assert np.isfinite(jv) and jv > 0.0 and np.isfinite(jp)
    # the coarse propagator at its limit is reported the same way
    jv, jp = h.parareal_iterate(Y, Fk, Gk, N_s, 0, 0.0, 0.004, 1e-3, 2e-3, good, capped, check=False)
    assert h.last_status == gpu.NSP_ERR_NOT_CONVERGED and np.isfinite(jv)
    h.close()


def test_error_paths(gpu):
    _say("error paths")
    n = 8
    h = gpu.Handle(n, n, n, max_batch=1)
    y = h.zeros_state(1)
    with pytest.raises(gpu.NSPError) as e:
        h.fine_step(y, 0.0, 0.0025, 1e-3)
    assert e.value.status == gpu.NSP_ERR_ARG
    # maxit = 1: not converged, state still written, info filled
    with pytest.raises(gpu.NSPError) as e:
        h.fine_step(y, 0.0, 0.001, 1e-3, gpu.PoissonOpts(rtol=1e-10, maxit=1))
    assert e.value.status == gpu.NSP_ERR_NOT_CONVERGED
    assert e.value.info[0]["iters"] == 1
    assert float(y[0].abs().max()) > 0.0
    # NaN input: non-finite
    y2 = h.zeros_state(1)
    y2[0][0, 3, 3, 3] = float("nan")
    with pytest.raises(gpu.NSPError) as e:
        h.fine_step(y2, 0.0, 0.001, 1e-3)
    assert e.value.status == gpu.NSP_ERR_NONFINITE
    # wrong dtype / shape rejected before the ABI
    import torch
    with pytest.raises(TypeError):
        h.fine_step(tuple(t.float() for t in y), 0.0, 0.001, 1e-3)
    with pytest.raises(ValueError):
        h.fine_step((y[0][:, :, :, :-1].contiguous(),) + y[1:], 0.0, 0.001, 1e-3)
    with pytest.raises(ValueError):
        h.fine_step(tuple(t.cpu() for t in y), 0.0, 0.001, 1e-3)
    # zero steps is a no-op
    y3 = h.zeros_state(1)
    h.fine_step(y3, 0.5, 0.5, 1e-3)
    assert float(y3[0].abs().max()) == 0.0
    # an empty batch is a no-op (null pointers from empty tensors)
    assert h.fine_step(h.zeros_state(0), 0.0, 0.002, 1e-3) == []
    e0 = torch.zeros((0, n, n, n), dtype=torch.float64, device="cuda")
    assert h.poisson_solve(e0, e0.clone()) == []
    # a grouped launch skips a group with an empty batch
    h2 = gpu.Handle(n + 2, n, n, max_batch=1)
    ya, yb = h.zeros_state(0), h2.zeros_state(1)
    gpu.group_fine_step([h, h2], [ya, yb], 0.0, 0.002, 1e-3)
    ref = h2.zeros_state(1)
    h2.fine_step(ref, 0.0, 0.002, 1e-3)
    for a, b in zip(yb, ref):
        assert torch.equal(a, b)
    h2.close()
    h.close()
    del torch


def test_zero_lid_stays_zero(gpu):
    _say("zero lid stays zero")
    n = 16
    h = gpu.Handle(n, n, n, max_batch=1)
    import torch
    h.set_lid(torch.zeros((n, n + 1), dtype=torch.float64, device="cuda"))
    y = h.zeros_state(1)
    info = h.fine_step(y, 0.0, 0.005, 1e-3)
    for t in y:
        assert float(t.abs().max()) == 0.0
    assert info[0]["iters"] == 0
    h.close()


def test_launch_stats_count_what_ran(gpu):
    """nsp_launch_stats_get: launches, cell-steps and CG cell-iterations per
    launch kind, matching the per-slice solve info; autotune trials are not
    counted; reset clears."""
    n, B = 16, 3
    _say("launch stats")
    h = gpu.Handle(n, n, n, re=200.0, max_batch=B)
    h.launch_stats(reset=True)
    y = tuple(T(np.stack([a] * B)) for a in inputs.random_state(n, n, n, seed=1, scale=0.1, pscale=0.0))
    info = h.fine_step(y, 0.0, 0.004, 1e-3)
    b = T(np.random.default_rng(2).standard_normal((B, n, n, n)))
    pinfo = h.poisson_solve(b, T(np.zeros((B, n, n, n))))
    h.autotune(B, gpu.FP64)
    st = h.launch_stats(reset=True)
    cells = n ** 3
    assert st["fine"]["launches"] == 1 and st["poisson"]["launches"] == 1 and st["project"]["launches"] == 0
    assert st["fine"]["cell_steps"] == B * cells * 4
    assert st["fine"]["cg_cell_iters"] == cells * sum(x["iters"] for x in info)
    assert st["poisson"]["cell_steps"] == B * cells
    assert st["poisson"]["cg_cell_iters"] == cells * sum(x["iters"] for x in pinfo)
    assert st["fine"]["ms"] > 0 and st["poisson"]["ms"] > 0
    assert st["fine"]["cg64_cell_iters"] == st["fine"]["cg_cell_iters"]
    assert st["fine"]["cg32_cell_iters"] == 0 and st["fine"]["bicg_cell_iters"] == 0
    st = h.launch_stats()
    assert all(v["launches"] == 0 for v in st.values())
    # mixed precision and BiCGStab land in their own fields
    mi = h.poisson_solve(b, T(np.zeros((B, n, n, n))), gpu.PoissonOpts(prec=gpu.MIXED))
    bi = h.poisson_solve(b, T(np.zeros((B, n, n, n))), gpu.PoissonOpts(solver=gpu.BICGSTAB))
    st = h.launch_stats(reset=True)["poisson"]
    assert st["cg32_cell_iters"] == cells * sum(x["iters"] for x in mi)
    assert st["mixed_cell_sweeps"] == cells * sum(x["outer"] for x in mi)
    assert st["bicg_cell_iters"] == cells * sum(x["iters"] for x in bi)
    assert st["cg64_cell_iters"] == 0
    h.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", [(512, 16, 32), (32, 128, 64)])
def test_column_tile_extreme_row_widths(gpu, oracle, shape, prec):
    """Column tiles at the widest rows they take (nx = 512: two rows per tile,
    every thread also computes a halo value) and the narrowest (nx = 32: 32
    rows, one halo wave), 2^18 cells each: Poisson solves and projection
    steps with obstacles against the oracle."""
    nx, ny, nz = shape
    _say("column tiles, row width", nx, "prec", prec)
    from scipy import ndimage
    rng = np.random.default_rng(8)
    solid = np.zeros((nz, ny, nx), np.uint8)
    for _ in range(12):
        sx, sy, sz = rng.integers(2, 5, 3)
        x0, y0, z0 = rng.integers(1, nx - sx - 1), rng.integers(1, ny - sy - 2), rng.integers(1, nz - sz - 1)
        solid[z0:z0 + sz, y0:y0 + sy, x0:x0 + sx] = 1
    lab, _ = ndimage.label(solid == 0)
    top = np.unique(lab[:, ny - 1, :])
    solid[~np.isin(lab, top[top > 0])] = 1
    ls = dict(lx=nx / 128.0, ly=ny / 128.0, lz=nz / 128.0)   # cubic cells, h = 1/128
    g = oracle.Grid(nx, ny, nz, re=300.0, solid=solid, **ls)
    fluid = g.fluid()
    b = mean_free(rng.standard_normal((nz, ny, nx)), fluid)
    h = gpu.Handle(nx, ny, nz, re=300.0, solid=solid, max_batch=1, **ls)
    pt = T(np.zeros((1, nz, ny, nx)))
    info = h.poisson_solve(T(b[None]), pt, gpu.PoissonOpts(rtol=1e-12, prec=prec))[0]
    ref, oinfo = oracle.pcg(g, b, rtol=1e-12) if prec == 0 else oracle.pcg_mixed(g, b, rtol=1e-12)
    assert oinfo["status"] == 0
    e = np.linalg.norm(N(pt)[0] - ref) / np.linalg.norm(ref)
    _say("  poisson rel err", e, "iters gpu", info["iters"], "oracle", oinfo["iters"])
    assert e < 1e-9
    assert info["status"] == 0 and info["rel_res_true"] <= 2e-12
    if prec == 0:
        assert abs(info["iters"] - oinfo["iters"]) <= 2
    st = inputs.random_state(nx, ny, nz, seed=2, scale=0.2, pscale=0.0)
    refs, _, _, s = oracle.fine_steps(g, st, 2, 1e-3, prec=prec, rtol=1e-11)
    assert s == 0
    y = tuple(T(a[None]) for a in st)
    h.fine_step(y, 0.0, 0.002, 1e-3, gpu.PoissonOpts(rtol=1e-11, prec=prec))
    e = rel_l2([N(a)[0] for a in y[:3]], refs[:3])
    _say("  step velocity rel L2", e)
    assert e <= (1e-10 if prec == 0 else 1e-8)
    h.close()
