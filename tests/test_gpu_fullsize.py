"""Parity at the benchmark sizes, in the launch configuration the benchmark
times, on sampled outputs the oracle computes one by one.

* 128^3 cavity, Re 1000, dt 5e-4: 200 FP64 steps and 200 mixed-precision
  steps on the GPU; mixed vs FP64 velocity (relative L2 <= 1e-8); the last
  FP64 step against one oracle step from the GPU's state before it (<= 1e-10).
* Obstacles, uneven batch: 16 states on each of 64^3, 96^3, 128^3 (seeded
  cuboid masks, seeds 1, 2, 3) advanced together by one grouped launch; one
  sampled slice per grid against the oracle's step from the same input, and
  the same slice advanced alone (bitwise).
* Groups of small obstacle grids: grouped Parareal equals each grid's serial
  fine solution after N iterations on N slices (bitwise), iterates match the
  single-grid Parareal bitwise, and the slice ends match the oracle.
* Parareal at 96^3 with 32 slices, in the benchmark's configuration
  (autotuned launch, mixed-precision F, FP64 G, dt 5e-4, DT 5e-3): after the
  first iteration slice 1 is bitwise the batch-1 fine propagation of y0,
  sampled F outputs are bitwise the batch-1 propagation of their inputs, and
  each updated slice end is F + (G_new - G_old) of the stored pieces.
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


def test_cavity128_fp64_mixed_200_steps(gpu, oracle):
    n, re_, dt, steps = 128, 1000.0, 5e-4, 200
    _say("cavity 128^3 fp64 + mixed", steps, "steps")
    h = gpu.Handle(n, n, n, re=re_, max_batch=1)
    o64 = gpu.PoissonOpts(rtol=1e-10, prec=gpu.FP64)
    omx = gpu.PoissonOpts(rtol=1e-10, prec=gpu.MIXED, inner_rtol=1e-5)
    y64 = h.zeros_state(1)
    h.fine_step(y64, 0.0, (steps - 1) * dt, dt, o64)
    before = tuple(N(a)[0].copy() for a in y64)
    info = h.fine_step(y64, (steps - 1) * dt, steps * dt, dt, o64)
    ymx = h.zeros_state(1)
    h.fine_step(ymx, 0.0, steps * dt, dt, omx)
    v64 = [N(a)[0] for a in y64[:3]]
    vmx = [N(a)[0] for a in ymx[:3]]
    e_mx = rel_l2(vmx, v64)
    e_p = rel_l2([N(ymx[3])[0]], [N(y64[3])[0]])
    _say("  mixed vs fp64 velocity rel L2", e_mx, "pressure", e_p)
    assert e_mx <= 1e-8
    g = oracle.Grid(n, n, n, re=re_)
    ref, iters, _, st = oracle.fine_steps(g, before, 1, dt, rtol=1e-10)
    assert st == 0
    e = rel_l2(v64, ref[:3])
    _say("  last step vs oracle", e, "iters gpu/oracle", info[0]["iters"], int(iters[0]))
    assert e <= 1e-10
    h.close()


def _obstacle_grids():
    return [(64, 1), (96, 2), (128, 3)]


def test_obstacles_grouped_step_full_size(gpu, oracle):
    B, dt, re_ = 16, 5e-4, 1000.0
    opts = gpu.PoissonOpts(rtol=1e-10, prec=gpu.FP64)
    hs, ys, inputs_kept, masks = [], [], [], []
    for n, seed in _obstacle_grids():
        _say("obstacles grid", n, "seed", seed, "batch", B)
        m = inputs.obstacle_mask(n, seed)
        masks.append(m)
        h = gpu.Handle(n, n, n, re=re_, solid=m, max_batch=B)
        hs.append(h)
        st = [inputs.random_state(n, n, n, seed=100 * seed + b, scale=0.1, pscale=0.0) for b in range(B)]
        y = tuple(T(np.stack([s[c] for s in st])) for c in range(4))
        ys.append(y)
        pick = (3 * seed) % B
        inputs_kept.append((pick, st[pick]))
    gpu.group_fine_step(hs, ys, 0.0, dt, dt, opts)
    for (n, seed), h, y, (pick, s0), m in zip(_obstacle_grids(), hs, ys, inputs_kept, masks):
        got = [N(a)[pick] for a in y]
        # the same slice alone
        y1 = tuple(T(a[None]) for a in s0)
        h.fine_step(y1, 0.0, dt, dt, opts)
        for c in range(4):
            assert np.array_equal(N(y1[c])[0], got[c]), (n, c)
        g = oracle.Grid(n, n, n, re=re_, solid=m)
        ref, iters, _, st = oracle.fine_steps(g, s0, 1, dt, rtol=1e-10)
        assert st == 0
        e = rel_l2(got[:3], ref[:3])
        _say("  grid", n, "slice", pick, "vs oracle", e)
        assert e <= 1e-10
    for h in hs:
        h.close()


def test_group_parareal_obstacles_exact(gpu, oracle):
    grids = [(12, 1), (14, 2), (16, 3)]
    Ns, dt, DT, T_end, re_ = 3, 1e-3, 2e-3, 0.012, 500.0
    sl = T_end / Ns
    opts = gpu.PoissonOpts(rtol=1e-11)
    hs, Ys, Fks, Gks, serial, masks = [], [], [], [], [], []
    for n, seed in grids:
        _say("group parareal obstacles", n, seed)
        m = inputs.obstacle_mask(n, seed, frac=0.05, smin=2, smax=4)
        masks.append(m)
        h = gpu.Handle(n, n, n, re=re_, solid=m, max_batch=Ns)
        hs.append(h)
        y0 = inputs.rest_state(n, n, n)
        ys = tuple(T(a[None]) for a in y0)
        ser = [tuple(N(t)[0] for t in ys)]
        for s in range(Ns):
            h.fine_step(ys, s * sl, (s + 1) * sl, dt, opts)
            ser.append(tuple(N(t)[0] for t in ys))
        serial.append(ser)
        Ys.append(tuple(T(np.stack([a] * (Ns + 1))) for a in y0))
        Fks.append(tuple(T(np.zeros((Ns,) + a.shape)) for a in y0))
        Gks.append(tuple(T(np.zeros((Ns,) + a.shape)) for a in y0))
    # the same iteration on one grid alone, for the group == single check
    Y1 = tuple(t.clone() for t in Ys[1])
    F1 = tuple(t.clone() for t in Fks[1])
    G1 = tuple(t.clone() for t in Gks[1])
    gpu.group_parareal_start(hs, Ys, Gks, Ns, 0.0, T_end, DT, opts)
    hs[1].parareal_start(Y1, G1, Ns, 0.0, T_end, DT, opts)
    for k in range(Ns):
        jumps = gpu.group_parareal_iterate(hs, Ys, Fks, Gks, Ns, k, 0.0, T_end, dt, DT, opts, opts)
        j1 = hs[1].parareal_iterate(Y1, F1, G1, Ns, k, 0.0, T_end, dt, DT, opts, opts)
        _say("  k", k, "jumps", jumps)
        assert jumps[1] == j1
        for c in range(4):
            assert np.array_equal(N(Ys[1][c]), N(Y1[c])), (k, c)
        for g_i in range(len(grids)):
            for mth in range(k + 2):
                for c in range(4):
                    assert np.array_equal(N(Ys[g_i][c])[mth], serial[g_i][mth][c]), (g_i, k, mth, c)
    for (n, seed), m, Y in zip(grids, masks, Ys):
        g = oracle.Grid(n, n, n, re=re_, solid=m)
        ref, _, _, st = oracle.fine_steps(g, inputs.rest_state(n, n, n), int(round(T_end / dt)), dt, rtol=1e-11)
        e = rel_l2([N(t)[Ns] for t in Y[:3]], ref[:3])
        _say("  grid", n, "end vs oracle", e)
        assert e <= 1e-10
    for h in hs:
        h.close()


def test_parareal96_full_size_first_iteration(gpu):
    n, Ns, dt, DT, T_end = 96, 32, 5e-4, 5e-3, 0.64
    sl = T_end / Ns
    _say("parareal full size", n, Ns)
    h = gpu.Handle(n, n, n, re=1000.0, max_batch=Ns)
    wg, planes, items = h.autotune(Ns, gpu.MIXED)
    _say("  autotuned", wg, planes, items)
    fine = gpu.PoissonOpts(rtol=1e-10, prec=gpu.MIXED, inner_rtol=1e-5)
    coarse = gpu.PoissonOpts(rtol=1e-10, prec=gpu.FP64)
    y0 = inputs.rest_state(n, n, n)
    Y = tuple(T(np.stack([a] * (Ns + 1))) for a in y0)
    Fk = tuple(T(np.zeros((Ns,) + a.shape)) for a in y0)
    Gk = tuple(T(np.zeros((Ns,) + a.shape)) for a in y0)
    h.parareal_start(Y, Gk, Ns, 0.0, T_end, DT, coarse)
    Y_old = [N(a) for a in Y]
    G_old = [N(a) for a in Gk]
    jv, jp = h.parareal_iterate(Y, Fk, Gk, Ns, 0, 0.0, T_end, dt, DT, fine, coarse)
    _say("  jump", jv, jp)
    assert np.isfinite(jv) and 0 < jv < 1
    Yn = [N(a) for a in Y]
    Fn = [N(a) for a in Fk]
    Gn = [N(a) for a in Gk]
    # slice 1: exact after one iteration, the batch-1 fine solve of y0
    ys = tuple(T(a[None]) for a in y0)
    h.fine_step(ys, 0.0, sl, dt, fine)
    for c in range(4):
        assert np.array_equal(Yn[c][1], N(ys[c])[0]), c
    # sampled F outputs equal the batch-1 propagation of their inputs
    for m in (7, 31):
        ys = tuple(T(a[m][None]) for a in Y_old)
        h.fine_step(ys, m * sl, (m + 1) * sl, dt, fine)
        for c in range(4):
            assert np.array_equal(Fn[c][m], N(ys[c])[0]), (m, c)
    # the update of Eq. (6) from the stored pieces
    for m in (1, 8, 32):
        for c in range(4):
            assert np.array_equal(Yn[c][m], Fn[c][m - 1] + (Gn[c][m - 1] - G_old[c][m - 1])), (m, c)
    # the jump is the max over slices of |Y_new - Y_old| in u, v, w
    j = max(float(np.max(np.abs(Yn[c][1:] - Y_old[c][1:]))) for c in range(3))
    assert j == jv
    h.close()
