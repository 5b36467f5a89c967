"""The hand-written adjoint on the GPU (through the C ABI and the autograd
wrapper): against the oracle's adjoint on a small grid with obstacles, and
against central finite differences of the GPU forward solve at the full
adjoint workload (96^3, Re 400, 100 steps of 1e-3, checkpoints every 10)."""
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


def test_adjoint_matches_oracle(gpu, oracle):
    n, steps, dt = 12, 5, 1e-3
    _say("adjoint vs oracle", n, steps)
    solid = np.zeros((n, n, n), np.uint8)
    solid[4:7, 3:5, 5:8] = 1
    rng = np.random.default_rng(1)
    lid = 1.0 + 0.1 * rng.standard_normal((n, n + 1))
    g = oracle.Grid(n, n, n, re=400.0, solid=solid, lid=lid)
    u0 = inputs.div_free_perturbation(n, n, n, seed=5, sigma=1e-2)
    st0 = (u0[0], u0[1], u0[2], np.zeros((n, n, n)))
    J, grad, glid = oracle.adjoint_gradient(g, st0, steps, dt, rtol=1e-12, ckpt_every=2)
    h = gpu.Handle(n, n, n, re=400.0, solid=solid, max_batch=1)
    h.set_lid(T(lid))
    y0 = tuple(T(a[None]) for a in st0)
    Jg, gg, gl = h.fine_solve_adjoint(y0, steps, dt, ckpt_every=2, opts=gpu.PoissonOpts(rtol=1e-12))
    _say("  J", Jg, J)
    assert Jg == pytest.approx(J, rel=1e-12)
    num = np.sqrt(sum(np.sum((N(a)[0] - b) ** 2) for a, b in zip(gg, grad)))
    den = np.sqrt(sum(np.sum(b ** 2) for b in grad))
    _say("  grad rel L2", num / den)
    assert num / den <= 1e-9
    assert np.linalg.norm(N(gl) - glid) <= 1e-9 * np.linalg.norm(glid)
    # checkpoint spacing does not matter
    Jg2, gg2, gl2 = h.fine_solve_adjoint(y0, steps, dt, ckpt_every=0, opts=gpu.PoissonOpts(rtol=1e-12))
    assert Jg2 == Jg
    for a, b in zip(gg, gg2):
        assert np.max(np.abs(N(a) - N(b))) <= 1e-13 * np.max(np.abs(N(a)))
    h.close()


def _small_case(gpu, n=14):
    solid = np.zeros((n, n, n), np.uint8)
    solid[4:7, 3:5, 5:8] = 1
    solid[2, n - 2, 3] = 1  # an obstacle under the lid
    lid = 1.0 + 0.1 * np.random.default_rng(2).standard_normal((n, n + 1))
    h = gpu.Handle(n, n, n, re=400.0, solid=solid, max_batch=1)
    h.set_lid(T(lid))
    u0 = inputs.div_free_perturbation(n, n, n, seed=5, sigma=1e-1)
    y0 = tuple(T(a[None]) for a in (u0[0], u0[1], u0[2], np.zeros((n, n, n))))
    return h, y0, lid


def test_record_and_reverse(gpu):
    """nsp_fine_solve_record + nsp_fine_solve_reverse give the one-call
    gradient bitwise; a record can be reversed twice; set_lid or a newer
    record makes it stale (NSP_ERR_ARG, outputs untouched)."""
    steps, dt = 6, 1e-3
    _say("record/reverse", steps)
    h, y0, lid = _small_case(gpu)
    opts = gpu.PoissonOpts(rtol=1e-12)
    J1, g1, gl1 = h.fine_solve_adjoint(y0, steps, dt, ckpt_every=3, opts=opts)
    J2, tape = h.fine_solve_record(y0, steps, dt, ckpt_every=3, opts=opts)
    assert J2 == J1 and tape != 0 and h.tape_valid(tape)
    g2, gl2 = h.fine_solve_reverse(tape)
    g3, gl3 = h.fine_solve_reverse(tape)
    for a, b, c in zip(g1 + (gl1,), g2 + (gl2,), g3 + (gl3,)):
        assert np.array_equal(N(a), N(b)) and np.array_equal(N(a), N(c))
    assert float(gl1.abs().max()) > 0.0
    # J only: nothing is kept, the old record goes stale all the same
    J3, t0 = h.fine_solve_record(y0, steps, dt, ckpt_every=3, opts=opts, keep=False)
    assert J3 == J1 and t0 == 0 and not h.tape_valid(tape) and not h.tape_valid(0)
    _, tape = h.fine_solve_record(y0, steps, dt, ckpt_every=3, opts=opts)
    h.set_lid(T(lid))
    assert not h.tape_valid(tape)
    with pytest.raises(gpu.NSPError) as e:
        h.fine_solve_reverse(tape)
    assert e.value.status == gpu.NSP_ERR_ARG
    h.close()


def test_autograd_backward_reuses_the_forward_record(gpu):
    """J.backward() reverses the record its forward made: the fine steps run
    in backward are only the segment recomputations (nseg (ck - 1) steps),
    not another forward sweep; a stale record is recorded again."""
    import torch
    from paper_1705_06149_amd.autograd import kinetic_energy

    n, steps, dt, ck = 14, 6, 1e-3, 3
    _say("autograd record reuse", steps)
    h, y0, lid = _small_case(gpu, n)
    opts = gpu.PoissonOpts(rtol=1e-12)
    ref = h.fine_solve_adjoint(y0, steps, dt, ckpt_every=ck, opts=opts)
    cells = n ** 3

    def run(stale):
        u = [y0[c][0].clone().requires_grad_() for c in range(3)]
        lid_t = T(lid).requires_grad_()
        J = kinetic_energy(h, u[0], u[1], u[2], lid_t, steps, dt, ckpt_every=ck, opts=opts)
        if stale:
            h.fine_solve_record(y0, steps, dt, ckpt_every=ck, opts=opts)
        h.launch_stats(reset=True)
        J.backward()
        st = h.launch_stats()
        return float(J.detach()), u, lid_t, st["fine"]["cell_steps"], st["project"]["launches"]

    J, u, lid_t, fine_cells, nproj = run(False)
    assert J == ref[0]
    assert fine_cells == (steps // ck) * (ck - 1) * cells
    assert nproj == steps
    for a, b in zip(u, ref[1]):
        assert np.array_equal(N(a.grad), N(b[0]))
    assert np.array_equal(N(lid_t.grad), N(ref[2]))
    J, u, lid_t, fine_cells, nproj = run(True)
    assert fine_cells == (steps + (steps // ck) * (ck - 1)) * cells
    for a, b in zip(u, ref[1]):
        assert np.array_equal(N(a.grad), N(b[0]))
    h.close()


def test_momentum_adjoint_entry_matches_oracle(gpu, oracle):
    """nsp_momentum_adjoint alone against the oracle's momentum_adjoint on a
    non-cubic grid with obstacles (one under the lid), a random lid, random
    velocities (every SMART branch and both transport signs) and random
    adjoint weights, closed faces holding garbage on input: lam to 1e-12 of
    its max norm, g_lid accumulated onto a nonzero start, bitwise repeat,
    and lam aliasing mu refused."""
    import torch
    nx, ny, nz, dt = 13, 11, 12, 1e-2
    _say("momentum adjoint entry", nx, ny, nz)
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[3:6, 2:5, 4:7] = 1
    solid[7, ny - 2, 2] = 1
    solid[2, 5, nx - 2] = 1
    rng = np.random.default_rng(11)
    lid = 1.0 + 0.3 * rng.standard_normal((nz, nx + 1))
    g = oracle.Grid(nx, ny, nz, re=50.0, solid=solid, lid=lid)
    su, sv, sw, _ = g.shapes()
    vel = [0.5 * rng.standard_normal(s) for s in (su, sv, sw)]
    mu = [rng.standard_normal(s) for s in (su, sv, sw)]
    lam_ref, glid_ref = oracle.momentum_adjoint(g, *vel, dt, mu)
    h = gpu.Handle(nx, ny, nz, re=50.0, solid=solid, max_batch=1)
    h.set_lid(T(lid))
    g0 = rng.standard_normal((nz, nx + 1))
    outs = []
    for _ in range(2):
        lam = tuple(torch.full((1,) + s, 7.0, dtype=torch.float64, device="cuda") for s in (su, sv, sw))
        gl = T(g0)
        h.momentum_adjoint(tuple(T(a) for a in vel), tuple(T(a) for a in mu), lam, dt, gl)
        torch.cuda.synchronize()
        outs.append(([N(a)[0] for a in lam], N(gl)))
    for c in range(3):
        scale = np.abs(lam_ref[c]).max()
        err = np.abs(outs[0][0][c] - lam_ref[c]).max()
        _say("  lam", c, err, scale)
        assert err <= 1e-12 * scale, c
        assert np.array_equal(outs[0][0][c], outs[1][0][c])
    gerr = np.abs(outs[0][1] - (g0 + glid_ref)).max()
    _say("  g_lid", gerr, np.abs(glid_ref).max())
    assert np.abs(glid_ref).max() > 0.0
    assert gerr <= 1e-12 * np.abs(glid_ref).max() + 1e-15 * np.abs(g0).max()
    assert np.array_equal(outs[0][1], outs[1][1])
    m = tuple(T(a) for a in mu)
    with pytest.raises(gpu.NSPError) as e:
        h.momentum_adjoint(tuple(T(a) for a in vel), m, m, dt)
    assert e.value.status == gpu.NSP_ERR_ARG
    h.close()


def test_lid_modes_are_transposes(gpu):
    n, M = 20, 16
    h = gpu.Handle(n, n, n, max_batch=1)
    import torch
    g = torch.Generator(device="cuda").manual_seed(3)
    c = torch.randn((M, M), dtype=torch.float64, device="cuda", generator=g)
    r = torch.randn((n, n + 1), dtype=torch.float64, device="cuda", generator=g)
    lid = h.lid_from_modes(c)
    gc = h.lid_modes_grad(r, M)
    lhs = float(((lid - 1.0) * r).sum())
    rhs = float((c * gc).sum())
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # side walls: every mode vanishes at x = 0 and x = 1
    assert float((lid[:, [0, -1]] - 1.0).abs().max()) < 1e-13
    h.close()


def test_autograd_gradient_matches_finite_differences_full_size(gpu):
    """96^3 cavity, Re 400, 100 steps of 1e-3, divergence-free N(0, 1e-2)
    start, 16x16 lid sine modes with c ~ N(0, 1e-3^2): d J / d u0 and
    d J / d c along random directions against central differences of the
    GPU forward solve (Poisson rtol 1e-12), bar 1e-6."""
    import torch
    from paper_1705_06149_amd.autograd import LidFromModes, kinetic_energy

    n, steps, dt, M = 96, 100, 1e-3, 16
    _say("adjoint full size", n, steps)
    h = gpu.Handle(n, n, n, re=400.0, max_batch=1)
    opts = gpu.PoissonOpts(rtol=1e-12)
    u0 = [T(a).requires_grad_() for a in inputs.div_free_perturbation(n, n, n, seed=5, sigma=1e-2)]
    c = T(np.random.default_rng(6).normal(0.0, 1e-3, (M, M))).requires_grad_()
    lid = LidFromModes.apply(c, h)
    J = kinetic_energy(h, u0[0], u0[1], u0[2], lid, steps, dt, ckpt_every=10, opts=opts)
    J.backward()
    _say("  J", float(J.detach()))
    du = [T(a) for a in inputs.div_free_perturbation(n, n, n, seed=7, sigma=1e-2)]
    gnorm = float(torch.sqrt(sum((g.grad ** 2).sum() for g in u0)))
    dg = [g.grad.detach() * (1e-2 * np.sqrt(sum(a.numel() for a in u0)) / gnorm) for g in u0]
    dc = T(np.random.default_rng(8).normal(0.0, 1e-3, (M, M)))
    pred = {"random": sum(float((g.grad * d).sum()) for g, d in zip(u0, du)),
            "gradient": sum(float((g.grad * d).sum()) for g, d in zip(u0, dg)),
            "lid": float((c.grad * dc).sum())}

    def Jof(us, cc):
        with torch.no_grad():
            return float(kinetic_energy(h, us[0], us[1], us[2], LidFromModes.apply(cc, h), steps, dt, 10, opts))

    # J carries solver noise of ~1e-14 relative (CG to 1e-12), so steps much
    # below 1e-4 are noise-limited; large steps cross SMART branch changes
    errs = {k: [] for k in pred}
    for eps in (1e-3, 3e-4, 1e-4):
        fd = {
            "random": (Jof([a + eps * d for a, d in zip(u0, du)], c) - Jof([a - eps * d for a, d in zip(u0, du)], c))
            / (2 * eps),
            "gradient": (Jof([a + eps * d for a, d in zip(u0, dg)], c) - Jof([a - eps * d for a, d in zip(u0, dg)], c))
            / (2 * eps),
            "lid": (Jof(u0, c + eps * dc) - Jof(u0, c - eps * dc)) / (2 * eps),
        }
        for k in pred:
            errs[k].append(abs(fd[k] - pred[k]) / abs(pred[k]))
            _say("  eps", eps, k, fd[k], pred[k], errs[k][-1])
    assert min(errs["gradient"]) <= 1e-6
    assert min(errs["lid"]) <= 1e-6
    # the random direction is nearly orthogonal to the gradient (its
    # derivative is ~1e-4 of |grad J| |d|): measure its error on that scale
    scale = abs(pred["gradient"])  # = |grad J| |d| since |dg| = |du|
    assert min(errs["random"]) * abs(pred["random"]) <= 1e-6 * scale
    h.close()
