"""Repeatability on the GPU (the library's race detector: every reduction has a
fixed order and no floating-point atomics feed a result): the same call on
the same inputs twice gives bitwise the same outputs, for the FP64, mixed and
BiCGStab solves, a projection step with obstacles and the adjoint gradient;
and a Parareal run
saved after iteration k (Y, Gk and k through torch.save) and resumed in a new
handle finishes bitwise like the uninterrupted run."""
import io

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


@pytest.mark.parametrize("prec,solver", [(0, 0), (1, 0), (0, 1), (0, 2), (2, 0)])
def test_repeat_runs_are_bitwise_equal(gpu, prec, solver):
    n = 64
    _say("repeat runs", n, "prec", prec, "solver", solver)
    solid = inputs.obstacle_mask(n, 5)
    h = gpu.Handle(n, n, n, re=1000.0, solid=solid, max_batch=2)
    st = inputs.random_state(n, n, n, seed=2, scale=0.2, pscale=0.0)
    opts = gpu.PoissonOpts(rtol=1e-10, prec=prec, solver=solver, inner_rtol=0.01 if prec == 2 else 1e-5,
                           max_outer=64 if prec == 2 else 8)
    outs = []
    for rep in range(2):
        y = tuple(T(np.stack([a, a[::-1].copy()])) for a in st)
        info = h.fine_step(y, 0.0, 0.003, 1e-3, opts)
        outs.append(([N(a) for a in y], [x["iters"] for x in info]))
    for c in range(4):
        assert np.array_equal(outs[0][0][c], outs[1][0][c]), c
    assert outs[0][1] == outs[1][1]
    h.close()


def test_adjoint_gradients_repeat_bitwise(gpu):
    """The momentum adjoint is a gather without atomics: two gradient
    computations from the same state give bitwise equal J, dJ/du0 and
    dJ/dlid."""
    n, steps, dt = 64, 4, 1e-3
    _say("adjoint repeat", n, steps)
    solid = inputs.obstacle_mask(n, 5)
    h = gpu.Handle(n, n, n, re=400.0, solid=solid, max_batch=1)
    lid = 1.0 + 0.1 * np.random.default_rng(4).standard_normal((n, n + 1))
    h.set_lid(T(lid))
    st = inputs.random_state(n, n, n, seed=3, scale=0.2, pscale=0.0)
    y0 = tuple(T(a[None]) for a in st)
    outs = [h.fine_solve_adjoint(y0, steps, dt, ckpt_every=2, opts=gpu.PoissonOpts(rtol=1e-12)) for _ in range(2)]
    assert outs[0][0] == outs[1][0]
    for a, b in zip(outs[0][1] + (outs[0][2],), outs[1][1] + (outs[1][2],)):
        assert np.array_equal(N(a), N(b))
    assert float(outs[0][2].abs().max()) > 0.0
    h.close()


def test_parareal_resume_after_save(gpu):
    import torch
    n, Ns, dt, DT, T_end = 16, 4, 1e-3, 2e-3, 0.016
    _say("parareal save / resume", n, Ns)
    y0 = inputs.random_state(n, n, n, seed=6, scale=0.1, pscale=0.0)
    opts = gpu.PoissonOpts(rtol=1e-11)

    def fresh():
        h = gpu.Handle(n, n, n, re=250.0, max_batch=Ns)
        Y = tuple(T(np.stack([a] * (Ns + 1))) for a in y0)
        Fk = tuple(T(np.zeros((Ns,) + a.shape)) for a in y0)
        Gk = tuple(T(np.zeros((Ns,) + a.shape)) for a in y0)
        return h, Y, Fk, Gk

    h, Y, Fk, Gk = fresh()
    h.parareal_start(Y, Gk, Ns, 0.0, T_end, DT, opts)
    jumps = []
    for k in range(3):
        jumps.append(h.parareal_iterate(Y, Fk, Gk, Ns, k, 0.0, T_end, dt, DT, opts, opts))
    ref = [N(a) for a in Y]
    h.close()

    h, Y, Fk, Gk = fresh()
    h.parareal_start(Y, Gk, Ns, 0.0, T_end, DT, opts)
    h.parareal_iterate(Y, Fk, Gk, Ns, 0, 0.0, T_end, dt, DT, opts, opts)
    buf = io.BytesIO()
    torch.save({"Y": [a.cpu() for a in Y], "Gk": [a.cpu() for a in Gk], "k": 1}, buf)
    h.close()
    buf.seek(0)
    saved = torch.load(buf, weights_only=True)
    h, Y, Fk, Gk = fresh()
    for dst, src in zip(Y, saved["Y"]):
        dst.copy_(src.cuda())
    for dst, src in zip(Gk, saved["Gk"]):
        dst.copy_(src.cuda())
    res = []
    for k in range(saved["k"], 3):
        res.append(h.parareal_iterate(Y, Fk, Gk, Ns, k, 0.0, T_end, dt, DT, opts, opts))
    assert res == jumps[1:]
    for a, b in zip(Y, ref):
        assert np.array_equal(N(a), b)
    h.close()


def test_maximum_batch_of_64_slices(gpu):
    """A launch with the maximum of 64 slices (random states on a ragged
    20 x 18 x 14 grid with obstacles): every sampled slice equals its
    single-slice launch bitwise; 65 slices are refused."""
    nx, ny, nz, B = 20, 18, 14, 64
    _say("maximum batch", B)
    from scipy import ndimage
    solid = np.ascontiguousarray(inputs.obstacle_mask(20, 4, frac=0.05, smin=2, smax=4)[:nz, :ny, :nx])
    lab, _ = ndimage.label(solid == 0)
    top = np.unique(lab[:, ny - 1, :])
    solid[~np.isin(lab, top[top > 0])] = 1
    h = gpu.Handle(nx, ny, nz, re=300.0, solid=solid, max_batch=B)
    sts = [inputs.random_state(nx, ny, nz, seed=100 + b, scale=0.2, pscale=0.0) for b in range(B)]
    y = tuple(T(np.stack([s[c] for s in sts])) for c in range(4))
    opts = gpu.PoissonOpts(rtol=1e-10)
    h.fine_step(y, 0.0, 0.002, 1e-3, opts)
    for b in (0, 37, 63):
        y1 = tuple(T(a[None]) for a in sts[b])
        h.fine_step(y1, 0.0, 0.002, 1e-3, opts)
        for c in range(4):
            assert np.array_equal(N(y[c])[b], N(y1[c])[0]), (b, c)
    h.close()
    with pytest.raises(gpu.NSPError):
        gpu.Handle(nx, ny, nz, max_batch=B + 1)
