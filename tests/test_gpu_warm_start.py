"""The extrapolated warm start on the GPU (PoissonOpts(extrapolate=True)):
from the second step of a call on, each Poisson solve starts from
2 p^s - p^(s-1) instead of p^s.

- Against the oracle taking the same start (fine_steps(extrapolate=True)):
  velocity to 1e-10 relative L2 and CG iterations within a few per call, on
  flat tiles (32^3) and on the register-resident column tiles (64^3); with
  reliable-update mixed precision to 1e-8, the bound of the other
  mixed-precision parity tests.
- It saves iterations against the plain warm start on the GPU too, with the
  same result to the solver tolerance.
- The register-resident loop equals the streaming one bit for bit, and a
  batch equals its slices run alone, with the option on.
- The adjoint entry points ignore it (their recomputed steps must repeat the
  recorded ones), so a gradient is bitwise the same either way.
"""
import numpy as np
import pytest

from paper_1705_06149_amd import inputs

pytestmark = pytest.mark.gpu

RE, DT = 1000.0, 5e-4


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def T(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _rel(a, b):
    num = np.sqrt(sum(float(np.sum((x - y) ** 2)) for x, y in zip(a, b)))
    den = np.sqrt(sum(float(np.sum(y * y)) for y in b))
    return num / den


@pytest.mark.parametrize("n,dev,steps,prec", [(32, 10, 15, 0), (64, 6, 6, 0), (32, 10, 15, 2)])
def test_matches_oracle_with_the_same_start(gpu, oracle, n, dev, steps, prec):
    _say("extrapolated warm start vs oracle", n, "steps", steps, "prec", prec)
    ru = dict(prec=2, eta=0.01, max_outer=64) if prec == 2 else {}
    g = oracle.Grid(n, n, n, re=RE)
    st0, _, _, s = oracle.fine_steps(g, g.zeros_state(), dev, DT, rtol=1e-10)
    assert s == 0
    ref, it_ref, _, s = oracle.fine_steps(g, st0, steps, DT, rtol=1e-10, extrapolate=True, **ru)
    assert s == 0
    plain_ref_iters = int(oracle.fine_steps(g, st0, steps, DT, rtol=1e-10, **ru)[1].sum())
    h = gpu.Handle(n, n, n, re=RE, max_batch=1)
    h.launch_stats(reset=True)
    y = tuple(T(a[None]) for a in st0)
    opts = (gpu.PoissonOpts(rtol=1e-10, prec=gpu.MIXED_RU, inner_rtol=0.01, max_outer=64, extrapolate=True)
            if prec == 2 else gpu.PoissonOpts(rtol=1e-10, extrapolate=True))
    info = h.fine_step(y, 0.0, steps * DT, DT, opts)
    rr = h.launch_stats()["fine"]["rr_launches"]
    got = [a[0].cpu().numpy() for a in y]
    err = _rel(got[:3], ref[:3])
    _say("  velocity rel L2", err, "iterations gpu", info[0]["iters"], "oracle", int(it_ref.sum()),
         "oracle plain", plain_ref_iters, "register-resident launches", rr)
    assert err <= (1e-10 if prec == 0 else 1e-8)
    assert abs(info[0]["iters"] - int(it_ref.sum())) <= 2 * steps
    assert int(it_ref.sum()) < plain_ref_iters
    if n == 64:
        assert rr == 1  # the register-resident loop took the extrapolated start
    h.close()


def test_saves_iterations_with_the_same_result(gpu):
    n, steps = 64, 10
    _say("extrapolated vs plain warm start on the GPU", n, steps)
    h = gpu.Handle(n, n, n, re=RE, max_batch=1)
    y0 = h.zeros_state(1)
    h.fine_step(y0, 0.0, 10 * DT, DT, gpu.PoissonOpts(rtol=1e-10))
    res = []
    for ex in (False, True):
        y = tuple(a.clone() for a in y0)
        info = h.fine_step(y, 0.0, steps * DT, DT, gpu.PoissonOpts(rtol=1e-10, extrapolate=ex))
        res.append((y, info[0]["iters"]))
    (ya, ia), (yb, ib) = res
    err = _rel([a[0].cpu().numpy() for a in yb[:3]], [a[0].cpu().numpy() for a in ya[:3]])
    _say("  iterations plain", ia, "extrapolated", ib, "velocity rel L2", err)
    assert ib <= 0.9 * ia
    assert err <= 1e-9
    h.close()


def test_rr_equals_streaming_and_batch_equals_single(gpu):
    import torch
    n, steps = 64, 4
    _say("extrapolated warm start: register-resident vs streaming, batch vs single", n)
    opts = gpu.PoissonOpts(rtol=1e-10, extrapolate=True)
    sts = [inputs.random_state(n, n, n, seed=20 + b, scale=0.2, pscale=0.0) for b in range(3)]
    h1 = gpu.Handle(n, n, n, re=RE, max_batch=1)
    res = []
    for wg in (0, 32):
        h1.set_launch(wg)
        h1.launch_stats(reset=True)
        y = tuple(T(a[None]) for a in sts[0])
        h1.fine_step(y, 0.0, steps * 1e-3, 1e-3, opts)
        res.append((y, h1.launch_stats()["fine"]["rr_launches"]))
    (ya, ra), (yb, rb) = res
    assert ra == 1 and rb == 0
    for c in range(4):
        assert torch.equal(ya[c], yb[c]), c
    h1.set_launch(0)
    hb = gpu.Handle(n, n, n, re=RE, max_batch=3)
    yb3 = tuple(T(np.stack([s[c] for s in sts])) for c in range(4))
    hb.fine_step(yb3, 0.0, steps * 1e-3, 1e-3, opts)
    for b in range(3):
        y = tuple(T(a[None]) for a in sts[b])
        hb.fine_step(y, 0.0, steps * 1e-3, 1e-3, opts)
        for c in range(4):
            assert torch.equal(y[c][0], yb3[c][b]), (b, c)
    h1.close()
    hb.close()


def test_adjoint_ignores_the_option(gpu):
    import torch
    n = 16
    _say("adjoint with and without the extrapolate option", n)
    h = gpu.Handle(n, n, n, re=400.0, max_batch=1)
    u0 = inputs.div_free_perturbation(n, n, n, seed=5, sigma=1e-2)
    y0 = tuple(T(a[None]) for a in u0) + (torch.zeros((1, n, n, n), dtype=torch.float64, device="cuda"),)
    out = []
    for ex in (False, True):
        J, g, gl = h.fine_solve_adjoint(y0, 8, 1e-3, ckpt_every=4,
                                        opts=gpu.PoissonOpts(rtol=1e-12, extrapolate=ex))
        out.append((J, g, gl))
    assert out[0][0] == out[1][0]
    for a, b in zip(out[0][1], out[1][1]):
        assert torch.equal(a, b)
    assert torch.equal(out[0][2], out[1][2])
    h.close()
