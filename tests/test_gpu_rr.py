"""Register-resident CG on the GPU: when a launch has no more CG column
tiles than workgroups, each workgroup keeps its tile's CG vectors in
registers for the whole solve and exchanges only tile-boundary values
through memory.  It computes the streaming kernel's values with the same
formulas and the same partial-sum blocks, so its results must equal the
streaming kernel's bit for bit; the streaming kernel is forced by a launch
with fewer workgroups than tiles.  Parity with the oracle is covered by the
parity tests, which run the register-resident path at 64^3, 96^3 and 128^3.
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


CASES = [(128, None, False), (96, None, True), (64, 5, False)]


def _opts(gpu, prec, rtol=1e-10):
    if prec == 2:  # reliable updates: the loop pauses in registers for each update
        return gpu.PoissonOpts(rtol=rtol, prec=prec, inner_rtol=0.01, max_outer=64)
    return gpu.PoissonOpts(rtol=rtol, prec=prec, inner_rtol=1e-5)


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("n,seed,periodic", CASES)
def test_rr_steps_equal_streaming(gpu, n, seed, periodic, prec):
    import torch
    _say("register-resident vs streaming", n, "obstacles seed", seed, "periodic", periodic, "prec", prec)
    solid = inputs.obstacle_mask(n, seed) if seed else None
    h = gpu.Handle(n, n, n, re=1000.0, solid=solid, periodic_z=periodic, max_batch=1)
    st = inputs.random_state(n, n, n, seed=3, scale=0.2, pscale=0.0)
    if periodic:
        st = (st[0], st[1], np.concatenate([st[2][:-1], st[2][:1]], axis=0), st[3])
    opts = _opts(gpu, prec)
    res = []
    for wg in (0, 32):
        h.set_launch(wg)
        h.launch_stats(reset=True)
        y = tuple(T(a[None]) for a in st)
        info = h.fine_step(y, 0.0, 0.002, 1e-3, opts)
        stats = h.launch_stats()["fine"]
        res.append((y, info, stats["rr_launches"]))
        _say("  workgroups", wg, "register-resident launches", stats["rr_launches"], "iters", info[0]["iters"])
    (ya, ia, ra), (yb, ib, rb) = res
    assert ra == 1 and rb == 0
    for c in range(4):
        assert torch.equal(ya[c], yb[c]), c
    assert ia == ib
    h.set_launch(0)
    h.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_rr_poisson_equals_streaming_with_cold_start(gpu, prec):
    """Poisson solves (one with a warm start worse than none) in registers
    and streaming, bitwise."""
    import torch
    n = 64
    _say("register-resident poisson", n, "prec", prec)
    h = gpu.Handle(n, n, n, max_batch=2)
    rng = np.random.default_rng(9)
    b = T(rng.standard_normal((2, n, n, n)))
    p0 = T(np.stack([rng.standard_normal((n, n, n)) * 1e-4, rng.standard_normal((n, n, n)) * 1e4]))
    opts = _opts(gpu, prec, 1e-11)
    out = []
    for wg in (0, 32):
        h.set_launch(wg)
        h.launch_stats(reset=True)
        p = p0.clone()
        info = h.poisson_solve(b, p, opts)
        out.append((p, info, h.launch_stats()["poisson"]["rr_launches"]))
    assert out[0][2] == 1 and out[1][2] == 0
    assert torch.equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]
    h.set_launch(0)
    h.close()
