"""The 128^3 FP64 / mixed-precision workload at full size against the
oracle's serial FP64 run: lid-driven cavity, Re 1000, from rest, 200
projection steps of 5e-4, Jacobi-PCG to 1e-10.  The reference (tests/golden/
c2_cavity128_re1000_T01_fp64.npz, written by make_cavity_reference.py with
the oracle alone) holds 16384 seeded sample points per component and the L2
and max norms of the whole end state.

- The GPU's FP64 run matches it to 1e-10 (sampled relative L2 of velocity,
  and each component's max sample error over its max norm).
- The mixed-precision runs (FP32 inner CG with FP64 defect correction: with
  restarts, and with reliable updates) reach the same 1e-10 residual, so
  they match it to 1e-8; the measured errors are printed.
- The FP64 run with the extrapolated warm start (the fine benchmark's
  setting; 50 steps per call) solves the same equations to the same
  tolerance from another start, so it matches it to 1e-10 as well.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
REF = os.path.join(HERE, "golden", "c2_cavity128_re1000_T01_fp64.npz")
N, RE, DT, STEPS = 128, 1000.0, 5e-4, 200


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _errors(z, state):
    """sampled relative L2 of (u, v, w); per component max sample error over
    its max norm, and L2-norm difference over the L2 norm"""
    num = den = 0.0
    out = {}
    for c, name in enumerate("uvwp"):
        a = state[c].detach().cpu().numpy().ravel()
        idx, val = z["idx_" + name], z["val_" + name]
        d = a[idx] - val
        if c < 3:
            num += float(np.sum(d * d))
            den += float(np.sum(val * val))
        out[name] = (float(np.max(np.abs(d))) / float(z["max_" + name]),
                     abs(float(np.linalg.norm(a)) - float(z["l2_" + name])) / float(z["l2_" + name]))
    out["vel_rel_l2"] = (num / den) ** 0.5
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_ru", "fp64_extrapolated"])
def test_128_cavity_200_steps_matches_oracle(gpu, prec):
    if not os.path.exists(REF):
        pytest.skip("the oracle reference %s has not been generated" % os.path.basename(REF))
    z = np.load(REF)
    assert int(z["n"]) == N and float(z["re"]) == RE and float(z["dt"]) == DT and int(z["nsteps"]) == STEPS
    _say("c2", prec, N, STEPS)
    opts = {"fp64": gpu.PoissonOpts(rtol=1e-10, prec=gpu.FP64),
            "fp64_extrapolated": gpu.PoissonOpts(rtol=1e-10, prec=gpu.FP64, extrapolate=True),
            "mixed": gpu.PoissonOpts(rtol=1e-10, prec=gpu.MIXED, inner_rtol=1e-5, max_outer=8),
            "mixed_ru": gpu.PoissonOpts(rtol=1e-10, prec=gpu.MIXED_RU, inner_rtol=0.01, max_outer=64)}[prec]
    h = gpu.Handle(N, N, N, re=RE, max_batch=1)
    y = h.zeros_state(1)
    for s in range(4):
        h.fine_step(y, s * STEPS * DT / 4, (s + 1) * STEPS * DT / 4, DT, opts)
    err = _errors(z, tuple(a[0] for a in y))
    _say("  errors", err)
    tol = 1e-10 if prec.startswith("fp64") else 1e-8
    assert err["vel_rel_l2"] <= tol
    for name in "uvwp":
        assert err[name][0] <= tol, name
        assert err[name][1] <= tol, name
    h.close()
