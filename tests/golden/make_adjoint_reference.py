"""Write the oracle's gradient of the full-size adjoint workload.

The workload: 96^3 lid-driven cavity, Re = 400, 100 fine steps of 1e-3
(Sec. 2 projection step, Jacobi-PCG to 1e-12), objective J = kinetic energy
at T (1/2 hx hy hz sum over open faces of u^2 + v^2 + w^2); the initial
velocity is the seeded divergence-free perturbation of face standard
deviation 1e-2 (seed 5), the lid is 1 + sum over m, n = 1..16 of
c_mn sin(m pi x) sin(n pi z) with c ~ N(0, 1e-3^2) (seed 6).  Only the
oracle runs here (its adjoint_gradient keeps every forward state).

The file written holds J; dJ/d(u0, v0, w0) at 16384 seeded sample points per
component with the max norm of each; dJ/dlid at every top u-face position;
dJ/dc (16 x 16, the lid gradient projected on the sine basis).  Usage:

    python tests/golden/make_adjoint_reference.py

It takes about an hour on 8 CPU cores (measured: 57 min) and 3 GB of memory.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1705_06149_amd import inputs  # noqa: E402

N, RE, DT, NSTEPS, M = 96, 400.0, 1e-3, 100, 16
NSAMPLE, SEED = 16384, 20170518
OUT = os.path.join(HERE, "c5_adjoint96_re400_100steps.npz")


def main():
    O.build()
    coef = np.random.default_rng(6).normal(0.0, 1e-3, (M, M))
    basis = inputs.lid_profile_basis(N, N, M)
    lid = 1.0 + np.tensordot(coef, basis, axes=([0, 1], [0, 1]))
    g = O.Grid(N, N, N, re=RE, lid=lid)
    u0 = inputs.div_free_perturbation(N, N, N, seed=5, sigma=1e-2)
    st0 = (u0[0], u0[1], u0[2], np.zeros((N, N, N)))
    t0 = time.time()
    J, grad, glid = O.adjoint_gradient(g, st0, NSTEPS, DT, rtol=1e-12, ckpt_every=None)
    print("adjoint gradient done in %.0f s, J = %.17g" % (time.time() - t0, J), flush=True)
    gcoef = np.tensordot(basis, glid, axes=([2, 3], [0, 1]))
    rng = np.random.default_rng(SEED)
    out = dict(n=N, re=RE, dt=DT, nsteps=NSTEPS, nmodes=M, seed=SEED, J=J, glid=glid, gcoef=gcoef)
    for name, a in zip("uvw", grad):
        idx = np.sort(rng.choice(a.size, size=NSAMPLE, replace=False)).astype(np.int64)
        out["idx_" + name] = idx
        out["val_" + name] = a.ravel()[idx]
        out["max_" + name] = float(np.max(np.abs(a)))
        out["l2_" + name] = float(np.sqrt(np.sum(a * a)))
    np.savez_compressed(OUT, **out)
    print("wrote", OUT, os.path.getsize(OUT), "bytes", flush=True)


if __name__ == "__main__":
    main()
