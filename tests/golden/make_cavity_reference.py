"""Write the oracle's serial FP64 reference of a full-size cavity workload.

Cases (lid-driven cavity on the unit cube, Re = 1000, lid u = 1, start from
rest as in Sec. 3, fine step dt = 5e-4, Jacobi-PCG to ||r|| <= 1e-10 ||b||):

  c3: 96^3 up to T = 0.64 (1280 projection steps), the Parareal workload.
      Parareal converges to the serial fine solution (Sec. 2.1.2, Eqs.
      (6)-(7)), so this run is what the GPU's Parareal end state is checked
      against.
  c2: 128^3 up to T = 0.1 (200 steps), the FP64 / mixed-precision workload.
  c4_64: the 64^3 grid of the obstacle batch, with its seeded cuboid
      obstacles (seed 1; no-slip), up to T = 0.32 (640 steps): the
      reference of that grid's Parareal end state.

Only the oracle runs here.  The file written holds, per component u, v, w,
p: 16384 flat indices drawn with a fixed seed and the end-state values
there, the L2 and max norms of the whole component, and the CG iterations of
every step.  Usage:

    python tests/golden/make_cavity_reference.py --case c3|c2|c4_64 [--checkpoint FILE]

With --checkpoint the state is saved every 40 steps and a rerun resumes from
it.  A full run takes hours on a few CPU cores.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1705_06149_amd import inputs  # noqa: E402  (the seeded obstacle mask only)

# n, Re, dt, T, obstacle seed (None: empty cavity), file
CASES = {
    "c3": (96, 1000.0, 5e-4, 0.64, None, "c3_cavity96_re1000_T064_fp64.npz"),
    "c2": (128, 1000.0, 5e-4, 0.1, None, "c2_cavity128_re1000_T01_fp64.npz"),
    "c4_64": (64, 1000.0, 5e-4, 0.32, 1, "c4_obstacles64_seed1_re1000_T032_fp64.npz"),
}
RTOL = 1e-10
NSAMPLE, SEED = 16384, 20170518


def sample_indices(shapes):
    rng = np.random.default_rng(SEED)
    return [np.sort(rng.choice(int(np.prod(s)), size=NSAMPLE, replace=False)).astype(np.int64) for s in shapes]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", choices=sorted(CASES), default="c3")
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--chunk", type=int, default=40)
    a = ap.parse_args()
    N, RE, DT, T, oseed, name = CASES[a.case]
    NSTEPS = int(round(T / DT))
    OUT = os.path.join(HERE, name)
    solid = inputs.obstacle_mask(N, oseed) if oseed is not None else None
    g = O.Grid(N, N, N, re=RE, solid=solid)
    state, step, iters = g.zeros_state(), 0, []
    if a.checkpoint and os.path.exists(a.checkpoint):
        z = np.load(a.checkpoint)
        state = tuple(z[k] for k in ("u", "v", "w", "p"))
        step, iters = int(z["step"]), list(z["iters"])
        print("resumed at step %d" % step, flush=True)
    t0 = time.time()
    while step < NSTEPS:
        n = min(a.chunk, NSTEPS - step)
        state, it, rel, st = O.fine_steps(g, state, n, DT, rtol=RTOL)
        if st != 0:
            raise RuntimeError("oracle step failed with status %d at step %d" % (st, step))
        step += n
        iters += [int(x) for x in it]
        print("step %d/%d  CG iterations of the last %d steps: %d  (%.0f s)"
              % (step, NSTEPS, n, int(np.sum(it)), time.time() - t0), flush=True)
        if a.checkpoint:
            tmp = a.checkpoint + ".tmp.npz"
            np.savez(tmp, u=state[0], v=state[1], w=state[2], p=state[3], step=step, iters=np.array(iters))
            os.replace(tmp, a.checkpoint)
    idx = sample_indices(g.shapes())
    out = dict(n=N, re=RE, dt=DT, T=T, rtol=RTOL, nsteps=NSTEPS, seed=SEED, iters=np.array(iters, np.int32),
               obstacle_seed=-1 if oseed is None else oseed)
    for name, arr, ix in zip("uvwp", state, idx):
        out["idx_" + name] = ix
        out["val_" + name] = arr.ravel()[ix]
        out["l2_" + name] = float(np.sqrt(np.sum(arr * arr)))
        out["max_" + name] = float(np.max(np.abs(arr)))
    np.savez_compressed(OUT, **out)
    print("wrote", OUT, os.path.getsize(OUT), "bytes", flush=True)


if __name__ == "__main__":
    main()
