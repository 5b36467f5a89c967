"""Plain FP64 CPU oracle: Python side.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg import this module; the product path
(``paper_1705_06149_amd``) never does, and this module imports nothing from
it.  The arithmetic of the projection step lives in ``nsp_oracle.c`` (plain
C, built here with gcc, ``-ffp-contract=off``); this file marshals NumPy
arrays into it and writes out the Parareal iteration of Eq. (6) of
Croce, Ruprecht & Krause (Sec. 2.1.2) in NumPy.

Array layout (x fastest, NumPy C order):
    u: (nz, ny, nx+1)   v: (nz, ny+1, nx)   w: (nz+1, ny, nx)   p: (nz, ny, nx)
    solid: (nz, ny, nx) uint8, nonzero = solid      lid: (nz, nx+1)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nsp_oracle.c")
_LIB = os.path.join(_HERE, "libnsp_oracle.so")


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
                ("re", ctypes.c_double), ("solid", ctypes.c_void_p), ("lid", ctypes.c_void_p),
                ("periodic_z", ctypes.c_int), ("slip_obstacles", ctypes.c_int), ("upwind", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer", ctypes.c_int), ("status", ctypes.c_int),
                ("rel_res_true", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        D = ctypes.c_double
        I = ctypes.c_int
        G = ctypes.POINTER(_Grid)
        _lib.og_smart.argtypes = [D, D, D]
        _lib.og_smart.restype = D
        _lib.og_momentum.argtypes = [G, P, P, P, D, P, P, P]
        _lib.og_momentum_branches.argtypes = [G, P, P, P, P, P, P]
        _lib.og_divergence.argtypes = [G, P, P, P, P]
        _lib.og_gradient.argtypes = [G, P, P, P, P]
        _lib.og_apply_A.argtypes = [G, P, P]
        _lib.og_pcg.argtypes = [G, P, P, D, I, ctypes.POINTER(_Info)]
        _lib.og_pcg.restype = I
        _lib.og_pcg_mixed.argtypes = [G, P, P, D, D, I, I, ctypes.POINTER(_Info)]
        _lib.og_pcg_mixed.restype = I
        _lib.og_correct.argtypes = [G, P, P, P, P, D, P, P, P]
        _lib.og_rhs.argtypes = [G, P, P, P, D, P]
        _lib.og_fine_steps.argtypes = [G, P, P, P, P, I, D, I, D, I, D, I, P, P]
        _lib.og_fine_steps.restype = I
        _lib.og_fine_steps_solver.argtypes = [G, P, P, P, P, I, D, I, I, D, I, D, I, P, P]
        _lib.og_fine_steps_solver.restype = I
        _lib.og_fine_steps_ex.argtypes = [G, P, P, P, P, I, D, I, I, D, I, D, I, I, P, P]
        _lib.og_fine_steps_ex.restype = I
        _lib.og_bicgstab.argtypes = [G, P, P, D, I, ctypes.POINTER(_Info)]
        _lib.og_bicgstab.restype = I
        _lib.og_pcg_sr.argtypes = [G, P, P, D, I, ctypes.POINTER(_Info)]
        _lib.og_pcg_sr.restype = I
        _lib.og_pcg_mixed_ru.argtypes = [G, P, P, D, D, I, I, ctypes.POINTER(_Info)]
        _lib.og_pcg_mixed_ru.restype = I
        _lib.og_num_threads.restype = I
        _lib.og_set_num_threads.argtypes = [I]
        _lib.og_momentum_adjoint.argtypes = [G, P, P, P, D, P, P, P, P, P, P, P]
        _lib.og_stencil_form_value.argtypes = [G, I, P, I, I, I, I, I]
        _lib.og_stencil_form_value.restype = D
        _lib.og_stencil_value.argtypes = [G, I, P, I, I, I, I, I]
        _lib.og_stencil_value.restype = D
    return _lib


@dataclass
class Grid:
    """Uniform staggered grid on [0,lx]x[0,ly]x[0,lz], y vertical."""
    nx: int
    ny: int
    nz: int
    lx: float = 1.0
    ly: float = 1.0
    lz: float = 1.0
    re: float = 100.0
    solid: np.ndarray | None = None
    lid: np.ndarray | None = None
    periodic_z: bool = False
    slip_obstacles: bool = False
    upwind: bool = False  # first-order upwind (donor-cell) convection instead of SMART
    _keep: list = field(default_factory=list, repr=False)

    def __post_init__(self):
        if self.solid is not None:
            self.solid = np.ascontiguousarray(self.solid, dtype=np.uint8)
            assert self.solid.shape == (self.nz, self.ny, self.nx)
        if self.lid is None:
            self.lid = np.ones((self.nz, self.nx + 1))
        self.lid = np.ascontiguousarray(self.lid, dtype=np.float64)
        assert self.lid.shape == (self.nz, self.nx + 1)

    @property
    def h(self):
        return (self.lx / self.nx, self.ly / self.ny, self.lz / self.nz)

    def c(self) -> _Grid:
        hx, hy, hz = self.h
        g = _Grid(self.nx, self.ny, self.nz, hx, hy, hz, float(self.re),
                  self.solid.ctypes.data if self.solid is not None else None, self.lid.ctypes.data,
                  1 if self.periodic_z else 0, 1 if self.slip_obstacles else 0, 1 if self.upwind else 0)
        return g

    def shapes(self):
        nx, ny, nz = self.nx, self.ny, self.nz
        return (nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx), (nz, ny, nx)

    def zeros_state(self):
        return tuple(np.zeros(s) for s in self.shapes())

    def fluid(self):
        if self.solid is None:
            return np.ones((self.nz, self.ny, self.nx), dtype=bool)
        return self.solid == 0


def _p(a):
    assert a.flags.c_contiguous
    return a.ctypes.data


def _chk(a, shape, dtype=np.float64):
    a = np.ascontiguousarray(a, dtype=dtype)
    assert a.shape == tuple(shape), (a.shape, shape)
    return a


def num_threads():
    """Threads the oracle's OpenMP loops use."""
    return int(lib().og_num_threads())


def set_num_threads(n):
    lib().og_set_num_threads(int(n))


def smart(U, C, D):
    return lib().og_smart(float(U), float(C), float(D))


def momentum(g: Grid, u, v, w, dt):
    su, sv, sw, _ = g.shapes()
    u, v, w = _chk(u, su), _chk(v, sv), _chk(w, sw)
    Fu, Fv, Fw = np.empty(su), np.empty(sv), np.empty(sw)
    gc = g.c()
    lib().og_momentum(ctypes.byref(gc), _p(u), _p(v), _p(w), float(dt), _p(Fu), _p(Fv), _p(Fw))
    return Fu, Fv, Fw


def momentum_branches(g: Grid, u, v, w):
    """The branch every convective flux of the predictor takes at (u, v, w):
    per component an int8 array of the face array's shape plus a last axis
    of 6 (direction d, side -1/+1 at 2 d, 2 d + 1); 0 for a zero transport
    velocity, else 1 + (velocity < 0) + 2 * SMART segment; -1 on closed
    faces."""
    su, sv, sw, _ = g.shapes()
    u, v, w = _chk(u, su), _chk(v, sv), _chk(w, sw)
    out = [np.empty(s + (6,), dtype=np.int8) for s in (su, sv, sw)]
    gc = g.c()
    lib().og_momentum_branches(ctypes.byref(gc), _p(u), _p(v), _p(w), _p(out[0]), _p(out[1]), _p(out[2]))
    return out


def divergence(g: Grid, u, v, w):
    su, sv, sw, sp = g.shapes()
    u, v, w = _chk(u, su), _chk(v, sv), _chk(w, sw)
    out = np.empty(sp)
    gc = g.c()
    lib().og_divergence(ctypes.byref(gc), _p(u), _p(v), _p(w), _p(out))
    return out


def gradient(g: Grid, p):
    su, sv, sw, sp = g.shapes()
    p = _chk(p, sp)
    Gu, Gv, Gw = np.empty(su), np.empty(sv), np.empty(sw)
    gc = g.c()
    lib().og_gradient(ctypes.byref(gc), _p(p), _p(Gu), _p(Gv), _p(Gw))
    return Gu, Gv, Gw


def apply_A(g: Grid, p):
    sp = g.shapes()[3]
    p = _chk(p, sp)
    q = np.empty(sp)
    gc = g.c()
    lib().og_apply_A(ctypes.byref(gc), _p(p), _p(q))
    return q


def rhs(g: Grid, Fu, Fv, Fw, dt):
    su, sv, sw, sp = g.shapes()
    b = np.empty(sp)
    gc = g.c()
    lib().og_rhs(ctypes.byref(gc), _p(_chk(Fu, su)), _p(_chk(Fv, sv)), _p(_chk(Fw, sw)), float(dt), _p(b))
    return b


def pcg(g: Grid, b, x0=None, rtol=1e-10, maxit=100000):
    sp = g.shapes()[3]
    b = _chk(b, sp)
    x = np.zeros(sp) if x0 is None else _chk(x0, sp).copy()
    info = _Info()
    gc = g.c()
    lib().og_pcg(ctypes.byref(gc), _p(b), _p(x), float(rtol), int(maxit), ctypes.byref(info))
    return x, dict(iters=info.iters, outer=info.outer, status=info.status, rel_res_true=info.rel_res_true)


def bicgstab(g: Grid, b, x0=None, rtol=1e-10, maxit=100000):
    """FP64 Jacobi-preconditioned BiCGStab, the paper's pressure solver (Sec. 2)."""
    sp = g.shapes()[3]
    b = _chk(b, sp)
    x = np.zeros(sp) if x0 is None else _chk(x0, sp).copy()
    info = _Info()
    gc = g.c()
    lib().og_bicgstab(ctypes.byref(gc), _p(b), _p(x), float(rtol), int(maxit), ctypes.byref(info))
    return x, dict(iters=info.iters, outer=info.outer, status=info.status, rel_res_true=info.rel_res_true)


def pcg_sr(g: Grid, b, x0=None, rtol=1e-10, maxit=100000):
    """FP64 Jacobi-PCG with one merged inner-product stage per iteration
    (Chronopoulos & Gear): the same Krylov iterates as pcg in exact
    arithmetic."""
    sp = g.shapes()[3]
    b = _chk(b, sp)
    x = np.zeros(sp) if x0 is None else _chk(x0, sp).copy()
    info = _Info()
    gc = g.c()
    lib().og_pcg_sr(ctypes.byref(gc), _p(b), _p(x), float(rtol), int(maxit), ctypes.byref(info))
    return x, dict(iters=info.iters, outer=info.outer, status=info.status, rel_res_true=info.rel_res_true)


def pcg_mixed(g: Grid, b, x0=None, rtol=1e-10, eta=1e-5, maxit=100000, max_outer=8):
    sp = g.shapes()[3]
    b = _chk(b, sp)
    x = np.zeros(sp) if x0 is None else _chk(x0, sp).copy()
    info = _Info()
    gc = g.c()
    lib().og_pcg_mixed(ctypes.byref(gc), _p(b), _p(x), float(rtol), float(eta), int(maxit), int(max_outer),
                       ctypes.byref(info))
    return x, dict(iters=info.iters, outer=info.outer, status=info.status, rel_res_true=info.rel_res_true)


def pcg_mixed_ru(g: Grid, b, x0=None, rtol=1e-10, delta=0.1, maxit=100000, max_updates=64):
    """FP32 Jacobi-PCG on the correction with reliable updates: the FP64
    residual replaces the FP32 one whenever it has fallen by `delta`, and the
    search direction is kept.  outer = number of updates."""
    sp = g.shapes()[3]
    b = _chk(b, sp)
    x = np.zeros(sp) if x0 is None else _chk(x0, sp).copy()
    info = _Info()
    gc = g.c()
    lib().og_pcg_mixed_ru(ctypes.byref(gc), _p(b), _p(x), float(rtol), float(delta), int(maxit), int(max_updates),
                          ctypes.byref(info))
    return x, dict(iters=info.iters, outer=info.outer, status=info.status, rel_res_true=info.rel_res_true)


def correct(g: Grid, Fu, Fv, Fw, p, dt):
    su, sv, sw, sp = g.shapes()
    u, v, w = np.empty(su), np.empty(sv), np.empty(sw)
    gc = g.c()
    lib().og_correct(ctypes.byref(gc), _p(_chk(Fu, su)), _p(_chk(Fv, sv)), _p(_chk(Fw, sw)), _p(_chk(p, sp)),
                     float(dt), _p(u), _p(v), _p(w))
    return u, v, w


def fine_steps(g: Grid, state, nsteps, dt, prec=0, rtol=1e-10, maxit=100000, eta=1e-5, max_outer=8, solver=0,
               extrapolate=False):
    """nsteps projection steps of size dt; returns (new state, iters, rel_true, status).
    solver 0: Jacobi-PCG (prec 0 FP64, 1 mixed restarts, 2 mixed reliable
    updates with eta = delta and max_outer = update limit); 1: FP64
    Jacobi-BiCGStab; 2: single-reduction Jacobi-PCG (FP64).  extrapolate:
    from the second step of the call on, each Poisson solve starts from
    2 p^s - p^(s-1) instead of p^s (same equation and stopping test).

    The input state tuple (u, v, w, p) is not modified."""
    su, sv, sw, sp = g.shapes()
    u, v, w, p = (_chk(a, s).copy() for a, s in zip(state, (su, sv, sw, sp)))
    iters = np.zeros(max(nsteps, 1), dtype=np.int32)
    rel = np.zeros(max(nsteps, 1))
    gc = g.c()
    st = lib().og_fine_steps_ex(ctypes.byref(gc), _p(u), _p(v), _p(w), _p(p), int(nsteps), float(dt),
                                int(prec), int(solver), float(rtol), int(maxit), float(eta), int(max_outer),
                                int(bool(extrapolate)), _p(iters), _p(rel))
    return (u, v, w, p), iters[:nsteps], rel[:nsteps], st


def propagate(g: Grid, state, t0, t1, step, **opts):
    """F or G of the paper: integrate from t0 to t1 with steps of size `step`.

    The number of steps (t1 - t0)/step must be an integer (Eq. (5) asks the
    same of the coarse/fine ratio)."""
    n = (t1 - t0) / step
    ns = int(round(n))
    if ns < 0 or abs(n - ns) > 1e-9 * max(1.0, abs(n)):
        raise ValueError("(t1-t0)/step = %r is not an integer" % n)
    out, iters, rel, st = fine_steps(g, state, ns, step, **opts)
    if st != 0:
        raise RuntimeError("oracle solve failed with status %d" % st)
    return out


# ------------------------------------------------------------------ Parareal

def parareal(y0, nslices, F, G, n_it=None, tol=None, jump_norm=None, combine=None):
    """Parareal, Eq. (6): y^{k+1}_{n+1} = G(y^{k+1}_n) + F(y^k_n) - G(y^k_n).

    y0: initial value (any object; states are tuples of arrays or scalars).
    F(y, n), G(y, n): fine / coarse propagator over slice n.
    The correction is evaluated as F + (G_new - G_old), so an unchanged coarse
    input gives a correction of exactly zero.
    Iterates until k+1 == n_it, until the jump max_n |y^{k+1}_{n+1} - y^k_{n+1}|
    is below tol, or until k+1 == nslices (then every slice is exact).
    Returns (Y, history) with Y[n] the slice-end values (Y[0] = y0) and
    history a list of dicts with the jump of each iteration.
    """
    if combine is None:
        def combine(f, gn, go):
            if isinstance(f, tuple):
                return tuple(a + (b - c) for a, b, c in zip(f, gn, go))
            return f + (gn - go)
    if jump_norm is None:
        def jump_norm(a, b):
            if isinstance(a, tuple):
                return max(float(np.max(np.abs(x - y))) if np.size(x) else 0.0 for x, y in zip(a, b))
            return float(abs(a - b))
    N = nslices
    Y = [y0]
    Gold = []
    for n in range(N):  # initial coarse sweep
        g = G(Y[n], n)
        Gold.append(g)
        Y.append(g)
    history = [dict(k=-1, jump=None, Y=list(Y))]
    k = 0
    while True:
        Fk = [F(Y[n], n) for n in range(N)]
        Ynew = [y0]
        Gnew = []
        for n in range(N):
            g = G(Ynew[n], n)
            Gnew.append(g)
            Ynew.append(combine(Fk[n], g, Gold[n]))
        jump = max(jump_norm(Ynew[n + 1], Y[n + 1]) for n in range(N))
        Y, Gold = Ynew, Gnew
        history.append(dict(k=k, jump=jump, Y=list(Y)))
        if (n_it is not None and k + 1 >= n_it) or (tol is not None and jump < tol) or k + 1 >= N:
            break
        k += 1
    return Y, history


# ------------------------------------------------- coarser-grid coarse propagator

# The paper takes G on the fine grid with a larger time step and leaves other
# coarse propagators to future work (Sec. 2.1.2).  The variant here runs G on
# a grid with half the cells in each direction:
#     G~(y) = P( G_c( R(y) ) ),
# R the restriction to the coarse grid, P the prolongation back.  Fine cell
# (k, j, i) lies in coarse cell (k//2, j//2, i//2).  R averages the four fine
# faces that tile a coarse face (so the flux through it, and with it the
# discrete divergence, is kept) and the eight fine cells of a coarse cell; P
# copies a coarse face value to the fine faces inside it, interpolates
# linearly along the normal for fine faces halfway between two coarse faces,
# and copies a coarse cell's pressure to its eight fine cells.  So R(P(y)) = y
# and P keeps a divergence-free field divergence-free.  Parareal, Eq. (6),
# is unchanged with G~ in place of G.


def _coarse_ok(g: Grid, gc: Grid):
    if (g.nx, g.ny, g.nz) != (2 * gc.nx, 2 * gc.ny, 2 * gc.nz):
        raise ValueError("the coarse grid must have half the cells of the fine grid in every direction")
    if (g.lx, g.ly, g.lz, g.periodic_z) != (gc.lx, gc.ly, gc.lz, gc.periodic_z):
        raise ValueError("fine and coarse grids must cover the same box with the same boundaries")
    if g.solid is not None or gc.solid is not None:
        raise NotImplementedError("coarser-grid G is defined here for cavities without obstacles")


def restrict(g: Grid, gc: Grid, state):
    """R: fine state (u, v, w, p) -> coarse state.  Sums are taken pairwise
    in a fixed order: (a + b) + (c + d), then scaled."""
    _coarse_ok(g, gc)
    u, v, w, p = state
    # u faces at even x positions; the four fine faces (k, j) in {2K, 2K+1} x {2J, 2J+1}
    U = u[:, :, 0::2]
    Uc = 0.25 * ((U[0::2, 0::2] + U[0::2, 1::2]) + (U[1::2, 0::2] + U[1::2, 1::2]))
    V = v[:, 0::2, :]
    Vc = 0.25 * ((V[0::2, :, 0::2] + V[0::2, :, 1::2]) + (V[1::2, :, 0::2] + V[1::2, :, 1::2]))
    W = w[0::2]
    Wc = 0.25 * ((W[:, 0::2, 0::2] + W[:, 0::2, 1::2]) + (W[:, 1::2, 0::2] + W[:, 1::2, 1::2]))
    pz0 = (p[0::2, 0::2, 0::2] + p[0::2, 0::2, 1::2]) + (p[0::2, 1::2, 0::2] + p[0::2, 1::2, 1::2])
    pz1 = (p[1::2, 0::2, 0::2] + p[1::2, 0::2, 1::2]) + (p[1::2, 1::2, 0::2] + p[1::2, 1::2, 1::2])
    Pc = 0.125 * (pz0 + pz1)
    return tuple(np.ascontiguousarray(a) for a in (Uc, Vc, Wc, Pc))


def prolong(g: Grid, gc: Grid, state_c):
    """P: coarse state -> fine state."""
    _coarse_ok(g, gc)
    Uc, Vc, Wc, Pc = state_c
    nx, ny, nz = g.nx, g.ny, g.nz
    u = np.empty((nz, ny, nx + 1))
    v = np.empty((nz, ny + 1, nx))
    w = np.empty((nz + 1, ny, nx))
    # copy across the face (each coarse face value to its 2 x 2 fine faces)
    Ue = np.repeat(np.repeat(Uc, 2, axis=0), 2, axis=1)
    u[:, :, 0::2] = Ue
    u[:, :, 1::2] = 0.5 * (Ue[:, :, :-1] + Ue[:, :, 1:])
    Ve = np.repeat(np.repeat(Vc, 2, axis=0), 2, axis=2)
    v[:, 0::2, :] = Ve
    v[:, 1::2, :] = 0.5 * (Ve[:, :-1, :] + Ve[:, 1:, :])
    We = np.repeat(np.repeat(Wc, 2, axis=1), 2, axis=2)
    w[0::2] = We
    w[1::2] = 0.5 * (We[:-1] + We[1:])
    p = np.repeat(np.repeat(np.repeat(Pc, 2, axis=0), 2, axis=1), 2, axis=2)
    return u, v, w, np.ascontiguousarray(p)


def coarse_grid_propagator(g: Grid, gc: Grid, DT, **opts):
    """G~(y, t0, t1) = P(G_c(R(y))) with steps DT on the coarse grid."""
    def G(y, t0, t1):
        return prolong(g, gc, propagate(gc, restrict(g, gc, y), t0, t1, DT, **opts))
    return G


# ------------------------------------------------------------------ adjoint

def stencil_value(g: Grid, c, phi, f, d, m, as_form=False):
    """Stencil value of component c at open face f, offset m along d (the
    image rule), evaluated directly or through its linear form."""
    fn = lib().og_stencil_form_value if as_form else lib().og_stencil_value
    gc = g.c()
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    return fn(ctypes.byref(gc), int(c), _p(phi), int(f[0]), int(f[1]), int(f[2]), int(d), int(m))


def _no_periodic(g: Grid):
    if g.upwind:
        raise NotImplementedError("the adjoint differentiates the SMART fine propagator")
    if g.periodic_z:
        raise NotImplementedError("the adjoint is implemented for walls in z only")
    if g.slip_obstacles:
        raise NotImplementedError("the adjoint is implemented for no-slip obstacles only")


def momentum_adjoint(g: Grid, u, v, w, dt, mu):
    """lam = mu + dt (dR/du)^T mu and dt (dR/dlid)^T mu at the state (u, v, w)."""
    _no_periodic(g)
    su, sv, sw, _ = g.shapes()
    u, v, w = _chk(u, su), _chk(v, sv), _chk(w, sw)
    mu = [_chk(m, s) for m, s in zip(mu, (su, sv, sw))]
    lam = [np.empty(su), np.empty(sv), np.empty(sw)]
    glid = np.zeros_like(g.lid)
    gc = g.c()
    lib().og_momentum_adjoint(ctypes.byref(gc), _p(u), _p(v), _p(w), float(dt), _p(mu[0]), _p(mu[1]), _p(mu[2]),
                              _p(lam[0]), _p(lam[1]), _p(lam[2]), _p(glid))
    return lam, glid


def project(g: Grid, F, rtol=1e-12, maxit=100000, p0=None):
    """P F: the projection of the step applied to a face field (dt = 1)."""
    b = rhs(g, *F, 1.0)
    p, info = pcg(g, b, p0, rtol=rtol, maxit=maxit)
    if info["status"] != 0:
        raise RuntimeError("oracle projection solve failed: %r" % info)
    return correct(g, *F, p, 1.0), p


def kinetic_energy(g: Grid, state):
    """J = 1/2 * cell volume * sum of squared face velocities (closed faces are 0)."""
    hx, hy, hz = g.h
    vol = hx * hy * hz
    s = 0.0
    for a, op in zip(state[:3], _open_masks(g)):
        s += float(np.sum(a[op] ** 2))
    return 0.5 * vol * s


def _open_masks(g: Grid):
    """Boolean open-face masks of u, v, w."""
    fl = g.fluid()
    nz, ny, nx = fl.shape
    mu = np.zeros((nz, ny, nx + 1), bool)
    mu[:, :, 1:nx] = fl[:, :, :-1] & fl[:, :, 1:]
    mv = np.zeros((nz, ny + 1, nx), bool)
    mv[:, 1:ny, :] = fl[:, :-1, :] & fl[:, 1:, :]
    mw = np.zeros((nz + 1, ny, nx), bool)
    mw[1:nz] = fl[:-1] & fl[1:]
    return mu, mv, mw


def adjoint_gradient(g: Grid, state0, nsteps, dt, rtol=1e-12, ckpt_every=None):
    """J(u_T) = kinetic energy after nsteps FP64 steps from state0, and its
    gradient with respect to the initial face velocities and to the lid
    values (per top u-face position).  Forward states are kept at every
    `ckpt_every`-th step and recomputed inside each segment (all kept if
    None)."""
    _no_periodic(g)
    ck = ckpt_every or nsteps or 1
    ckpts = {0: tuple(a.copy() for a in state0)}
    y = tuple(a.copy() for a in state0)
    for n in range(nsteps):
        y, _, _, st = fine_steps(g, y, 1, dt, rtol=rtol)
        if st != 0:
            raise RuntimeError("oracle forward step failed")
        if (n + 1) % ck == 0 and n + 1 < nsteps:
            ckpts[n + 1] = tuple(a.copy() for a in y)
    J = kinetic_energy(g, y)
    hx, hy, hz = g.h
    masks = _open_masks(g)
    lam = [hx * hy * hz * np.where(m, a, 0.0) for a, m in zip(y[:3], masks)]
    glid = np.zeros_like(g.lid)
    seg_starts = sorted(ckpts)
    for s0 in reversed(seg_starts):
        s1 = min(s0 + ck, nsteps)
        states = [ckpts[s0]]
        for n in range(s0, s1 - 1):
            nxt, _, _, _ = fine_steps(g, states[-1], 1, dt, rtol=rtol)
            states.append(nxt)
        for n in range(s1 - 1, s0 - 1, -1):
            mu, _ = project(g, lam, rtol=rtol)
            u, v, w = states[n - s0][:3]
            lam, gl = momentum_adjoint(g, u, v, w, dt, mu)
            glid += gl
    return J, lam, glid
