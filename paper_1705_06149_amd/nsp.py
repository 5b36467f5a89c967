"""Python binding of libnsp (include/nsp.h): argument marshalling only.

Every array is a contiguous float64 torch tensor on the current HIP device;
this module checks dtype, device, contiguity and shapes, then passes raw
pointers and the current stream to the C ABI.  All arithmetic happens in the
library's gfx950 kernels.  If libnsp.so is missing or a tensor is not on the
GPU, calls raise: there is no CPU path.

Layout of one slice of a grid with nx*ny*nz cells (y vertical, lid in +x):
    u (nz, ny, nx+1)   v (nz, ny+1, nx)   w (nz+1, ny, nx)   p (nz, ny, nx)
A batch adds a leading dimension B.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from dataclasses import dataclass

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnsp.so")

NSP_OK, NSP_ERR_ARG, NSP_ERR_NOT_CONVERGED, NSP_ERR_NONFINITE, NSP_ERR_HIP, NSP_ERR_UNSUPPORTED = range(6)
PCG, BICGSTAB, PCG_SR = 0, 1, 2
_STATUS = {0: "NSP_OK", 1: "NSP_ERR_ARG", 2: "NSP_ERR_NOT_CONVERGED", 3: "NSP_ERR_NONFINITE",
           4: "NSP_ERR_HIP", 5: "NSP_ERR_UNSUPPORTED"}
FP64, MIXED, MIXED_RU = 0, 1, 2
CONV_SMART, CONV_UPWIND = 0, 1


class NSPError(RuntimeError):
    def __init__(self, status, msg, info=None):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status
        self.info = info


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("re", ctypes.c_double), ("periodic_z", ctypes.c_int),
                ("solid_host", ctypes.c_void_p), ("max_batch", ctypes.c_int), ("slip_obstacles", ctypes.c_int)]


class _Opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("maxit", ctypes.c_int), ("prec", ctypes.c_int),
                ("inner_rtol", ctypes.c_double), ("max_outer", ctypes.c_int), ("solver", ctypes.c_int),
                ("extrapolate", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("max_iters", ctypes.c_int), ("outer", ctypes.c_int),
                ("status", ctypes.c_int), ("rel_res_true", ctypes.c_double), ("div_l2", ctypes.c_double)]


class _LaunchStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_longlong), ("ms", ctypes.c_double), ("cell_steps", ctypes.c_double),
                ("cg_cell_iters", ctypes.c_double), ("cell_sweeps", ctypes.c_double),
                ("cg64_cell_iters", ctypes.c_double), ("cg32_cell_iters", ctypes.c_double),
                ("bicg_cell_iters", ctypes.c_double), ("mixed_cell_sweeps", ctypes.c_double),
                ("rr_launches", ctypes.c_longlong)]


class _State(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("v", ctypes.c_void_p), ("w", ctypes.c_void_p), ("p", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libnsp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch first: its HIP runtime is then the one libnsp binds to (loading
        # libnsp first and torch afterwards leaves two runtimes in the process)
        _torch()
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("libnsp.so is not built: run paper_1705_06149_amd/build.py")
        L = ctypes.CDLL(_LIB_PATH)
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        S = ctypes.c_int
        L.nsp_create.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(P)]
        L.nsp_destroy.argtypes = [P]
        L.nsp_last_error.argtypes = [P]
        L.nsp_last_error.restype = ctypes.c_char_p
        L.nsp_set_lid.argtypes = [P, P, P]
        L.nsp_poisson_solve.argtypes = [P, P, P, I, ctypes.POINTER(_Opts), P, P]
        L.nsp_poisson_solve_noalloc.argtypes = [P, P, P, I, ctypes.POINTER(_Opts), P, P]
        L.nsp_fine_step.argtypes = [P, _State, I, D, D, D, ctypes.POINTER(_Opts), P, P]
        L.nsp_coarse_step.argtypes = [P, _State, I, D, D, D, ctypes.POINTER(_Opts), P, P]
        L.nsp_group_fine_step.argtypes = [P, P, P, I, D, D, D, ctypes.POINTER(_Opts), P, P]
        L.nsp_parareal_start.argtypes = [P, _State, _State, I, D, D, D, ctypes.POINTER(_Opts), P]
        L.nsp_parareal_iterate.argtypes = [P, _State, _State, _State, I, I, D, D, D, D,
                                           ctypes.POINTER(_Opts), ctypes.POINTER(_Opts), P, P]
        L.nsp_group_parareal_start.argtypes = [P, P, P, I, I, D, D, D, ctypes.POINTER(_Opts), P]
        L.nsp_group_parareal_iterate.argtypes = [P, P, P, P, I, I, I, D, D, D, D, ctypes.POINTER(_Opts),
                                                 ctypes.POINTER(_Opts), P, P]
        L.nsp_restrict.argtypes = [P, P, _State, _State, I, P]
        L.nsp_prolong.argtypes = [P, P, _State, _State, I, P]
        L.nsp_parareal_start_cgrid.argtypes = [P, P, _State, _State, I, D, D, D, ctypes.POINTER(_Opts), P]
        L.nsp_parareal_iterate_cgrid.argtypes = [P, P, _State, _State, _State, I, I, D, D, D, D,
                                                 ctypes.POINTER(_Opts), ctypes.POINTER(_Opts), P, P]
        L.nsp_launch_stats_get.argtypes = [P, P, I]
        L.nsp_set_launch.argtypes = [P, I]
        L.nsp_set_coarse_convection.argtypes = [P, I]
        L.nsp_autotune.argtypes = [P, I, I, P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]
        L.nsp_last_launch_ms.argtypes = [P, ctypes.POINTER(D)]
        L.nsp_fine_solve_adjoint.argtypes = [P, _State, I, D, I, ctypes.POINTER(_Opts), _State, P,
                                             ctypes.POINTER(D), P]
        L.nsp_fine_solve_record.argtypes = [P, _State, I, D, I, ctypes.POINTER(_Opts), ctypes.POINTER(D),
                                            ctypes.POINTER(ctypes.c_ulonglong), P]
        L.nsp_fine_solve_reverse.argtypes = [P, ctypes.c_ulonglong, _State, P, P]
        L.nsp_fine_solve_tape_valid.argtypes = [P, ctypes.c_ulonglong]
        L.nsp_momentum_adjoint.argtypes = [P, _State, _State, _State, P, D, P]
        L.nsp_fine_step_graph_create.argtypes = [P, _State, I, D, D, D, ctypes.POINTER(_Opts),
                                                 ctypes.POINTER(ctypes.c_void_p)]
        L.nsp_graph_launch.argtypes = [P, P]
        L.nsp_graph_finish.argtypes = [P, P, P]
        L.nsp_graph_destroy.argtypes = [P]
        L.nsp_fine_solve_tape_valid.restype = I
        L.nsp_lid_from_modes.argtypes = [P, P, I, P, P]
        L.nsp_lid_modes_grad.argtypes = [P, P, I, P, P]
        for name in ("nsp_create", "nsp_destroy", "nsp_set_lid", "nsp_poisson_solve", "nsp_poisson_solve_noalloc",
                     "nsp_fine_step",
                     "nsp_coarse_step", "nsp_group_fine_step", "nsp_parareal_start", "nsp_parareal_iterate",
                     "nsp_group_parareal_start", "nsp_group_parareal_iterate", "nsp_set_launch", "nsp_autotune",
                     "nsp_last_launch_ms", "nsp_fine_solve_adjoint", "nsp_lid_from_modes", "nsp_lid_modes_grad",
                     "nsp_restrict", "nsp_prolong", "nsp_parareal_start_cgrid", "nsp_parareal_iterate_cgrid",
                     "nsp_launch_stats_get", "nsp_set_coarse_convection", "nsp_fine_solve_record",
                     "nsp_fine_solve_reverse", "nsp_momentum_adjoint", "nsp_fine_step_graph_create",
                     "nsp_graph_launch", "nsp_graph_finish", "nsp_graph_destroy"):
            getattr(L, name).restype = S
        _lib = L
    return _lib


@dataclass
class PoissonOpts:
    """Options of the Poisson solve (nsp_poisson_opts)."""
    rtol: float = 1e-10
    maxit: int = 20000
    prec: int = FP64
    inner_rtol: float = 1e-5
    max_outer: int = 8
    solver: int = 0  # PCG, BICGSTAB or PCG_SR
    extrapolate: bool = False  # warm start 2 p^s - p^(s-1) from the second step of a call on

    def c(self):
        return _Opts(float(self.rtol), int(self.maxit), int(self.prec), float(self.inner_rtol), int(self.max_outer),
                     int(self.solver), int(bool(self.extrapolate)))


def _torch():
    import torch
    return torch


def _stream_ptr():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(t, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64, got %s" % (name, t.dtype))
    if not t.is_cuda:
        raise ValueError("%s must be on the GPU (libnsp has no CPU path)" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return t.data_ptr()


# Handles still open when the interpreter exits are destroyed by an atexit
# hook, while the HIP runtime (and any profiler attached to it) is still up;
# a handle reached only by garbage collection during interpreter teardown is
# left to the process exit instead of calling into HIP from a finalizer.
_live_handles = weakref.WeakSet()


def _close_live_handles():
    for h in list(_live_handles):
        try:
            h.close()
        except Exception:
            pass


atexit.register(_close_live_handles)


class Handle:
    """One grid (nsp_create / nsp_destroy)."""

    def __init__(self, nx, ny, nz, lx=1.0, ly=1.0, lz=1.0, re=100.0, solid=None, max_batch=1, periodic_z=False,
                 slip_obstacles=False):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.periodic_z = bool(periodic_z)
        self.lx, self.ly, self.lz, self.re = float(lx), float(ly), float(lz), float(re)
        self.max_batch = int(max_batch)
        self._solid = None
        if solid is not None:
            s = np.ascontiguousarray(np.asarray(solid), dtype=np.uint8)
            if s.shape != (self.nz, self.ny, self.nx):
                raise ValueError("solid mask must have shape (nz, ny, nx)")
            self._solid = s
        self.slip_obstacles = bool(slip_obstacles)
        g = _Grid(self.nx, self.ny, self.nz, self.lx, self.ly, self.lz, self.re, 1 if self.periodic_z else 0,
                  self._solid.ctypes.data if self._solid is not None else None, self.max_batch,
                  1 if self.slip_obstacles else 0)
        h = ctypes.c_void_p()
        st = lib().nsp_create(ctypes.byref(g), ctypes.byref(h))
        if st != NSP_OK:
            raise NSPError(st, "nsp_create failed (sizes, max_batch <= 64, connected fluid region)")
        self._h = h
        _live_handles.add(self)

    def close(self):
        for g in list(getattr(self, "_graphs", ())):
            g.close()  # a graph uses the handle's workspace
        if getattr(self, "_h", None):
            lib().nsp_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    @property
    def ptr(self):
        return self._h

    def shapes(self, batch=None):
        nx, ny, nz = self.nx, self.ny, self.nz
        s = [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx), (nz, ny, nx)]
        if batch is not None:
            s = [(batch,) + x for x in s]
        return s

    def zeros_state(self, batch=1, device="cuda"):
        torch = _torch()
        return tuple(torch.zeros(s, dtype=torch.float64, device=device) for s in self.shapes(batch))

    def _err(self, st, what, info=None):
        if st != NSP_OK:
            msg = lib().nsp_last_error(self._h)
            raise NSPError(st, "%s: %s" % (what, msg.decode() if msg else ""), info)

    def _state(self, y, batch, name="y"):
        shp = self.shapes(batch)
        ptrs = [_check(t, s, "%s[%d]" % (name, i)) for i, (t, s) in enumerate(zip(y, shp))]
        return _State(*ptrs)

    @staticmethod
    def _batch_of(y):
        return int(y[0].shape[0])

    def set_lid(self, lid):
        _check(lid, (self.nz, self.nx + 1), "lid")
        self._err(lib().nsp_set_lid(self._h, ctypes.c_void_p(lid.data_ptr()), _stream_ptr()), "nsp_set_lid")

    def poisson_solve(self, b, p, opts=None, check=True):
        """Solve A p = b in place on p (batch = leading dimension)."""
        opts = opts or PoissonOpts()
        B = int(b.shape[0])
        sp = (B, self.nz, self.ny, self.nx)
        pb, pp = _check(b, sp, "b"), _check(p, sp, "p")
        info = (_Info * B)()
        o = opts.c()
        st = lib().nsp_poisson_solve(self._h, ctypes.c_void_p(pb), ctypes.c_void_p(pp), B, ctypes.byref(o),
                                     _stream_ptr(), info)
        res = [_info_dict(x) for x in info]
        if check:
            self._err(st, "nsp_poisson_solve", res)
        return res

    def poisson_solve_noalloc(self, b, p, opts=None, check=True):
        """poisson_solve through nsp_poisson_solve_noalloc: the library's fixed
        device array as workspace, no device allocation by the call."""
        opts = opts or PoissonOpts()
        B = int(b.shape[0])
        sp = (B, self.nz, self.ny, self.nx)
        pb, pp = _check(b, sp, "b"), _check(p, sp, "p")
        info = (_Info * B)()
        o = opts.c()
        st = lib().nsp_poisson_solve_noalloc(self._h, ctypes.c_void_p(pb), ctypes.c_void_p(pp), B, ctypes.byref(o),
                                             _stream_ptr(), info)
        res = [_info_dict(x) for x in info]
        if check:
            self._err(st, "nsp_poisson_solve_noalloc", res)
        return res

    def _prop(self, fn, y, t0, t1, step, opts, check):
        opts = opts or PoissonOpts()
        B = self._batch_of(y)
        s = self._state(y, B)
        info = (_Info * B)()
        o = opts.c()
        st = fn(self._h, s, B, float(t0), float(t1), float(step), ctypes.byref(o), _stream_ptr(), info)
        res = [_info_dict(x) for x in info]
        if check:
            self._err(st, fn.__name__, res)
        return res

    def fine_step(self, y, t0, t1, dt, opts=None, check=True):
        """F(y, t1, t0): (t1-t0)/dt projection steps in place on the batch y."""
        return self._prop(lib().nsp_fine_step, y, t0, t1, dt, opts, check)

    def fine_step_graph(self, y, t0, t1, dt, opts=None):
        """Record F(y, t1, t0) on the batch y as a replayable HIP graph
        (nsp_fine_step_graph_create); returns a FineStepGraph.  The graph keeps
        references to the tensors of y, whose storage it writes."""
        opts = opts or PoissonOpts()
        B = self._batch_of(y)
        s = self._state(y, B)
        o = opts.c()
        out = ctypes.c_void_p()
        st = lib().nsp_fine_step_graph_create(self._h, s, B, float(t0), float(t1), float(dt), ctypes.byref(o),
                                              ctypes.byref(out))
        self._err(st, "nsp_fine_step_graph_create")
        g = FineStepGraph(self, out, tuple(y), B)
        if not hasattr(self, "_graphs"):
            self._graphs = weakref.WeakSet()
        self._graphs.add(g)
        return g

    def coarse_step(self, y, t0, t1, DT, opts=None, check=True):
        """G(y, t1, t0): (t1-t0)/DT projection steps in place on the batch y."""
        return self._prop(lib().nsp_coarse_step, y, t0, t1, DT, opts, check)

    def parareal_start(self, Y, Gk, nslices, t0, T, DT, coarse=None):
        coarse = coarse or PoissonOpts()
        o = coarse.c()
        st = lib().nsp_parareal_start(self._h, self._state(Y, nslices + 1, "Y"), self._state(Gk, nslices, "Gk"),
                                      int(nslices), float(t0), float(T), float(DT), ctypes.byref(o), _stream_ptr())
        self._err(st, "nsp_parareal_start")

    def parareal_iterate(self, Y, Fk, Gk, nslices, k, t0, T, dt, DT, fine=None, coarse=None, check=True):
        """Iteration k of Eq. (6); returns (velocity jump, pressure jump).  With
        check=False a solve that hit its limit (NSP_ERR_NOT_CONVERGED) does not
        raise; the jumps are returned and self.last_status holds the status."""
        fine = fine or PoissonOpts()
        coarse = coarse or PoissonOpts()
        of, oc = fine.c(), coarse.c()
        jump = (ctypes.c_double * 2)()
        st = lib().nsp_parareal_iterate(self._h, self._state(Y, nslices + 1, "Y"), self._state(Fk, nslices, "Fk"),
                                        self._state(Gk, nslices, "Gk"), int(nslices), int(k), float(t0), float(T),
                                        float(dt), float(DT), ctypes.byref(of), ctypes.byref(oc), _stream_ptr(),
                                        jump)
        self.last_status = st
        if check or st != NSP_ERR_NOT_CONVERGED:
            self._err(st, "nsp_parareal_iterate")
        return float(jump[0]), float(jump[1])

    def restrict(self, hc, yf, yc):
        """yc <- R(yf): fine-grid states (this handle) to states on the grid of
        the coarse handle hc (half the cells per direction); batch = leading
        dimension."""
        B = self._batch_of(yf)
        self._err(lib().nsp_restrict(self._h, hc._h, self._state(yf, B, "yf"), hc._state(yc, B, "yc"), B,
                                     _stream_ptr()), "nsp_restrict")

    def prolong(self, hc, yc, yf):
        """yf <- P(yc): states on hc's grid to fine-grid states."""
        B = self._batch_of(yc)
        self._err(lib().nsp_prolong(self._h, hc._h, hc._state(yc, B, "yc"), self._state(yf, B, "yf"), B,
                                    _stream_ptr()), "nsp_prolong")

    def parareal_start_cgrid(self, hc, Y, Gk, nslices, t0, T, DT, coarse=None):
        """parareal_start with the coarse propagator P(G_c(R(y))) on hc's grid."""
        o = (coarse or PoissonOpts()).c()
        st = lib().nsp_parareal_start_cgrid(self._h, hc._h, self._state(Y, nslices + 1, "Y"),
                                            self._state(Gk, nslices, "Gk"), int(nslices), float(t0), float(T),
                                            float(DT), ctypes.byref(o), _stream_ptr())
        self._err(st, "nsp_parareal_start_cgrid")

    def parareal_iterate_cgrid(self, hc, Y, Fk, Gk, nslices, k, t0, T, dt, DT, fine=None, coarse=None):
        """parareal_iterate with the coarse propagator P(G_c(R(y))) on hc's grid;
        returns (velocity jump, pressure jump)."""
        of, oc = (fine or PoissonOpts()).c(), (coarse or PoissonOpts()).c()
        jump = (ctypes.c_double * 2)()
        st = lib().nsp_parareal_iterate_cgrid(self._h, hc._h, self._state(Y, nslices + 1, "Y"),
                                              self._state(Fk, nslices, "Fk"), self._state(Gk, nslices, "Gk"),
                                              int(nslices), int(k), float(t0), float(T), float(dt), float(DT),
                                              ctypes.byref(of), ctypes.byref(oc), _stream_ptr(), jump)
        self._err(st, "nsp_parareal_iterate_cgrid")
        return float(jump[0]), float(jump[1])

    def launch_stats(self, reset=False):
        """Persistent-kernel launch statistics since the last reset, as dicts
        for the launch kinds 'fine', 'poisson' and 'project'."""
        arr = (_LaunchStats * 3)()
        self._err(lib().nsp_launch_stats_get(self._h, arr, 1 if reset else 0), "nsp_launch_stats_get")
        return {k: {f: getattr(x, f) for f, _ in _LaunchStats._fields_}
                for k, x in zip(("fine", "poisson", "project"), arr)}

    def set_coarse_convection(self, scheme):
        """CONV_SMART (the fine scheme) or CONV_UPWIND (donor cell) for the
        coarse propagator of this handle."""
        self._err(lib().nsp_set_coarse_convection(self._h, int(scheme)), "nsp_set_coarse_convection")

    def set_launch(self, workgroups):
        self._err(lib().nsp_set_launch(self._h, int(workgroups)), "nsp_set_launch")

    def autotune(self, batch, prec=FP64):
        """Time launch shapes for (batch, prec); returns (workgroups, column-tile
        planes, rows per thread), the last two 0 for flat tiles."""
        ch, pl, it = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._err(lib().nsp_autotune(self._h, int(batch), int(prec), _stream_ptr(), ctypes.byref(ch),
                                     ctypes.byref(pl), ctypes.byref(it)), "nsp_autotune")
        return ch.value, pl.value, it.value

    def fine_solve_adjoint(self, y0, nsteps, dt, ckpt_every=10, opts=None, grad=True):
        """J = kinetic energy after nsteps steps from y0 (batch 1), and if grad
        its gradient with respect to (u0, v0, w0) and to the lid values.
        Returns (J, (gu, gv, gw) or None, g_lid or None)."""
        torch = _torch()
        opts = opts or PoissonOpts(rtol=1e-12)
        s = self._state(y0, 1, "y0")
        o = opts.c()
        J = ctypes.c_double()
        if grad:
            g = tuple(torch.zeros(sh, dtype=torch.float64, device=y0[0].device) for sh in self.shapes(1)[:3])
            gl = torch.zeros((self.nz, self.nx + 1), dtype=torch.float64, device=y0[0].device)
            gs = _State(g[0].data_ptr(), g[1].data_ptr(), g[2].data_ptr(), None)
            glp = ctypes.c_void_p(gl.data_ptr())
        else:
            g, gl = None, None
            gs = _State(None, None, None, None)
            glp = None
        st = lib().nsp_fine_solve_adjoint(self._h, s, int(nsteps), float(dt), int(ckpt_every), ctypes.byref(o), gs,
                                          glp, ctypes.byref(J), _stream_ptr())
        self._err(st, "nsp_fine_solve_adjoint")
        return J.value, g, gl

    def fine_solve_record(self, y0, nsteps, dt, ckpt_every=10, opts=None, keep=True):
        """Forward half of fine_solve_adjoint: J after nsteps steps from y0
        (batch 1) and, if keep, the id of the record the handle now holds for
        fine_solve_reverse (else 0).  Returns (J, tape)."""
        opts = opts or PoissonOpts(rtol=1e-12)
        s = self._state(y0, 1, "y0")
        o = opts.c()
        J = ctypes.c_double()
        tape = ctypes.c_ulonglong(0)
        st = lib().nsp_fine_solve_record(self._h, s, int(nsteps), float(dt), int(ckpt_every), ctypes.byref(o),
                                         ctypes.byref(J), ctypes.byref(tape) if keep else None, _stream_ptr())
        self._err(st, "nsp_fine_solve_record")
        return J.value, tape.value

    def momentum_adjoint(self, vel, mu, lam, dt, g_lid=None):
        """lam = mu + dt (dR/du)^T mu at the velocity vel; g_lid += dt
        (dR/dlid)^T mu if given.  vel, mu, lam: (u, v, w) of one slice, with or
        without a batch dimension of 1.  Asynchronous on the current stream."""
        shp = self.shapes(1)[:3]

        def st(t, name):
            ptrs = [_check(a if a.dim() == 4 else a[None], s, "%s[%d]" % (name, i))
                    for i, (a, s) in enumerate(zip(t, shp))]
            return _State(ptrs[0], ptrs[1], ptrs[2], None)

        gl = None
        if g_lid is not None:
            gl = _check(g_lid, (self.nz, self.nx + 1), "g_lid")
        self._err(lib().nsp_momentum_adjoint(self._h, st(vel, "vel"), st(mu, "mu"), st(lam, "lam"), gl, float(dt),
                                             _stream_ptr()), "nsp_momentum_adjoint")

    def tape_valid(self, tape):
        """True while the record `tape` may still be reversed."""
        return bool(lib().nsp_fine_solve_tape_valid(self._h, ctypes.c_ulonglong(int(tape))))

    def fine_solve_reverse(self, tape, device=None):
        """Reverse sweep of the record `tape`: ((gu, gv, gw), g_lid)."""
        torch = _torch()
        dev = device or torch.device("cuda", torch.cuda.current_device())
        g = tuple(torch.zeros(sh, dtype=torch.float64, device=dev) for sh in self.shapes(1)[:3])
        gl = torch.zeros((self.nz, self.nx + 1), dtype=torch.float64, device=dev)
        gs = _State(g[0].data_ptr(), g[1].data_ptr(), g[2].data_ptr(), None)
        st = lib().nsp_fine_solve_reverse(self._h, ctypes.c_ulonglong(int(tape)), gs, ctypes.c_void_p(gl.data_ptr()),
                                          _stream_ptr())
        self._err(st, "nsp_fine_solve_reverse")
        return g, gl

    def lid_from_modes(self, coef):
        """lid = 1 + sum c[m,n] sin(m pi x) sin(n pi z) at the top u-faces."""
        torch = _torch()
        M = int(coef.shape[0])
        _check(coef, (M, M), "coef")
        lid = torch.empty((self.nz, self.nx + 1), dtype=torch.float64, device=coef.device)
        self._err(lib().nsp_lid_from_modes(self._h, ctypes.c_void_p(coef.data_ptr()), M,
                                           ctypes.c_void_p(lid.data_ptr()), _stream_ptr()), "nsp_lid_from_modes")
        return lid

    def lid_modes_grad(self, g_lid, nmodes):
        torch = _torch()
        _check(g_lid, (self.nz, self.nx + 1), "g_lid")
        gc = torch.empty((nmodes, nmodes), dtype=torch.float64, device=g_lid.device)
        self._err(lib().nsp_lid_modes_grad(self._h, ctypes.c_void_p(g_lid.data_ptr()), int(nmodes),
                                           ctypes.c_void_p(gc.data_ptr()), _stream_ptr()), "nsp_lid_modes_grad")
        return gc

    def last_launch_ms(self):
        ms = ctypes.c_double()
        self._err(lib().nsp_last_launch_ms(self._h, ctypes.byref(ms)), "nsp_last_launch_ms")
        return ms.value


def _info_dict(x):
    return dict(iters=x.iters, max_iters=x.max_iters, outer=x.outer, status=x.status,
                rel_res_true=x.rel_res_true, div_l2=x.div_l2)


def _group_arrays(handles, states, nslices_each, names=("y",)):
    n = len(handles)
    hs = (ctypes.c_void_p * n)(*[h.ptr for h in handles])
    arrs = []
    for name, st_list in zip(names, states):
        arr = (_State * n)()
        for g, (h, y) in enumerate(zip(handles, st_list)):
            arr[g] = h._state(y, nslices_each[g] if isinstance(nslices_each, (list, tuple)) else nslices_each, name)
        arrs.append(arr)
    return hs, arrs


def group_fine_step(handles, ys, t0, t1, dt, opts=None, check=True):
    """F over several grids (an uneven batch) in one launch."""
    opts = opts or PoissonOpts()
    batches = [int(y[0].shape[0]) for y in ys]
    hs, (arr,) = _group_arrays(handles, [ys], batches)
    bat = (ctypes.c_int * len(handles))(*batches)
    info = (_Info * sum(batches))()
    o = opts.c()
    st = lib().nsp_group_fine_step(hs, arr, bat, len(handles), float(t0), float(t1), float(dt), ctypes.byref(o),
                                   _stream_ptr(), info)
    res = [_info_dict(x) for x in info]
    if check:
        handles[0]._err(st, "nsp_group_fine_step", res)
    return res


def group_parareal_start(handles, Ys, Gks, nslices, t0, T, DT, coarse=None):
    coarse = coarse or PoissonOpts()
    o = coarse.c()
    n = len(handles)
    hs, (ya,) = _group_arrays(handles, [Ys], [nslices + 1] * n, ("Y",))
    _, (ga,) = _group_arrays(handles, [Gks], [nslices] * n, ("Gk",))
    st = lib().nsp_group_parareal_start(hs, ya, ga, n, int(nslices), float(t0), float(T), float(DT),
                                        ctypes.byref(o), _stream_ptr())
    handles[0]._err(st, "nsp_group_parareal_start")


def group_parareal_iterate(handles, Ys, Fks, Gks, nslices, k, t0, T, dt, DT, fine=None, coarse=None):
    """Iteration k over several grids; returns [(velocity jump, pressure jump)] per grid."""
    fine = fine or PoissonOpts()
    coarse = coarse or PoissonOpts()
    of, oc = fine.c(), coarse.c()
    n = len(handles)
    hs, (ya,) = _group_arrays(handles, [Ys], [nslices + 1] * n, ("Y",))
    _, (fa,) = _group_arrays(handles, [Fks], [nslices] * n, ("Fk",))
    _, (ga,) = _group_arrays(handles, [Gks], [nslices] * n, ("Gk",))
    jump = (ctypes.c_double * (2 * n))()
    st = lib().nsp_group_parareal_iterate(hs, ya, fa, ga, n, int(nslices), int(k), float(t0), float(T), float(dt),
                                          float(DT), ctypes.byref(of), ctypes.byref(oc), _stream_ptr(), jump)
    handles[0]._err(st, "nsp_group_parareal_iterate")
    return [(float(jump[2 * g]), float(jump[2 * g + 1])) for g in range(n)]


class FineStepGraph:
    """A recorded fine step (nsp_fine_step_graph_create).  launch() enqueues
    one replay on the current stream without synchronising; finish()
    synchronises and returns per-slice info summed over the replays since the
    previous finish (raising NSPError on a failed solve when check)."""

    def __init__(self, handle, ptr, y, batch):
        self._handle = handle
        self._g = ptr
        self._y = y  # the graph writes these tensors' storage
        self.batch = batch

    def _live(self):
        if not self._g:
            raise RuntimeError("the graph is closed (or its handle was)")

    def launch(self):
        self._live()
        self._handle._err(lib().nsp_graph_launch(self._g, _stream_ptr()), "nsp_graph_launch")

    def finish(self, check=True):
        self._live()
        info = (_Info * self.batch)()
        st = lib().nsp_graph_finish(self._g, _stream_ptr(), info)
        res = [_info_dict(x) for x in info]
        self.last_status = st
        if check:
            self._handle._err(st, "nsp_graph_finish", res)
        return res

    def close(self):
        if self._g:
            lib().nsp_graph_destroy(self._g)
            self._g = None
            self._y = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


EXPORTED = ("nsp_create", "nsp_destroy", "nsp_last_error", "nsp_set_lid", "nsp_poisson_solve",
            "nsp_poisson_solve_noalloc", "nsp_fine_step",
            "nsp_coarse_step", "nsp_group_fine_step", "nsp_parareal_start", "nsp_parareal_iterate",
            "nsp_group_parareal_start", "nsp_group_parareal_iterate", "nsp_set_launch", "nsp_autotune",
            "nsp_last_launch_ms", "nsp_fine_solve_adjoint", "nsp_lid_from_modes", "nsp_lid_modes_grad",
            "nsp_restrict", "nsp_prolong", "nsp_parareal_start_cgrid", "nsp_parareal_iterate_cgrid",
            "nsp_launch_stats_get", "nsp_set_coarse_convection", "nsp_fine_solve_record",
            "nsp_fine_solve_reverse", "nsp_fine_solve_tape_valid", "nsp_momentum_adjoint",
            "nsp_fine_step_graph_create", "nsp_graph_launch", "nsp_graph_finish", "nsp_graph_destroy")
