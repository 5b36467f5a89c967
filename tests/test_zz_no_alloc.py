"""The allocation-free Poisson solve, nsp_poisson_solve_noalloc, against the
allocating entry point nsp_poisson_solve: the same kernels, with every
scratch buffer in the library's fixed device array instead of the handle's
workspace.  Outputs and reports must be bitwise equal, on calls in a row
whose inputs shrink (the array keeps the previous call's contents)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _noalloc(gpu, h, b, p, opts):
    f = gpu.lib().nsp_poisson_solve_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(gpu._Opts),
                  ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    B = int(b.shape[0])
    info = (gpu._Info * B)()
    o = opts.c()
    st = f(h.ptr, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(p.data_ptr()), B, ctypes.byref(o),
           gpu._stream_ptr(), info)
    return st, [gpu._info_dict(x) for x in info]


def _case(gpu, h, batch, opts, seed):
    import torch
    rng = np.random.default_rng(seed)
    shp = (batch, h.nz, h.ny, h.nx)
    b = torch.from_numpy(rng.standard_normal(shp)).cuda()
    p0 = torch.from_numpy(rng.standard_normal(shp) * 1e-3).cuda()
    p_ref = p0.clone()
    ref = h.poisson_solve(b, p_ref, opts)
    p = p0.clone()
    st, info = _noalloc(gpu, h, b, p, opts)
    assert st == gpu.NSP_OK, gpu.lib().nsp_last_error(h.ptr)
    assert torch.equal(p, p_ref)
    assert info == ref
    return info


def test_noalloc_poisson_matches_the_allocating_solve(gpu):
    h = gpu.Handle(64, 64, 64, max_batch=2)
    _say("noalloc 64^3 batch 2 fp64")
    h.launch_stats(reset=True)
    _case(gpu, h, 2, gpu.PoissonOpts(rtol=1e-10), 1)
    # both launches (allocating and not) held the CG vectors in registers,
    # whose boundary values go through the workspace's d0, d1 and q
    assert h.launch_stats()["poisson"]["rr_launches"] == 2
    _say("noalloc 64^3 batch 1 mixed")
    _case(gpu, h, 1, gpu.PoissonOpts(rtol=1e-10, prec=gpu.MIXED), 2)
    _say("noalloc 64^3 batch 2 mixed with reliable updates")
    _case(gpu, h, 2, gpu.PoissonOpts(rtol=1e-10, prec=gpu.MIXED_RU, inner_rtol=1e-3, max_outer=64), 5)
    h.close()
    h2 = gpu.Handle(24, 20, 16, lx=1.2, periodic_z=True, max_batch=1)
    _say("noalloc 24x20x16 periodic batch 1 bicgstab")
    _case(gpu, h2, 1, gpu.PoissonOpts(rtol=1e-10, solver=gpu.BICGSTAB), 3)
    _say("noalloc 24x20x16 periodic batch 1 fp64 again")
    _case(gpu, h2, 1, gpu.PoissonOpts(rtol=1e-10), 4)
    h2.close()


def test_noalloc_rejects_a_solve_beyond_its_array(gpu):
    import torch
    _say("noalloc 128^3 bicgstab: beyond the array")
    h = gpu.Handle(128, 128, 128, max_batch=1)
    b = torch.ones((1, 128, 128, 128), dtype=torch.float64, device="cuda")
    p = torch.zeros_like(b)
    st, _ = _noalloc(gpu, h, b, p, gpu.PoissonOpts(solver=gpu.BICGSTAB))
    assert st == gpu.NSP_ERR_ARG
    assert b"bytes of workspace" in gpu.lib().nsp_last_error(h.ptr)
    assert float(p.abs().max()) == 0.0
    h.close()
