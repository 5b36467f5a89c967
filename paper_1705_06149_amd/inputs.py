"""Seeded synthetic inputs for the lid-driven cavity workloads.

This module holds no arithmetic of the projection method: it only builds
initial states, obstacle masks, lid profiles and configuration presets.  It
is the one module that both the HIP path's tests/benchmark and the CPU
oracle's tests draw inputs from; it imports neither of them.

Workload family (Croce, Ruprecht & Krause, Sec. 3): a cavity on a box with y
vertical, the top face moving with tangential velocity 1 in +x, no-slip on
every other wall and on solid obstacles, fluid at rest and p = 0 at t = 0.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def face_shapes(nx, ny, nz):
    """Shapes of u, v, w, p for one slice (x fastest)."""
    return (nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx), (nz, ny, nx)


def rest_state(nx, ny, nz, batch=None):
    """Fluid at rest, p = 0 (the paper's initial condition)."""
    shp = face_shapes(nx, ny, nz)
    if batch is not None:
        shp = [(batch,) + s for s in shp]
    return tuple(np.zeros(s) for s in shp)


def uniform_lid(nx, nz, value=1.0):
    """Lid velocity on the top face, one value per top u-face position (nz, nx+1)."""
    return np.full((nz, nx + 1), float(value))


def random_state(nx, ny, nz, seed, scale=1.0, pscale=None):
    """Random (u, v, w, p), normal with standard deviation `scale`; values at
    closed faces are random too (the solver must ignore them)."""
    rng = np.random.default_rng(seed)
    shp = face_shapes(nx, ny, nz)
    out = [rng.standard_normal(s) * scale for s in shp[:3]]
    out.append(rng.standard_normal(shp[3]) * (scale if pscale is None else pscale))
    return tuple(out)


def obstacle_mask(n, seed, frac=0.05, smin=4, smax=12, margin=1):
    """Seeded random axis-aligned cuboid obstacles in an n^3 cavity.

    Sides are independent uniform integers in [smin, smax] per axis (clipped
    to the box), positions uniform with `margin` fluid cells to every wall;
    overlaps are allowed; cuboids are added until the solid fraction reaches
    `frac`.  Fluid cells that cannot be reached from the row under the lid
    (face-connected) are made solid, so the fluid is one region.
    Returns uint8 (n, n, n) indexed [k, j, i], 1 = solid.
    """
    from scipy import ndimage

    rng = np.random.default_rng(seed)
    solid = np.zeros((n, n, n), dtype=np.uint8)
    lo = margin
    while solid.mean() < frac:
        size = rng.integers(smin, smax + 1, size=3)
        size = np.minimum(size, n - 2 * margin)
        start = [rng.integers(lo, n - margin - s + 1) for s in size]
        solid[start[2]:start[2] + size[2], start[1]:start[1] + size[1], start[0]:start[0] + size[0]] = 1
    fluid = solid == 0
    lab, _ = ndimage.label(fluid, structure=ndimage.generate_binary_structure(3, 1))
    top = np.unique(lab[:, n - 1, :])
    top = top[top > 0]
    keep = np.isin(lab, top)
    solid[~keep] = 1
    return solid


def median_plane_cubes(n, seed, count=49, smin=2, smax=3):
    """Seeded cubes along the median plane of an n^3 cavity periodic in z, a
    stand-in for the 49-cube geometry of the paper's fully 3D test case
    (Sec. 3), whose layout is not given.

    `count` cubes with edges uniform in [smin, smax] cells; the centre height
    is the middle of the box (y = n/2) up to one cell, x uniform with one
    fluid cell to the side walls, z uniform over the period (a cube may wrap
    across the periodic seam).  Fluid cells that cannot be reached from the
    row under the lid (face-connected, the seam included) are made solid.
    Returns uint8 (n, n, n) indexed [k, j, i], 1 = solid.
    """
    from scipy import ndimage

    rng = np.random.default_rng(seed)
    solid = np.zeros((n, n, n), dtype=np.uint8)
    for _ in range(count):
        s = int(rng.integers(smin, smax + 1))
        x0 = int(rng.integers(1, n - s))
        y0 = n // 2 - s // 2 + int(rng.integers(-1, 2))
        z0 = int(rng.integers(0, n))
        for k in range(s):
            solid[(z0 + k) % n, y0:y0 + s, x0:x0 + s] = 1
    lab, nlab = ndimage.label(solid == 0, structure=ndimage.generate_binary_structure(3, 1))
    # regions that touch across the periodic seam are one region
    root = np.arange(nlab + 1)

    def find(a):
        while root[a] != a:
            root[a] = root[root[a]]
            a = root[a]
        return a

    for a, b in set(zip(lab[0].ravel().tolist(), lab[-1].ravel().tolist())):
        if a and b:
            ra, rb = find(a), find(b)
            if ra != rb:
                root[rb] = ra
    lab = np.array([find(a) for a in range(nlab + 1)])[lab]
    top = np.unique(lab[:, n - 1, :])
    solid[~np.isin(lab, top[top > 0])] = 1
    return solid


def div_free_perturbation(nx, ny, nz, seed, sigma=1e-2, lx=1.0, ly=1.0, lz=1.0):
    """Seeded divergence-free velocity field: the staggered-grid curl of a
    random N(0,1) edge potential that vanishes on boundary edges (so every
    boundary face carries zero normal velocity), scaled to face-value
    standard deviation `sigma`."""
    rng = np.random.default_rng(seed)
    hx, hy, hz = lx / nx, ly / ny, lz / nz
    Ax = rng.standard_normal((nz + 1, ny + 1, nx))      # x-edges (i+1/2, j, k)
    Ay = rng.standard_normal((nz + 1, ny, nx + 1))      # y-edges (i, j+1/2, k)
    Az = rng.standard_normal((nz, ny + 1, nx + 1))      # z-edges (i, j, k+1/2)
    # edges lying in a boundary plane
    Ax[0, :, :] = Ax[-1, :, :] = 0.0
    Ax[:, 0, :] = Ax[:, -1, :] = 0.0
    Ay[0, :, :] = Ay[-1, :, :] = 0.0
    Ay[:, :, 0] = Ay[:, :, -1] = 0.0
    Az[:, 0, :] = Az[:, -1, :] = 0.0
    Az[:, :, 0] = Az[:, :, -1] = 0.0
    u = (Az[:, 1:, :] - Az[:, :-1, :]) / hy - (Ay[1:, :, :] - Ay[:-1, :, :]) / hz
    v = (Ax[1:, :, :] - Ax[:-1, :, :]) / hz - (Az[:, :, 1:] - Az[:, :, :-1]) / hx
    w = (Ay[:, :, 1:] - Ay[:, :, :-1]) / hx - (Ax[:, 1:, :] - Ax[:, :-1, :]) / hy
    allv = np.concatenate([u[:, :, 1:-1].ravel(), v[:, 1:-1, :].ravel(), w[1:-1].ravel()])
    s = sigma / allv.std()
    return u * s, v * s, w * s


def lid_profile_basis(nx, nz, nmodes=16, lx=1.0, lz=1.0):
    """Lid basis sin(m pi x) sin(n pi z), m, n = 1..nmodes, sampled at the
    top u-face positions x = i*hx, z = (k+1/2)*hz: array (nmodes, nmodes, nz, nx+1)."""
    x = np.arange(nx + 1) * (lx / nx)
    z = (np.arange(nz) + 0.5) * (lz / nz)
    m = np.arange(1, nmodes + 1)
    sx = np.sin(np.pi * m[:, None] * x[None, :] / lx)     # (M, nx+1)
    sz = np.sin(np.pi * m[:, None] * z[None, :] / lz)     # (M, nz)
    return sz[None, :, :, None] * sx[:, None, None, :]    # (m, n, nz, nx+1)


@dataclass(frozen=True)
class Workload:
    """One lid-driven cavity configuration.  DT is the coarse step of the
    same-grid coarse propagator as the benchmark runs it; DT_cgrid the coarse
    step with the half-resolution coarse grid (0: not used)."""
    name: str
    n: int
    re: float
    dt: float
    steps: int
    T: float = 0.0
    nslices: int = 1
    DT: float = 0.0
    jump_tol: float = 0.0
    DT_cgrid: float = 0.0


# The five workloads: plain FP64 fine propagator; FP64 vs mixed precision;
# batched Parareal; obstacles with an uneven batch; adjoint.
WORKLOADS = {
    "cavity32_re100": Workload("cavity32_re100", 32, 100.0, 1e-3, 50),
    "cavity128_re1000": Workload("cavity128_re1000", 128, 1000.0, 5e-4, 200),
    # a coarse step of 1e-2 on the fine grid itself is unstable at 96^3
    # (Courant number ~1 plus a diffusion term ~0.55): the same-grid G runs at
    # 5e-3 (2.5e-3 with the 128^3 grid of the uneven batch); on the 48^3
    # coarse grid 1e-2 is stable
    "parareal96_re1000": Workload("parareal96_re1000", 96, 1000.0, 5e-4, 1280, T=0.64, nslices=32, DT=5e-3,
                                  jump_tol=1e-6, DT_cgrid=1e-2),
    "obstacles_64_96_128": Workload("obstacles_64_96_128", 0, 1000.0, 5e-4, 640, T=0.32, nslices=16, DT=2.5e-3,
                                    jump_tol=1e-6),
    "adjoint96_re400": Workload("adjoint96_re400", 96, 400.0, 1e-3, 100),
}
