// Host side of libnsp: the C ABI declared in include/nsp.h.
//
// A handle owns one grid (flags, lid, Jacobi table), the workspace of
// max_batch slices, and the launch resources (per-slice control blocks,
// tile partials, barrier words, a device copy of the launch parameters).
// Every entry point validates its arguments, fills a KParams block, copies
// it to the device on the caller's stream, launches the persistent kernel
// cooperatively (all workgroups co-resident, which the grid barrier needs),
// and reads the per-slice control blocks back.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "nsp.h"
#include "nsp_internal.h"

using namespace nsp;

struct LaunchRes {
    int cap_slices = 0, cap_tiles = 0;
    SliceCtl *ctl = nullptr;
    SliceCtl *ctl_host = nullptr;  // pinned
    double *part = nullptr;
    SyncWords *sync = nullptr;
    KParams *params = nullptr;       // device
    KParams *params_host = nullptr;  // pinned
    unsigned long long *jump = nullptr;       // device [2*kMaxGroups]
    unsigned long long *jump_host = nullptr;  // pinned
};

struct TuneEntry {
    int batch, prec, workgroups;
    int depth;  // CG column-tile depth in planes (0: by rule)
    int items;  // CG column items per thread (0: by rule)
};

struct nsp_handle {
    int device = 0;
    int nx = 0, ny = 0, nz = 0;
    double lx = 1, ly = 1, lz = 1, re = 1;
    int max_batch = 0;
    int tile = 0, ntiles = 0;
    int cby = 0, cbz = 0, cny = 0, cnz = 0, cgtiles = 0;  // CG column tiles (cby = 0: flat tiles), depth zsub
    int crb = 0, cnb = 0;  // rows per partial block (one workgroup-wide plane patch), blocks along y
    int zsh = 3;           // log2 of the planes per partial block (zsub = 8, or 4: see nsp_create)
    int cgparts = 0;                                      // CG partials per slice
    long long ncells = 0, nu = 0, nv = 0, nw = 0;
    double nfluid = 0;
    uint8_t *flags = nullptr;
    double *lid = nullptr;
    double *idiag = nullptr;
    float *idiag32 = nullptr;
    // workspace
    double *Fu = nullptr, *Fv = nullptr, *Fw = nullptr, *b = nullptr;
    double *r = nullptr, *d0 = nullptr, *d1 = nullptr, *q = nullptr;
    float *e = nullptr;
    double *bv0 = nullptr, *bv1 = nullptr, *brh = nullptr;  // BiCGStab (allocated on first use)
    double *pprev = nullptr;  // extrapolated warm start: previous pressure per slice (allocated on first use)
    nsp_state gs{nullptr, nullptr, nullptr, nullptr};  // scratch state for the coarse sweep
    LaunchRes L;
    // adjoint workspace (allocated on first use)
    int adj_nck = 0, adj_seg = 0;
    double *adj_ck = nullptr;    // checkpoints: adj_nck full states
    double *adj_segu = nullptr;  // velocities of one segment: adj_seg states
    double *adj_y = nullptr;     // working state
    double *adj_lam = nullptr, *adj_mu = nullptr, *adj_p = nullptr, *adj_glid = nullptr, *adj_part = nullptr;
    double *adj_fin = nullptr;   // dJ/du at the end of the recorded run
    // the recorded forward run (tape) the reverse sweep starts from
    unsigned long long tape = 0, tape_seq = 0;
    unsigned long long lid_version = 0, tape_lid_version = 0;
    int tape_nsteps = 0, tape_ck = 1, tape_nseg = 0;
    double tape_dt = 0.0;
    nsp_poisson_opts tape_opts{};
    int pz = 0;    // periodic in z
    int slip = 0;  // free-slip obstacle walls
    int coarse_upwind = 0;  // the coarse propagator's convection: donor cell instead of SMART
    int max_wg = 0;
    int fixed_wg = 0;
    int force_depth = 0;  // CG column-tile depth in planes, forced during autotuning
    int force_items = 0;  // CG column items per thread forced during autotuning
    std::vector<TuneEntry> tuned;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_ms = 0.0;
    nsp_launch_stats stats[3] = {};  // per launch kind (fine, poisson, project), since the last reset
    std::string err;
};

namespace {

nsp_status fail(nsp_handle *h, nsp_status st, const std::string &msg) {
    if (h) h->err = msg;
    return st;
}

#define HIPCHK(h, call)                                                                                    \
    do {                                                                                                   \
        hipError_t e_ = (call);                                                                            \
        if (e_ != hipSuccess)                                                                              \
            return fail((h), NSP_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));              \
    } while (0)

template <class T>
hipError_t dalloc(T **p, size_t n) {
    if (n == 0) n = 1;
    return hipMalloc(reinterpret_cast<void **>(p), n * sizeof(T));
}

// Tile size: a power of two between kBlock and 2 kBlock cells, about
// ncells/256, fixed by the grid alone so that reductions never depend on
// the batch.  Small tiles keep the window an XCD sweeps at a time (its
// workgroups times one tile, plus one plane on either side) inside its L2.
int tile_for(long long ncells) {
    long long t = kBlock;
    while (t * 2 <= ncells / 256 && t < 2 * kBlock) t *= 2;
    return (int)t;
}

// Cell flags: open faces, fluid, and whether any cell within Chebyshev
// distance 3 is solid or outside the domain (then the momentum stencil of
// the cell's low faces may meet a wall).
void build_flags(int nx, int ny, int nz, const uint8_t *solid, bool pz, std::vector<uint8_t> &fl, double &nfluid) {
    const long long n = (long long)nx * ny * nz;
    auto id = [&](int i, int j, int k) { return ((long long)k * ny + j) * nx + i; };
    // neighbours across the z ends wrap when the domain is periodic in z
    auto fluid = [&](int i, int j, int k) {
        if (pz) k = (k % nz + nz) % nz;
        if (i < 0 || j < 0 || k < 0 || i >= nx || j >= ny || k >= nz) return false;
        return !(solid && solid[id(i, j, k)]);
    };
    fl.assign(n, 0);
    nfluid = 0;
    // blocked[c] = 1 if cell is solid; dilate by 3 in each direction (box);
    // positions beyond any domain face count as blocked, so cells near the
    // periodic seam also take the general (image-rule, wrapping) path
    std::vector<uint8_t> bad(n), tmp(n);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) bad[id(i, j, k)] = !fluid(i, j, k);
    const int R = 3;
    auto dilate = [&](int dir) {
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    uint8_t v = 0;
                    for (int m = -R; m <= R && !v; ++m) {
                        int a = i + (dir == 0) * m, b = j + (dir == 1) * m, c = k + (dir == 2) * m;
                        if (a < 0 || b < 0 || c < 0 || a >= nx || b >= ny || c >= nz) v = 1;
                        else v = bad[id(a, b, c)];
                    }
                    tmp[id(i, j, k)] = v;
                }
        bad.swap(tmp);
    };
    dilate(0);
    dilate(1);
    dilate(2);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                uint8_t f = 0;
                if (fluid(i, j, k)) {
                    f |= FL_FLUID;
                    nfluid += 1;
                    if (fluid(i - 1, j, k)) f |= FL_XM;
                    if (fluid(i + 1, j, k)) f |= FL_XP;
                    if (fluid(i, j - 1, k)) f |= FL_YM;
                    if (fluid(i, j + 1, k)) f |= FL_YP;
                    if (fluid(i, j, k - 1)) f |= FL_ZM;
                    if (fluid(i, j, k + 1)) f |= FL_ZP;
                }
                if (bad[id(i, j, k)]) f |= FL_SLOW;
                fl[id(i, j, k)] = f;
            }
}

// true when the fluid cells form one face-connected region
bool fluid_connected(int nx, int ny, int nz, const std::vector<uint8_t> &fl, double nfluid) {
    // (z neighbours are taken modulo the grid, which only matters across a
    // periodic seam: with walls the z bits at the ends are never set)
    const long long n = (long long)nx * ny * nz;
    long long start = -1;
    for (long long c = 0; c < n; ++c)
        if (fl[c] & FL_FLUID) { start = c; break; }
    if (start < 0) return false;
    std::vector<uint8_t> seen(n, 0);
    std::vector<long long> stack{start};
    seen[start] = 1;
    long long count = 0;
    const long long sy = nx, sz = (long long)nx * ny;
    while (!stack.empty()) {
        long long c = stack.back();
        stack.pop_back();
        ++count;
        const uint8_t f = fl[c];
        const long long nb[6] = {c - 1, c + 1, c - sy, c + sy, (c - sz + n) % n, (c + sz) % n};
        for (int d = 0; d < 6; ++d)
            if ((f >> d) & 1)
                if (!seen[nb[d]]) { seen[nb[d]] = 1; stack.push_back(nb[d]); }
    }
    return (double)count == nfluid;
}

nsp_status ensure_launch_res(nsp_handle *h, int nslices, int ntiles) {
    LaunchRes &L = h->L;
    if (!L.sync) {
        HIPCHK(h, dalloc(&L.sync, 1));
        HIPCHK(h, hipMemset(L.sync, 0, sizeof(SyncWords)));
        HIPCHK(h, dalloc(&L.params, 1));
        HIPCHK(h, hipHostMalloc(reinterpret_cast<void **>(&L.params_host), sizeof(KParams)));
        HIPCHK(h, dalloc(&L.jump, 2 * kMaxGroups));
        HIPCHK(h, hipHostMalloc(reinterpret_cast<void **>(&L.jump_host), 2 * kMaxGroups * sizeof(unsigned long long)));
    }
    if (nslices > L.cap_slices) {
        if (L.ctl) (void)hipFree(L.ctl);
        if (L.ctl_host) (void)hipHostFree(L.ctl_host);
        L.ctl = nullptr;
        L.ctl_host = nullptr;
        HIPCHK(h, dalloc(&L.ctl, nslices));
        HIPCHK(h, hipHostMalloc(reinterpret_cast<void **>(&L.ctl_host), nslices * sizeof(SliceCtl)));
        L.cap_slices = nslices;
    }
    if (ntiles > L.cap_tiles) {
        if (L.part) (void)hipFree(L.part);
        L.part = nullptr;
        HIPCHK(h, dalloc(&L.part, (size_t)2 * kNQ * ntiles));
        L.cap_tiles = ntiles;
    }
    return NSP_OK;
}

bool valid_opts(const nsp_poisson_opts *o) {
    return o && o->rtol >= 0 && o->maxit >= 0 &&
           (o->prec == NSP_FP64 || o->prec == NSP_MIXED || o->prec == NSP_MIXED_RU) &&
           (o->prec == NSP_FP64 || (o->inner_rtol > 0 && o->inner_rtol < 1 && o->max_outer >= 0)) &&
           (o->solver == NSP_PCG || o->solver == NSP_BICGSTAB || o->solver == NSP_PCG_SR) &&
           (o->extrapolate == 0 || o->extrapolate == 1);
}

// number of steps (t1 - t0)/dt, which must be a non-negative integer
bool step_count(double t0, double t1, double dt, int *n) {
    if (!(dt > 0) || !std::isfinite(t0) || !std::isfinite(t1)) return false;
    const double x = (t1 - t0) / dt;
    const double rx = std::nearbyint(x);
    if (rx < 0 || std::fabs(x - rx) > 1e-9 * std::max(1.0, std::fabs(x)) || rx > 1e9) return false;
    *n = (int)rx;
    return true;
}

void fill_group(GroupDesc &G, nsp_handle *h, nsp_state y, int slice_off, int nslices, int slice0, int tile0,
                const double *bin, int cgtile0 = -1) {
    G.nx = h->nx;
    G.ny = h->ny;
    G.nz = h->nz;
    G.ncells = (int)h->ncells;
    G.nu = (int)h->nu;
    G.nv = (int)h->nv;
    G.nw = (int)h->nw;
    G.tile = h->tile;
    G.ntiles = h->ntiles;
    G.nslices = nslices;
    G.slice0 = slice0;
    G.tile0 = tile0;
    G.cby = h->cby;
    G.cbz = h->cbz;
    G.cny = h->cny;
    G.cnz = h->cnz;
    G.crb = h->crb;
    G.zsh = h->zsh;
    G.cni = 1;
    G.cnb = h->cnb;
    G.cgtiles = h->cgtiles;
    G.cgtile0 = cgtile0 >= 0 ? cgtile0 : slice0 * h->cgtiles;
    G.cgparts = h->cgparts;
    G.cgpart0 = slice0 * h->cgparts;  // launch prefixes are recomputed by run()
    G.nfluid = h->nfluid;
    G.pz = h->pz;
    G.slip = h->slip;
    G.upwind = 0;
    const double hh[3] = {h->lx / h->nx, h->ly / h->ny, h->lz / h->nz};
    for (int d = 0; d < 3; ++d) {
        G.ih[d] = 1.0 / hh[d];
        G.ih2[d] = 1.0 / (hh[d] * hh[d]);
        G.ih2f[d] = (float)G.ih2[d];
    }
    G.inv_re = 1.0 / h->re;
    G.flags = h->flags;
    G.lid = h->lid;
    G.idiag = h->idiag;
    G.idiag32 = h->idiag32;
    G.u = y.u ? y.u + (long long)slice_off * h->nu : nullptr;
    G.v = y.v ? y.v + (long long)slice_off * h->nv : nullptr;
    G.w = y.w ? y.w + (long long)slice_off * h->nw : nullptr;
    G.p = y.p ? y.p + (long long)slice_off * h->ncells : nullptr;
    G.pprev = nullptr;  // set by plan_launch when the launch extrapolates the warm start
    G.Fu = h->Fu;
    G.Fv = h->Fv;
    G.Fw = h->Fw;
    G.b = h->b;
    G.r = h->r;
    G.d0 = h->d0;
    G.d1 = h->d1;
    G.q = h->q;
    G.e = h->e;
    G.bv0 = h->bv0;
    G.bv1 = h->bv1;
    G.brh = h->brh;
    G.bin = bin;
}

int auto_workgroups(nsp_handle *h, int batch, int prec, int total_tiles) {
    if (h->fixed_wg > 0) return std::min(h->fixed_wg, std::min(h->max_wg, total_tiles));
    for (const TuneEntry &t : h->tuned)
        if (t.batch == batch && t.prec == prec) return std::min(t.workgroups, std::min(h->max_wg, total_tiles));
    return std::min(h->max_wg, total_tiles);
}

// Launch prefixes of the groups' tiles and partials, the CG tile depth and
// the items per thread.  Items: `items` if > 0, else in FP32 launches (fp32
// != 0) the count with the shorter estimated critical path, the largest
// number of plane steps one workgroup makes (tiles per workgroup x planes per
// tile), a two-item plane step costing 1.75 one-item ones (measured on 96^3
// and 128^3 batches); FP64 launches always use one item (two FP64 items would
// not fit the LDS plane buffers).  Depth D in planes, the same for every
// grid of the launch (a grid never goes below its zsub): `depth` if > 0,
// else the deepest of 32 and 16 planes that leaves at least two CG tiles per
// workgroup (deeper tiles refill the z pipeline less often), else 8 planes,
// or 4 when even 8-plane tiles leave workgroups idle.  Partial sums stay per
// crb rows and zsub planes, so neither choice changes a result.
void layout_groups(GroupDesc *G, int ngroups, int wg, int depth, int items, int fp32, int *ntiles, int *cgtiles,
                   int *cgparts) {
    auto planes = [](const GroupDesc &X, int D) { return std::max(D, 1 << X.zsh); };
    auto count = [&](int ni, int D) {
        long long t = 0;
        for (int g = 0; g < ngroups; ++g) {
            const GroupDesc &X = G[g];
            if (X.crb > 0) {
                const int rows = ni * X.crb, pl = planes(X, D);
                t += (long long)X.nslices * ((X.ny + rows - 1) / rows) * ((X.nz + pl - 1) / pl);
            } else {
                t += (long long)X.nslices * X.cgtiles;
            }
        }
        return t;
    };
    // estimated plane steps of the busiest workgroup, in quarters of a one-item step
    auto path = [&](int ni) {
        long long best = -1;
        for (int D : {8, 16, 32}) {
            const long long c = (count(ni, D) + wg - 1) / wg * D * (ni == 2 ? 7 : 4);
            if (best < 0 || c < best) best = c;
        }
        return best;
    };
    bool two = fp32 != 0, four = false;
    for (int g = 0; g < ngroups; ++g) {
        if (G[g].crb > 0 && G[g].cnb < 2) two = false;
        if (G[g].crb > 0 && G[g].zsh == 2) four = true;
    }
    if (!two) items = 1;
    if (items <= 0) items = path(2) < path(1) ? 2 : 1;
    if (depth <= 0) {
        depth = 8;
        for (int D : {32, 16})
            if (count(items, D) >= 2LL * wg) { depth = D; break; }
        if (depth == 8 && four && count(items, 8) < wg) depth = 4;
    }
    *ntiles = *cgtiles = *cgparts = 0;
    int slice0 = 0;
    for (int g = 0; g < ngroups; ++g) {
        GroupDesc &X = G[g];
        if (X.crb > 0) {
            X.cni = items;
            X.cby = std::min(items * X.crb, X.ny);
            X.cny = (X.ny + X.cby - 1) / X.cby;
            X.cbz = planes(X, depth);
            X.cnz = (X.nz + X.cbz - 1) / X.cbz;
            X.cgtiles = X.cny * X.cnz;
        }
        X.slice0 = slice0;
        X.tile0 = *ntiles;
        X.cgtile0 = *cgtiles;
        X.cgpart0 = *cgparts;
        slice0 += X.nslices;
        *ntiles += X.nslices * X.ntiles;
        *cgtiles += X.nslices * X.cgtiles;
        *cgparts += X.nslices * X.cgparts;
    }
}

// Launch the persistent kernel over ngroups groups and read back the
// per-slice control blocks into info (may be NULL).
// The launch shape and parameter block of one persistent launch (resource
// pointers not yet set); no device work.
struct LaunchPlan {
    GroupDesc lg[kMaxGroups];
    int ngroups = 0, nslices = 0, wg = 0, pstride = 0;
    KParams P;
};

nsp_status plan_launch(nsp_handle *const *hs, int ngroups, const GroupDesc *groups, int mode, int nsteps, double dt,
                       const nsp_poisson_opts *o, int workgroups_override, bool caller_ws, LaunchPlan &pl) {
    nsp_handle *h = hs[0];
    int nslices = 0, ntiles = 0, cgtiles = 0;
    for (int g = 0; g < ngroups; ++g) {
        nslices += groups[g].nslices;
        ntiles += groups[g].nslices * groups[g].ntiles;
        cgtiles += groups[g].nslices * groups[g].cgtiles;
    }
    pl.nslices = nslices;
    pl.ngroups = ngroups;
    if (nslices <= 0) return NSP_OK;
    if (nslices > kMaxSlices) return fail(h, NSP_ERR_ARG, "more than 64 slices in one launch");
    if (ngroups > kMaxGroups) return fail(h, NSP_ERR_ARG, "too many grids in one launch");
    if (o->solver != NSP_PCG && o->prec != NSP_FP64)
        return fail(h, NSP_ERR_UNSUPPORTED, "BiCGStab and single-reduction PCG run in FP64 only");
    // workgroups from the finest tiling, then the tile depth for that count
    const int units = std::max(ntiles, cgtiles);
    int wg = workgroups_override > 0 ? std::min(workgroups_override, std::min(h->max_wg, units))
                                     : auto_workgroups(h, nslices, o->prec != NSP_FP64 ? 1 : 0, units);
    if (wg < 1) wg = 1;
    if (wg > kMaxWG) wg = kMaxWG;
    GroupDesc *lg = pl.lg;
    for (int g = 0; g < ngroups; ++g) lg[g] = groups[g];
    // caller_ws: launch workspace brought in by the caller (every vector
    // pointer of the groups already set); nothing is allocated then
    if (o->solver != NSP_PCG && !caller_ws)
        for (int g = 0; g < ngroups; ++g) {
            nsp_handle *hg = hs[g];
            if (!hg->bv0) {
                const size_t n = (size_t)hg->max_batch * hg->ncells;
                HIPCHK(h, dalloc(&hg->bv0, n));
                HIPCHK(h, dalloc(&hg->bv1, n));
                HIPCHK(h, dalloc(&hg->brh, n));
            }
            lg[g].bv0 = hg->bv0;
            lg[g].bv1 = hg->bv1;
            lg[g].brh = hg->brh;
        }
    // extrapolated warm start: every grid of the launch needs its previous-
    // pressure array (one cell array per slice of max_batch)
    const bool extrap = o->extrapolate != 0 && mode == MODE_FINE && nsteps > 1;
    if (extrap) {
        if (caller_ws) return fail(h, NSP_ERR_UNSUPPORTED, "the extrapolated warm start needs the handle's workspace");
        for (int g = 0; g < ngroups; ++g) {
            nsp_handle *hg = hs[g];
            if (!hg->pprev) HIPCHK(h, dalloc(&hg->pprev, (size_t)hg->max_batch * hg->ncells));
            lg[g].pprev = hg->pprev;
        }
    }
    int depth = h->force_depth, items = h->force_items;
    if (depth <= 0 && items <= 0)
        for (const TuneEntry &t : h->tuned)
            if (t.batch == nslices && t.prec == (o->prec != NSP_FP64 ? 1 : 0)) {
                depth = t.depth;
                items = t.items;
            }
    int cgparts = 0;
    layout_groups(lg, ngroups, wg, depth, items, o->prec != NSP_FP64, &ntiles, &cgtiles, &cgparts);
    const int pstride = std::max(ntiles, cgparts);
    pl.wg = wg;
    pl.pstride = pstride;
    KParams &P = pl.P;
    std::memset(&P, 0, sizeof(P));
    for (int g = 0; g < ngroups; ++g) P.g[g] = lg[g];
    P.ngroups = ngroups;
    P.nslices = nslices;
    P.ntiles = ntiles;
    P.cgtiles = cgtiles;
    P.pstride = pstride;
    P.mode = mode;
    P.nsteps = nsteps;
    P.prec = o->prec == NSP_MIXED ? 1 : (o->prec == NSP_MIXED_RU ? 2 : 0);
    P.maxit = o->maxit;
    P.max_outer = o->max_outer;
    P.xcd_remap = 1;
    P.solver = o->solver;
    P.extrap = extrap ? 1 : 0;
    {
        // write-through CG stores while the launch is cache-resident (<= 8 M cells)
        long long cells = 0;
        for (int g = 0; g < ngroups; ++g) cells += (long long)lg[g].nslices * lg[g].ncells;
        P.wt = cells <= (8LL << 20) ? 1 : 0;
    }
    {
        // registers hold the CG vectors when every CG tile has its own
        // workgroup (PCG, FP64 or the FP32 inner solve)
        bool rr = o->solver == NSP_PCG && cgtiles <= wg;
        for (int g = 0; g < ngroups; ++g) {
            const GroupDesc &X = lg[g];
            rr = rr && X.cby > 0 && X.cni == 1 && X.cbz == (1 << X.zsh) && (X.cbz == 4 || X.cbz == 8) &&
                 X.nz % X.cbz == 0;
            // the loop publishes boundary values in d0, d1 and q
            rr = rr && X.d0 && X.d1 && X.q && X.r && (o->prec == NSP_FP64 || X.e);
        }
        P.rr = rr ? 1 : 0;
    }
    P.dt = dt;
    P.rtol = o->rtol;
    P.eta = o->inner_rtol;
    return NSP_OK;
}

// Per-slice results of a finished launch (control blocks copied to the
// host): launch statistics, info, and the status; `worst` is the worst
// slice status to report (the launch's own, or one kept across replays).
nsp_status collect_status(nsp_handle *h, const LaunchPlan &pl, const SliceCtl *ctl_host, float ms, int worst,
                          nsp_solve_info *info, int launches = 1) {
    const KParams &P = pl.P;
    const int mode = P.mode;
    nsp_launch_stats &S = h->stats[mode];
    S.launches += launches;
    S.rr_launches += (long long)P.rr * launches;
    S.ms += ms;
    for (int g = 0, s = 0; g < pl.ngroups; ++g)
        for (int k = 0; k < pl.lg[g].nslices; ++k, ++s) {
            const SliceCtl &c = ctl_host[s];
            const double cells = (double)pl.lg[g].ncells, it = cells * c.tot_it;
            S.cell_steps += cells * (mode == MODE_FINE ? P.nsteps : 1) * launches;
            S.cg_cell_iters += it;
            S.cell_sweeps += cells * c.tot_outer;
            if (P.prec != 0) {
                S.cg32_cell_iters += it;
                S.mixed_cell_sweeps += cells * c.tot_outer;
            } else if (P.solver == NSP_BICGSTAB) {
                S.bicg_cell_iters += it;
            } else {
                S.cg64_cell_iters += it;
            }
        }
    for (int s = 0; s < pl.nslices; ++s) {
        const SliceCtl &c = ctl_host[s];
        if (info) {
            info[s].iters = c.tot_it;
            info[s].max_iters = c.max_it;
            info[s].outer = c.tot_outer;
            info[s].status = c.status;
            info[s].rel_res_true = c.rel_true;
            info[s].div_l2 = mode == MODE_FINE ? P.dt * c.res_true : 0.0;
        }
    }
    if (worst == 2) return fail(h, NSP_ERR_NOT_CONVERGED, "Poisson solve reached its iteration limit");
    if (worst == 3) return fail(h, NSP_ERR_NONFINITE, "non-finite residual in the Poisson solve");
    return NSP_OK;
}

nsp_status run(nsp_handle *const *hs, int ngroups, const GroupDesc *groups, int mode, int nsteps, double dt,
               const nsp_poisson_opts *o, hipStream_t stream, nsp_solve_info *info, int workgroups_override,
               const LaunchRes *ws = nullptr) {
    nsp_handle *h = hs[0];
    LaunchPlan pl;
    nsp_status st = plan_launch(hs, ngroups, groups, mode, nsteps, dt, o, workgroups_override, ws != nullptr, pl);
    if (st != NSP_OK || pl.nslices <= 0) return st;
    const int nslices = pl.nslices;
    if (ws) {
        if (nslices > ws->cap_slices || pl.pstride > ws->cap_tiles)
            return fail(h, NSP_ERR_ARG, "launch workspace too small for this launch");
    } else {
        st = ensure_launch_res(h, nslices, pl.pstride);
        if (st != NSP_OK) return st;
    }
    const LaunchRes &L = ws ? *ws : h->L;
    KParams &P = *L.params_host;
    // the pinned block may still be read by an earlier copy on this stream
    HIPCHK(h, hipStreamSynchronize(stream));
    P = pl.P;
    P.ctl = L.ctl;
    P.part = L.part;
    P.sync = L.sync;
    static_assert(sizeof(SliceCtl) % sizeof(unsigned) == 0, "control blocks are zeroed as words");
    HIPCHK(h, launch_zero_words(L.ctl, (long long)nslices * (sizeof(SliceCtl) / sizeof(unsigned)), stream));
    HIPCHK(h, hipMemcpyAsync(L.params, &P, sizeof(KParams), hipMemcpyHostToDevice, stream));
    HIPCHK(h, launch_reset_sync(L.sync, stream));
    HIPCHK(h, hipEventRecord(h->ev0, stream));
    HIPCHK(h, launch_persistent(L.params, pl.wg, P.rr != 0, stream));
    HIPCHK(h, hipEventRecord(h->ev1, stream));
    HIPCHK(h, hipMemcpyAsync(L.ctl_host, L.ctl, nslices * sizeof(SliceCtl), hipMemcpyDeviceToHost, stream));
    int aborted = 0;
    HIPCHK(h, hipMemcpyAsync(&aborted, &L.sync->abort, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIPCHK(h, hipStreamSynchronize(stream));
    float ms = 0;
    if (hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) h->last_ms = ms;
    if (aborted) return fail(h, NSP_ERR_HIP, "grid barrier wait exceeded its limit; launch abandoned");
    int worst = 0;
    for (int s = 0; s < nslices; ++s) worst = std::max(worst, L.ctl_host[s].status);
    return collect_status(h, pl, L.ctl_host, ms, worst, info);
}

bool state_ok(const nsp_state &y) { return y.u && y.v && y.w && y.p; }

nsp_state offset_state(nsp_handle *h, nsp_state y, long long slice) {
    nsp_state o;
    o.u = y.u + slice * h->nu;
    o.v = y.v + slice * h->nv;
    o.w = y.w + slice * h->nw;
    o.p = y.p + slice * h->ncells;
    return o;
}

hipError_t copy_slices(nsp_handle *h, nsp_state dst, nsp_state src, long long n, hipStream_t s) {
    hipError_t e;
    if ((e = launch_copy_state(dst.u, src.u, n * h->nu, s)) != hipSuccess) return e;
    if ((e = launch_copy_state(dst.v, src.v, n * h->nv, s)) != hipSuccess) return e;
    if ((e = launch_copy_state(dst.w, src.w, n * h->nw, s)) != hipSuccess) return e;
    return launch_copy_state(dst.p, src.p, n * h->ncells, s);
}

// coarse: the steps of a coarse propagator (each handle's coarse convection)
nsp_status propagate(nsp_handle *const *hs, const nsp_state *ys, const int *batches, int ngroups, double t0,
                     double t1, double step, const nsp_poisson_opts *o, void *stream, nsp_solve_info *info,
                     bool coarse = false) {
    if (!hs || !ys || !batches || ngroups < 1 || ngroups > kMaxGroups || !hs[0])
        return fail(hs ? hs[0] : nullptr, NSP_ERR_ARG, "bad group arguments");
    nsp_handle *h = hs[0];
    if (!valid_opts(o)) return fail(h, NSP_ERR_ARG, "invalid Poisson options");
    int nsteps = 0;
    if (!step_count(t0, t1, step, &nsteps)) return fail(h, NSP_ERR_ARG, "(t1 - t0)/dt is not a non-negative integer");
    // groups with an empty batch take no part (their pointers may be null)
    GroupDesc G[kMaxGroups];
    nsp_handle *used[kMaxGroups];
    int ng = 0, slice0 = 0, tile0 = 0, cgtile0 = 0;
    for (int g = 0; g < ngroups; ++g) {
        if (!hs[g] || batches[g] < 0 || batches[g] > hs[g]->max_batch)
            return fail(h, NSP_ERR_ARG, "null handle or batch outside [0, max_batch]");
        if (batches[g] == 0) continue;
        if (!state_ok(ys[g])) return fail(h, NSP_ERR_ARG, "null state pointer");
        fill_group(G[ng], hs[g], ys[g], 0, batches[g], slice0, tile0, nullptr, cgtile0);
        G[ng].upwind = coarse ? hs[g]->coarse_upwind : 0;
        used[ng++] = hs[g];
        slice0 += batches[g];
        tile0 += batches[g] * hs[g]->ntiles;
        cgtile0 += batches[g] * hs[g]->cgtiles;
    }
    if (nsteps == 0 || slice0 == 0) return NSP_OK;
    return run(used, ng, G, MODE_FINE, nsteps, step, o, static_cast<hipStream_t>(stream), info, 0);
}

// A coarse handle for the coarser-grid coarse propagator: half the cells of
// the fine grid in every direction, the same box and boundaries, no obstacles.
nsp_status check_pair(nsp_handle *h, nsp_handle *hc) {
    if (!h || !hc) return fail(h ? h : hc, NSP_ERR_ARG, "null handle");
    if (h->nx != 2 * hc->nx || h->ny != 2 * hc->ny || h->nz != 2 * hc->nz)
        return fail(h, NSP_ERR_ARG, "the coarse grid must have half the fine grid's cells in every direction");
    if (h->lx != hc->lx || h->ly != hc->ly || h->lz != hc->lz || h->pz != hc->pz)
        return fail(h, NSP_ERR_ARG, "fine and coarse grids must cover the same box with the same boundaries");
    if (h->nfluid != (double)h->ncells || hc->nfluid != (double)hc->ncells)
        return fail(h, NSP_ERR_UNSUPPORTED, "the coarser-grid coarse propagator takes grids without obstacles");
    return NSP_OK;
}

// fine -> coarse (restriction) or coarse -> fine (prolongation) of `batch`
// slices; h is the fine handle
hipError_t transfer(nsp_handle *h, nsp_state src, nsp_state dst, int batch, bool prolong, hipStream_t s) {
    TransferParams T;
    T.prolong = prolong ? 1 : 0;
    T.nx = h->nx;
    T.ny = h->ny;
    T.nz = h->nz;
    T.batch = batch;
    T.src[0] = src.u;
    T.src[1] = src.v;
    T.src[2] = src.w;
    T.src[3] = src.p;
    T.dst[0] = dst.u;
    T.dst[1] = dst.v;
    T.dst[2] = dst.w;
    T.dst[3] = dst.p;
    return launch_transfer(T, s);
}

// Coarse propagator over one slice for every group: hs[g]->gs <- G(Y[g] slice
// n) with G on the handle's own grid, or, with coarse handles hcs, G~ =
// P(G_c(R(y))) on hcs[g]'s grid.
nsp_status coarse_slice(nsp_handle *const *hs, nsp_handle *const *hcs, const nsp_state *Y, int ngroups, int n,
                        double t0, double t1, double DT, const nsp_poisson_opts *coarse, hipStream_t s) {
    nsp_handle *h = hs[0];
    nsp_state gsv[kMaxGroups];
    int ones[kMaxGroups];
    for (int g = 0; g < ngroups; ++g) {
        ones[g] = 1;
        if (hcs) {
            HIPCHK(h, transfer(hs[g], offset_state(hs[g], Y[g], n), hcs[g]->gs, 1, false, s));
            gsv[g] = hcs[g]->gs;
        } else {
            HIPCHK(h, copy_slices(hs[g], hs[g]->gs, offset_state(hs[g], Y[g], n), 1, s));
            gsv[g] = hs[g]->gs;
        }
    }
    nsp_status st = propagate(hcs ? hcs : hs, gsv, ones, ngroups, t0, t1, DT, coarse, s, nullptr, true);
    if (hcs && st != NSP_OK) h->err = "coarse grid: " + hcs[0]->err;
    if (st != NSP_OK && st != NSP_ERR_NOT_CONVERGED) return st;
    if (hcs)
        for (int g = 0; g < ngroups; ++g) HIPCHK(h, transfer(hs[g], hcs[g]->gs, hs[g]->gs, 1, true, s));
    // a coarse solve that hit its limit still leaves its best iterate in gs
    return st;
}

// the worse of two statuses where the call goes on (OK < NOT_CONVERGED)
nsp_status worse(nsp_status a, nsp_status b) { return (a == NSP_ERR_NOT_CONVERGED || b == NSP_ERR_NOT_CONVERGED) ? NSP_ERR_NOT_CONVERGED : NSP_OK; }

nsp_status parareal_start_impl(nsp_handle *const *hs, nsp_handle *const *hcs, const nsp_state *Y,
                               const nsp_state *Gk, int ngroups, int nslices, double t0, double T, double DT,
                               const nsp_poisson_opts *coarse, void *stream) {
    if (!hs || !Y || !Gk || ngroups < 1 || ngroups > kMaxGroups || !hs[0] || nslices < 1)
        return fail(hs ? hs[0] : nullptr, NSP_ERR_ARG, "bad Parareal arguments");
    nsp_handle *h = hs[0];
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double len = (T - t0) / nslices;
    int nc = 0;
    if (!step_count(0.0, len, DT, &nc)) return fail(h, NSP_ERR_ARG, "slice length / DT is not an integer");
    for (int g = 0; g < ngroups; ++g)
        if (!hs[g] || !state_ok(Y[g]) || !state_ok(Gk[g])) return fail(h, NSP_ERR_ARG, "null state");
    nsp_status worst = NSP_OK;
    std::string msg;
    for (int n = 0; n < nslices; ++n) {
        nsp_status st = coarse_slice(hs, hcs, Y, ngroups, n, t0 + n * len, t0 + (n + 1) * len, DT, coarse, s);
        if (st != NSP_OK && st != NSP_ERR_NOT_CONVERGED) return st;
        if (st != NSP_OK && worst == NSP_OK) msg = h->err;
        worst = worse(worst, st);
        for (int g = 0; g < ngroups; ++g) {
            HIPCHK(h, copy_slices(hs[g], offset_state(hs[g], Y[g], n + 1), hs[g]->gs, 1, s));
            HIPCHK(h, copy_slices(hs[g], offset_state(hs[g], Gk[g], n), hs[g]->gs, 1, s));
        }
    }
    HIPCHK(h, hipStreamSynchronize(s));
    if (worst != NSP_OK) return fail(h, worst, "coarse sweep: " + msg);
    return NSP_OK;
}

nsp_status parareal_iterate_impl(nsp_handle *const *hs, nsp_handle *const *hcs, const nsp_state *Y,
                                 const nsp_state *Fk, const nsp_state *Gk, int ngroups, int nslices, int k, double t0,
                                 double T, double dt, double DT, const nsp_poisson_opts *fine,
                                 const nsp_poisson_opts *coarse, void *stream, double *jump) {
    if (!hs || !Y || !Fk || !Gk || ngroups < 1 || ngroups > kMaxGroups || !hs[0] || nslices < 1 || k < 0 || !jump)
        return fail(hs ? hs[0] : nullptr, NSP_ERR_ARG, "bad Parareal arguments");
    nsp_handle *h = hs[0];
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double len = (T - t0) / nslices;
    int nf = 0, nc = 0;
    if (!step_count(0.0, len, dt, &nf) || !step_count(0.0, len, DT, &nc))
        return fail(h, NSP_ERR_ARG, "slice length / dt or / DT is not an integer");
    for (int g = 0; g < ngroups; ++g) {
        if (!hs[g] || !state_ok(Y[g]) || !state_ok(Fk[g]) || !state_ok(Gk[g]))
            return fail(h, NSP_ERR_ARG, "null state");
        if (hs[g]->max_batch < nslices) return fail(h, NSP_ERR_ARG, "max_batch is smaller than nslices");
    }
    for (int g = 0; g < 2 * ngroups; ++g) jump[g] = 0.0;
    if (k >= nslices) return NSP_OK;  // every slice is already exact
    const int active = nslices - k;
    // F(Y[n]) for n >= k, all grids' slices in one launch
    nsp_state fsub[kMaxGroups];
    int nb[kMaxGroups];
    for (int g = 0; g < ngroups; ++g) {
        HIPCHK(h, copy_slices(hs[g], offset_state(hs[g], Fk[g], k), offset_state(hs[g], Y[g], k), active, s));
        fsub[g] = offset_state(hs[g], Fk[g], k);
        nb[g] = active;
    }
    nsp_status st = propagate(hs, fsub, nb, ngroups, t0 + k * len, t0 + (k + 1) * len, dt, fine, stream, nullptr);
    if (st != NSP_OK && st != NSP_ERR_NOT_CONVERGED) return st;
    // a solve that hit its limit does not stop the iteration: its best iterate
    // enters Eq. (6), and the call reports NOT_CONVERGED at the end
    nsp_status worst = st;
    std::string msg = st != NSP_OK ? "fine sweep: " + h->err : std::string();
    HIPCHK(h, hipMemsetAsync(h->L.jump, 0, 2 * kMaxGroups * sizeof(unsigned long long), s));
    for (int n = k; n < nslices; ++n) {
        st = coarse_slice(hs, hcs, Y, ngroups, n, t0 + n * len, t0 + (n + 1) * len, DT, coarse, s);
        if (st != NSP_OK && st != NSP_ERR_NOT_CONVERGED) return st;
        if (st != NSP_OK && worst == NSP_OK) msg = "coarse sweep: " + h->err;
        worst = worse(worst, st);
        UpdateParams U;
        std::memset(&U, 0, sizeof(U));
        U.jump = h->L.jump;
        for (int g = 0; g < ngroups; ++g) {
            nsp_handle *hg = hs[g];
            const nsp_state y1 = offset_state(hg, Y[g], n + 1), f = offset_state(hg, Fk[g], n),
                            go = offset_state(hg, Gk[g], n);
            double *ys[4] = {y1.u, y1.v, y1.w, y1.p};
            const double *fs[4] = {f.u, f.v, f.w, f.p};
            const double *gn[4] = {hg->gs.u, hg->gs.v, hg->gs.w, hg->gs.p};
            double *gos[4] = {go.u, go.v, go.w, go.p};
            const long long ns[4] = {hg->nu, hg->nv, hg->nw, hg->ncells};
            for (int c = 0; c < 4; ++c) {
                UpdateSeg &S = U.seg[U.nseg];
                S.y = ys[c];
                S.f = fs[c];
                S.g = gn[c];
                S.gold = gos[c];
                S.n = ns[c];
                S.jslot = c == 3 ? 1 : 0;
                U.group_of_seg[U.nseg] = g;
                ++U.nseg;
            }
        }
        HIPCHK(h, launch_parareal_update(U, s));
    }
    HIPCHK(h, hipMemcpyAsync(h->L.jump_host, h->L.jump, 2 * kMaxGroups * sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    for (int g = 0; g < 2 * ngroups; ++g) {
        double v;
        std::memcpy(&v, &h->L.jump_host[g], sizeof(v));
        jump[g] = v;
    }
    if (worst != NSP_OK) return fail(h, worst, msg);
    return NSP_OK;
}

}  // namespace

// A recorded fine step (nsp_fine_step_graph_create): a HIP graph of one
// persistent launch with launch resources of its own (parameter block,
// control blocks, partial sums, barrier words), so eager calls on the same
// handle between replays leave it intact.
struct nsp_graph {
    nsp_handle *h = nullptr;
    LaunchPlan pl;
    LaunchRes L;                   // params, ctl, ctl_host, part, sync
    GraphFold *fold = nullptr;     // device
    GraphFold *fold_host = nullptr;  // pinned
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int replays = 0;  // since the last nsp_graph_finish
};

namespace {

void free_graph(nsp_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    void *dev[] = {g->L.params, g->L.ctl, g->L.part, g->L.sync, g->fold};
    for (void *q : dev)
        if (q) (void)hipFree(q);
    if (g->L.ctl_host) (void)hipHostFree(g->L.ctl_host);
    if (g->fold_host) (void)hipHostFree(g->fold_host);
    if (g->ev0) (void)hipEventDestroy(g->ev0);
    if (g->ev1) (void)hipEventDestroy(g->ev1);
    delete g;
}

}  // namespace

extern "C" {

const char *nsp_last_error(const nsp_handle *h) { return h ? h->err.c_str() : "null handle"; }

nsp_status nsp_create(const nsp_grid *g, nsp_handle **out) {
    if (!g || !out) return NSP_ERR_ARG;
    *out = nullptr;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || !(g->lx > 0) || !(g->ly > 0) || !(g->lz > 0) || !(g->re > 0) ||
        g->max_batch < 1 || g->max_batch > kMaxSlices || (g->slip_obstacles != 0 && g->slip_obstacles != 1))
        return NSP_ERR_ARG;
    if ((long long)g->nx * g->ny * g->nz > (1LL << 30)) return NSP_ERR_ARG;
    nsp_handle *h = new (std::nothrow) nsp_handle();
    if (!h) return NSP_ERR_ARG;
    if (hipGetDevice(&h->device) != hipSuccess) { delete h; return NSP_ERR_HIP; }
    h->nx = g->nx; h->ny = g->ny; h->nz = g->nz;
    h->lx = g->lx; h->ly = g->ly; h->lz = g->lz;
    h->re = g->re;
    h->max_batch = g->max_batch;
    h->pz = g->periodic_z ? 1 : 0;
    h->slip = g->slip_obstacles;
    h->ncells = (long long)g->nx * g->ny * g->nz;
    h->nu = (long long)(g->nx + 1) * g->ny * g->nz;
    h->nv = (long long)g->nx * (g->ny + 1) * g->nz;
    h->nw = (long long)g->nx * g->ny * (g->nz + 1);
    h->tile = tile_for(h->ncells);
    h->ntiles = (int)((h->ncells + h->tile - 1) / h->tile);
    // CG column tiles for grids of at least 64^3 cells where two x rows fit in
    // a workgroup (nx a multiple of 32, so halo rows are whole waves): cby rows
    // (one workgroup-wide plane patch) by zsub planes (set below, once the
    // workgroup count is known)
    if (2 * g->nx <= kBlock && g->nx % 32 == 0 && h->ncells >= (1LL << 18)) {
        h->cby = h->crb = std::min(kBlock / g->nx, g->ny);
        h->cnb = (g->ny + h->crb - 1) / h->crb;
        h->cny = (g->ny + h->cby - 1) / h->cby;
    } else {
        h->cby = h->cbz = h->cny = h->cnz = h->crb = h->cnb = 0;
        h->cgtiles = h->ntiles;
        h->cgparts = h->ntiles;
    }
    std::vector<uint8_t> fl;
    build_flags(g->nx, g->ny, g->nz, g->solid_host, h->pz != 0, fl, h->nfluid);
    if (!fluid_connected(g->nx, g->ny, g->nz, fl, h->nfluid)) {
        delete h;
        return NSP_ERR_ARG;
    }
    // Jacobi table: 1/diag(A) for each of the 64 open-face patterns
    const double hh[3] = {g->lx / g->nx, g->ly / g->ny, g->lz / g->nz};
    double tab[64];
    float tab32[64];
    for (int m = 0; m < 64; ++m) {
        double dg = 0.0;
        for (int d = 0; d < 3; ++d)
            for (int s = 0; s < 2; ++s)
                if (m & (1 << (2 * d + s))) dg += 1.0 / (hh[d] * hh[d]);
        tab[m] = dg > 0 ? 1.0 / dg : 0.0;
        tab32[m] = dg > 0 ? (float)(1.0 / dg) : 0.0f;
    }
    const long long B = g->max_batch;
    auto fail_create = [&](hipError_t) {
        nsp_destroy(h);
        return NSP_ERR_HIP;
    };
    hipError_t e;
    if ((e = dalloc(&h->flags, h->ncells)) != hipSuccess) return fail_create(e);
    if ((e = hipMemcpy(h->flags, fl.data(), h->ncells, hipMemcpyHostToDevice)) != hipSuccess) return fail_create(e);
    std::vector<double> lid((size_t)g->nz * (g->nx + 1), 1.0);
    if ((e = dalloc(&h->lid, lid.size())) != hipSuccess) return fail_create(e);
    if ((e = hipMemcpy(h->lid, lid.data(), lid.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
        return fail_create(e);
    if ((e = dalloc(&h->idiag, 64)) != hipSuccess) return fail_create(e);
    if ((e = dalloc(&h->idiag32, 64)) != hipSuccess) return fail_create(e);
    if ((e = hipMemcpy(h->idiag, tab, sizeof(tab), hipMemcpyHostToDevice)) != hipSuccess) return fail_create(e);
    if ((e = hipMemcpy(h->idiag32, tab32, sizeof(tab32), hipMemcpyHostToDevice)) != hipSuccess) return fail_create(e);
    if ((e = dalloc(&h->Fu, B * h->nu)) != hipSuccess) return fail_create(e);
    if ((e = dalloc(&h->Fv, B * h->nv)) != hipSuccess) return fail_create(e);
    if ((e = dalloc(&h->Fw, B * h->nw)) != hipSuccess) return fail_create(e);
    if ((e = dalloc(&h->b, B * h->ncells)) != hipSuccess) return fail_create(e);
    if ((e = dalloc(&h->r, B * h->ncells)) != hipSuccess) return fail_create(e);
    if ((e = dalloc(&h->d0, B * h->ncells)) != hipSuccess) return fail_create(e);
    if ((e = dalloc(&h->d1, B * h->ncells)) != hipSuccess) return fail_create(e);
    if ((e = dalloc(&h->q, B * h->ncells)) != hipSuccess) return fail_create(e);
    if ((e = dalloc(&h->e, B * h->ncells)) != hipSuccess) return fail_create(e);
    if ((e = dalloc(&h->gs.u, h->nu)) != hipSuccess) return fail_create(e);
    if ((e = dalloc(&h->gs.v, h->nv)) != hipSuccess) return fail_create(e);
    if ((e = dalloc(&h->gs.w, h->nw)) != hipSuccess) return fail_create(e);
    if ((e = dalloc(&h->gs.p, h->ncells)) != hipSuccess) return fail_create(e);
    if ((e = hipEventCreate(&h->ev0)) != hipSuccess) return fail_create(e);
    if ((e = hipEventCreate(&h->ev1)) != hipSuccess) return fail_create(e);
    if ((e = max_coresident_workgroups(h->device, &h->max_wg)) != hipSuccess) return fail_create(e);
    if (h->max_wg < 1) return fail_create(hipErrorInvalidValue);
    if (h->crb > 0) {
        // partial sums per 8 planes, or per 4 where one slice has fewer
        // 8-plane tiles than workgroups (shallower tiles then keep more of the
        // chip busy); fixed for the grid, so every launch sums alike
        h->zsh = (long long)h->cnb * ((g->nz + 7) / 8) < h->max_wg ? 2 : 3;
        h->cbz = 1 << h->zsh;
        h->cnz = (g->nz + h->cbz - 1) / h->cbz;
        h->cgtiles = h->cny * h->cnz;
        h->cgparts = h->cgtiles;
    }
    if (ensure_launch_res(h, g->max_batch, g->max_batch * std::max(h->ntiles, h->cgtiles)) != NSP_OK)
        return fail_create(hipErrorOutOfMemory);
    *out = h;
    return NSP_OK;
}

nsp_status nsp_destroy(nsp_handle *h) {
    if (!h) return NSP_ERR_ARG;
    (void)hipDeviceSynchronize();
    void *ptrs[] = {h->flags, h->lid, h->idiag, h->idiag32, h->Fu, h->Fv, h->Fw, h->b, h->r, h->d0, h->d1, h->q,
                    h->e, h->gs.u, h->gs.v, h->gs.w, h->gs.p, h->L.ctl, h->L.part, h->L.sync, h->L.params,
                    h->L.jump};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    void *aptrs[] = {h->adj_ck, h->adj_segu, h->adj_y, h->adj_lam, h->adj_mu, h->adj_p, h->adj_glid, h->adj_part,
                     h->adj_fin,
                     h->bv0, h->bv1, h->brh, h->pprev};
    for (void *p : aptrs)
        if (p) (void)hipFree(p);
    if (h->L.ctl_host) (void)hipHostFree(h->L.ctl_host);
    if (h->L.params_host) (void)hipHostFree(h->L.params_host);
    if (h->L.jump_host) (void)hipHostFree(h->L.jump_host);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    delete h;
    return NSP_OK;
}

nsp_status nsp_set_lid(nsp_handle *h, const double *lid_dev, void *stream) {
    if (!h || !lid_dev) return fail(h, NSP_ERR_ARG, "null lid pointer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    ++h->lid_version;  // a recorded run used the previous lid
    HIPCHK(h, hipMemcpyAsync(h->lid, lid_dev, (size_t)h->nz * (h->nx + 1) * sizeof(double), hipMemcpyDeviceToDevice,
                             s));
    HIPCHK(h, hipStreamSynchronize(s));
    return NSP_OK;
}

nsp_status nsp_poisson_solve(nsp_handle *h, const double *b, double *p, int batch, const nsp_poisson_opts *o,
                             void *stream, nsp_solve_info *info) {
    if (!h) return NSP_ERR_ARG;
    if (batch < 0 || batch > h->max_batch) return fail(h, NSP_ERR_ARG, "batch outside [0, max_batch]");
    if (!valid_opts(o)) return fail(h, NSP_ERR_ARG, "invalid Poisson options");
    if (batch == 0) return NSP_OK;  // nothing to solve; b and p may be null
    if (!b || !p) return fail(h, NSP_ERR_ARG, "null pointer");
    GroupDesc G;
    nsp_state y{nullptr, nullptr, nullptr, p};
    fill_group(G, h, y, 0, batch, 0, 0, b);
    nsp_handle *hs[1] = {h};
    return run(hs, 1, &G, MODE_POISSON, 0, 1.0, o, static_cast<hipStream_t>(stream), info, 0);
}

nsp_status nsp_fine_step(nsp_handle *h, nsp_state y, int batch, double t0, double t1, double dt,
                         const nsp_poisson_opts *o, void *stream, nsp_solve_info *info) {
    if (!h) return NSP_ERR_ARG;
    nsp_handle *hs[1] = {h};
    return propagate(hs, &y, &batch, 1, t0, t1, dt, o, stream, info);
}

nsp_status nsp_fine_step_graph_create(nsp_handle *h, nsp_state y, int batch, double t0, double t1, double dt,
                                      const nsp_poisson_opts *o, nsp_graph **out) {
    if (!h || !out) return fail(h, NSP_ERR_ARG, "null handle or output pointer");
    *out = nullptr;
    if (!valid_opts(o)) return fail(h, NSP_ERR_ARG, "invalid Poisson options");
    int nsteps = 0;
    if (!step_count(t0, t1, dt, &nsteps) || nsteps == 0)
        return fail(h, NSP_ERR_ARG, "(t1 - t0)/dt is not a positive integer");
    if (!state_ok(y) || batch < 1 || batch > h->max_batch) return fail(h, NSP_ERR_ARG, "bad state or batch");
    GroupDesc G;
    fill_group(G, h, y, 0, batch, 0, 0, nullptr, 0);
    G.upwind = 0;
    nsp_handle *hs[1] = {h};
    nsp_graph *g = new nsp_graph;
    g->h = h;
#define GCHK(call)                                                                                         \
    do {                                                                                                   \
        hipError_t e_ = (call);                                                                            \
        if (e_ != hipSuccess) {                                                                            \
            free_graph(g);                                                                                 \
            return fail(h, NSP_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));                \
        }                                                                                                  \
    } while (0)
    nsp_status st = plan_launch(hs, 1, &G, MODE_FINE, nsteps, dt, o, 0, false, g->pl);
    if (st != NSP_OK) {
        free_graph(g);
        return st;
    }
    const int nslices = g->pl.nslices;
    GCHK(dalloc(&g->L.params, 1));
    GCHK(dalloc(&g->L.ctl, nslices));
    GCHK(hipHostMalloc(reinterpret_cast<void **>(&g->L.ctl_host), nslices * sizeof(SliceCtl)));
    GCHK(dalloc(&g->L.part, (size_t)2 * kNQ * g->pl.pstride));
    GCHK(dalloc(&g->L.sync, 1));
    GCHK(dalloc(&g->fold, 1));
    GCHK(hipHostMalloc(reinterpret_cast<void **>(&g->fold_host), sizeof(GraphFold)));
    GCHK(hipEventCreate(&g->ev0));
    GCHK(hipEventCreate(&g->ev1));
    GCHK(launch_zero_words(g->fold, (long long)(sizeof(GraphFold) / sizeof(unsigned)), nullptr));
    KParams P = g->pl.P;
    P.ctl = g->L.ctl;
    P.part = g->L.part;
    P.sync = g->L.sync;
    GCHK(hipMemcpy(g->L.params, &P, sizeof(KParams), hipMemcpyHostToDevice));
    GCHK(hipDeviceSynchronize());
    GCHK(hipGraphCreate(&g->graph, 0));
    GCHK(add_persistent_graph_nodes(g->graph, g->L.params, g->pl.wg, P.rr != 0, g->L.ctl, nslices, g->L.sync,
                                    g->fold));
    GCHK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
#undef GCHK
    *out = g;
    return NSP_OK;
}

nsp_status nsp_graph_launch(nsp_graph *g, void *stream) {
    if (!g) return NSP_ERR_ARG;
    nsp_handle *h = g->h;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g->replays == 0) HIPCHK(h, hipEventRecord(g->ev0, s));
    HIPCHK(h, hipGraphLaunch(g->exec, s));
    HIPCHK(h, hipEventRecord(g->ev1, s));
    ++g->replays;
    return NSP_OK;
}

nsp_status nsp_graph_finish(nsp_graph *g, void *stream, nsp_solve_info *info) {
    if (!g) return NSP_ERR_ARG;
    nsp_handle *h = g->h;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, hipStreamSynchronize(s));
    const int n = g->replays;
    if (n == 0) return NSP_OK;
    const int nslices = g->pl.nslices;
    HIPCHK(h, hipMemcpy(g->L.ctl_host, g->L.ctl, nslices * sizeof(SliceCtl), hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(g->fold_host, g->fold, sizeof(GraphFold), hipMemcpyDeviceToHost));
    HIPCHK(h, launch_zero_words(g->fold, (long long)(sizeof(GraphFold) / sizeof(unsigned)), s));
    HIPCHK(h, hipStreamSynchronize(s));
    g->replays = 0;
    float ms = 0;
    if (hipEventElapsedTime(&ms, g->ev0, g->ev1) == hipSuccess) h->last_ms = ms;
    const GraphFold &F = *g->fold_host;
    if (F.abort) return fail(h, NSP_ERR_HIP, "grid barrier wait exceeded its limit; launch abandoned");
    // every replay's iterations and the worst status; the rest from the last
    int worst = 0;
    for (int k = 0; k < nslices; ++k) {
        SliceCtl &c = g->L.ctl_host[k];
        c.tot_it = (int)F.it[k];
        c.tot_outer = (int)F.outer[k];
        c.max_it = F.max_it[k];
        c.status = F.status[k];
        worst = std::max(worst, F.status[k]);
    }
    return collect_status(h, g->pl, g->L.ctl_host, ms, worst, info, n);
}

nsp_status nsp_graph_destroy(nsp_graph *g) {
    if (!g) return NSP_OK;
    (void)hipDeviceSynchronize();  // no replay may still use what is freed
    free_graph(g);
    return NSP_OK;
}

nsp_status nsp_coarse_step(nsp_handle *h, nsp_state y, int batch, double t0, double t1, double DT,
                           const nsp_poisson_opts *o, void *stream, nsp_solve_info *info) {
    if (!h) return NSP_ERR_ARG;
    nsp_handle *hs[1] = {h};
    return propagate(hs, &y, &batch, 1, t0, t1, DT, o, stream, info, true);
}

nsp_status nsp_set_coarse_convection(nsp_handle *h, nsp_convection scheme) {
    if (!h) return NSP_ERR_ARG;
    if (scheme != NSP_CONV_SMART && scheme != NSP_CONV_UPWIND) return fail(h, NSP_ERR_ARG, "unknown convection");
    h->coarse_upwind = scheme == NSP_CONV_UPWIND ? 1 : 0;
    return NSP_OK;
}

nsp_status nsp_group_fine_step(nsp_handle *const *hs, const nsp_state *ys, const int *batches, int ngroups, double t0,
                               double t1, double dt, const nsp_poisson_opts *o, void *stream, nsp_solve_info *info) {
    return propagate(hs, ys, batches, ngroups, t0, t1, dt, o, stream, info);
}

nsp_status nsp_group_parareal_start(nsp_handle *const *hs, const nsp_state *Y, const nsp_state *Gk, int ngroups,
                                    int nslices, double t0, double T, double DT, const nsp_poisson_opts *coarse,
                                    void *stream) {
    return parareal_start_impl(hs, nullptr, Y, Gk, ngroups, nslices, t0, T, DT, coarse, stream);
}

nsp_status nsp_parareal_start(nsp_handle *h, nsp_state Y, nsp_state Gk, int nslices, double t0, double T, double DT,
                              const nsp_poisson_opts *coarse, void *stream) {
    nsp_handle *hs[1] = {h};
    return parareal_start_impl(hs, nullptr, &Y, &Gk, 1, nslices, t0, T, DT, coarse, stream);
}

nsp_status nsp_group_parareal_iterate(nsp_handle *const *hs, const nsp_state *Y, const nsp_state *Fk,
                                      const nsp_state *Gk, int ngroups, int nslices, int k, double t0, double T,
                                      double dt, double DT, const nsp_poisson_opts *fine,
                                      const nsp_poisson_opts *coarse, void *stream, double *jump) {
    return parareal_iterate_impl(hs, nullptr, Y, Fk, Gk, ngroups, nslices, k, t0, T, dt, DT, fine, coarse, stream,
                                 jump);
}

nsp_status nsp_parareal_iterate(nsp_handle *h, nsp_state Y, nsp_state Fk, nsp_state Gk, int nslices, int k,
                                double t0, double T, double dt, double DT, const nsp_poisson_opts *fine,
                                const nsp_poisson_opts *coarse, void *stream, double *jump) {
    nsp_handle *hs[1] = {h};
    return parareal_iterate_impl(hs, nullptr, &Y, &Fk, &Gk, 1, nslices, k, t0, T, dt, DT, fine, coarse, stream, jump);
}

nsp_status nsp_restrict(nsp_handle *h, nsp_handle *hc, nsp_state yf, nsp_state yc, int batch, void *stream) {
    nsp_status st = check_pair(h, hc);
    if (st != NSP_OK) return st;
    if (!state_ok(yf) || !state_ok(yc) || batch < 0) return fail(h, NSP_ERR_ARG, "null state or negative batch");
    HIPCHK(h, transfer(h, yf, yc, batch, false, static_cast<hipStream_t>(stream)));
    return NSP_OK;
}

nsp_status nsp_prolong(nsp_handle *h, nsp_handle *hc, nsp_state yc, nsp_state yf, int batch, void *stream) {
    nsp_status st = check_pair(h, hc);
    if (st != NSP_OK) return st;
    if (!state_ok(yf) || !state_ok(yc) || batch < 0) return fail(h, NSP_ERR_ARG, "null state or negative batch");
    HIPCHK(h, transfer(h, yc, yf, batch, true, static_cast<hipStream_t>(stream)));
    return NSP_OK;
}

nsp_status nsp_parareal_start_cgrid(nsp_handle *h, nsp_handle *hc, nsp_state Y, nsp_state Gk, int nslices, double t0,
                                    double T, double DT, const nsp_poisson_opts *coarse, void *stream) {
    nsp_status st = check_pair(h, hc);
    if (st != NSP_OK) return st;
    nsp_handle *hs[1] = {h}, *hcs[1] = {hc};
    return parareal_start_impl(hs, hcs, &Y, &Gk, 1, nslices, t0, T, DT, coarse, stream);
}

nsp_status nsp_parareal_iterate_cgrid(nsp_handle *h, nsp_handle *hc, nsp_state Y, nsp_state Fk, nsp_state Gk,
                                      int nslices, int k, double t0, double T, double dt, double DT,
                                      const nsp_poisson_opts *fine, const nsp_poisson_opts *coarse, void *stream,
                                      double *jump) {
    nsp_status st = check_pair(h, hc);
    if (st != NSP_OK) return st;
    nsp_handle *hs[1] = {h}, *hcs[1] = {hc};
    return parareal_iterate_impl(hs, hcs, &Y, &Fk, &Gk, 1, nslices, k, t0, T, dt, DT, fine, coarse, stream, jump);
}

}  // extern "C"

namespace {

long long state_len(const nsp_handle *h) { return h->nu + h->nv + h->nw + h->ncells; }

// a state stored contiguously: u, v, w, p back to back
nsp_state packed_state(const nsp_handle *h, double *base) {
    nsp_state s;
    s.u = base;
    s.v = base + h->nu;
    s.w = base + h->nu + h->nv;
    s.p = base + h->nu + h->nv + h->nw;
    return s;
}

AdjParams adj_params(const nsp_handle *h, double dt) {
    AdjParams A;
    A.nx = h->nx;
    A.ny = h->ny;
    A.nz = h->nz;
    const double L[3] = {h->lx, h->ly, h->lz};
    const int n[3] = {h->nx, h->ny, h->nz};
    for (int d = 0; d < 3; ++d) {
        A.L[d] = L[d];
        A.h[d] = L[d] / n[d];
        A.ih[d] = 1.0 / A.h[d];
        A.ih2[d] = 1.0 / (A.h[d] * A.h[d]);
    }
    A.inv_re = 1.0 / h->re;
    A.dt = dt;
    A.flags = h->flags;
    A.lid = h->lid;
    return A;
}

// the momentum adjoint kernel indexes faces in 32 bits
bool adj_size_ok(const nsp_handle *h) {
    return (long long)(h->nx + 1) * (h->ny + 1) * (h->nz + 1) < (1LL << 31);
}

// Each buffer is allocated on its own test, so a call after a failed
// allocation retries what is missing instead of running with a null buffer;
// a checkpoint store is counted only once it exists.
nsp_status ensure_adj(nsp_handle *h, int nck, int seg) {
    const long long L = state_len(h);
    const long long F3 = h->nu + h->nv + h->nw;
    if (!h->adj_y) HIPCHK(h, dalloc(&h->adj_y, L));
    if (!h->adj_lam) HIPCHK(h, dalloc(&h->adj_lam, F3));
    if (!h->adj_mu) HIPCHK(h, dalloc(&h->adj_mu, F3));
    if (!h->adj_p) HIPCHK(h, dalloc(&h->adj_p, h->ncells));
    if (!h->adj_glid) HIPCHK(h, dalloc(&h->adj_glid, (size_t)h->nz * (h->nx + 1)));
    if (!h->adj_part) HIPCHK(h, dalloc(&h->adj_part, 3 * kSumBlocks + 1));
    if (!h->adj_fin) HIPCHK(h, dalloc(&h->adj_fin, F3));
    if (nck > h->adj_nck) {
        if (h->adj_ck) (void)hipFree(h->adj_ck);
        h->adj_ck = nullptr;
        h->adj_nck = 0;
        HIPCHK(h, dalloc(&h->adj_ck, (size_t)nck * L));
        h->adj_nck = nck;
    }
    if (seg > h->adj_seg) {
        if (h->adj_segu) (void)hipFree(h->adj_segu);
        h->adj_segu = nullptr;
        h->adj_seg = 0;
        HIPCHK(h, dalloc(&h->adj_segu, (size_t)seg * F3));
        h->adj_seg = seg;
    }
    return NSP_OK;
}

}  // namespace

extern "C" {

nsp_status nsp_fine_solve_record(nsp_handle *h, nsp_state y0, int nsteps, double dt, int ckpt_every,
                                 const nsp_poisson_opts *o, double *J, unsigned long long *tape, void *stream) {
    if (!h) return NSP_ERR_ARG;
    if (h->pz) return fail(h, NSP_ERR_UNSUPPORTED, "the adjoint is implemented for walls in z only");
    if (h->slip) return fail(h, NSP_ERR_UNSUPPORTED, "the adjoint is implemented for no-slip obstacles only");
    if (!adj_size_ok(h)) return fail(h, NSP_ERR_UNSUPPORTED, "the adjoint takes grids of fewer than 2^31 faces");
    if (!state_ok(y0) || nsteps < 0 || !(dt > 0) || !J) return fail(h, NSP_ERR_ARG, "bad adjoint arguments");
    if (!valid_opts(o)) return fail(h, NSP_ERR_ARG, "invalid Poisson options");
    const bool keep = tape != nullptr;
    if (keep) *tape = 0;
    h->tape = 0;  // the workspace is about to be overwritten
    // the reverse sweep recomputes steps one call at a time, where no
    // extrapolation happens: the record must take the same plain warm start
    nsp_poisson_opts of = *o;
    of.extrapolate = 0;
    o = &of;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int ck = ckpt_every > 0 ? std::min(ckpt_every, std::max(nsteps, 1)) : std::max(nsteps, 1);
    const int nseg = nsteps > 0 ? (nsteps + ck - 1) / ck : 0;
    nsp_status st = ensure_adj(h, keep ? nseg : 0, keep ? ck : 0);
    if (st != NSP_OK) return st;
    const long long L = state_len(h);
    nsp_state y = packed_state(h, h->adj_y);
    HIPCHK(h, copy_slices(h, y, y0, 1, s));
    nsp_handle *hs[1] = {h};
    int one = 1;
    // forward sweep, storing the state at the start of every segment
    for (int sg = 0; sg < nseg; ++sg) {
        if (keep) HIPCHK(h, launch_copy_state(h->adj_ck + (long long)sg * L, h->adj_y, L, s));
        const int len = std::min(ck, nsteps - sg * ck);
        st = propagate(hs, &y, &one, 1, 0.0, len * dt, dt, o, stream, nullptr);
        if (st != NSP_OK) return st;
    }
    const AdjParams A = adj_params(h, dt);
    const double *vel[3] = {y.u, y.v, y.w};
    HIPCHK(h, launch_sumsq_open(A, vel, h->adj_part, h->adj_part + 3 * kSumBlocks, s));
    double ss = 0.0;
    HIPCHK(h, hipMemcpyAsync(&ss, h->adj_part + 3 * kSumBlocks, sizeof(double), hipMemcpyDeviceToHost, s));
    const double vol = A.h[0] * A.h[1] * A.h[2];
    if (keep) {
        // dJ/du_T = vol * u_T on open faces, the reverse sweep's start
        double *fin[3] = {h->adj_fin, h->adj_fin + h->nu, h->adj_fin + h->nu + h->nv};
        HIPCHK(h, launch_scale_open(A, vel, vol, fin, s));
    }
    HIPCHK(h, hipStreamSynchronize(s));
    *J = 0.5 * vol * ss;
    if (keep) {
        h->tape = *tape = ++h->tape_seq;
        h->tape_lid_version = h->lid_version;
        h->tape_nsteps = nsteps;
        h->tape_ck = ck;
        h->tape_nseg = nseg;
        h->tape_dt = dt;
        h->tape_opts = *o;
    }
    return NSP_OK;
}

int nsp_fine_solve_tape_valid(const nsp_handle *h, unsigned long long tape) {
    return h && tape != 0 && tape == h->tape && h->tape_lid_version == h->lid_version ? 1 : 0;
}

nsp_status nsp_fine_solve_reverse(nsp_handle *h, unsigned long long tape, nsp_state grad, double *g_lid,
                                  void *stream) {
    if (!h) return NSP_ERR_ARG;
    if (!(grad.u && grad.v && grad.w)) return fail(h, NSP_ERR_ARG, "null gradient arrays");
    if (!nsp_fine_solve_tape_valid(h, tape))
        return fail(h, NSP_ERR_ARG, "stale tape: another run was recorded or the lid changed since");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long long L = state_len(h);
    const long long F3 = h->nu + h->nv + h->nw;
    const int nsteps = h->tape_nsteps, ck = h->tape_ck, nseg = h->tape_nseg;
    const double dt = h->tape_dt;
    const nsp_poisson_opts o = h->tape_opts;
    nsp_state y = packed_state(h, h->adj_y);
    nsp_handle *hs[1] = {h};
    int one = 1;
    nsp_status st;
    const AdjParams A = adj_params(h, dt);
    double *lam[3] = {h->adj_lam, h->adj_lam + h->nu, h->adj_lam + h->nu + h->nv};
    double *mu[3] = {h->adj_mu, h->adj_mu + h->nu, h->adj_mu + h->nu + h->nv};
    HIPCHK(h, launch_copy_state(h->adj_lam, h->adj_fin, F3, s));
    HIPCHK(h, launch_zero_words(h->adj_glid, 2LL * h->nz * (h->nx + 1), s));
    HIPCHK(h, launch_zero_words(h->adj_p, 2LL * h->ncells, s));
    nsp_poisson_opts po = o;
    po.prec = NSP_FP64;  // the adjoint differentiates the exact projection
    for (int sg = nseg - 1; sg >= 0; --sg) {
        const int len = std::min(ck, nsteps - sg * ck);
        // recompute the segment, keeping the velocity at the start of each step
        HIPCHK(h, launch_copy_state(h->adj_y, h->adj_ck + (long long)sg * L, L, s));
        for (int m = 0; m < len; ++m) {
            HIPCHK(h, launch_copy_state(h->adj_segu + (long long)m * F3, h->adj_y, F3, s));
            if (m + 1 < len) {
                st = propagate(hs, &y, &one, 1, 0.0, dt, dt, &o, stream, nullptr);
                if (st != NSP_OK) return st;
            }
        }
        for (int m = len - 1; m >= 0; --m) {
            // mu = P lam: the projection of the step applied to lam
            HIPCHK(h, launch_copy_state(h->Fu, lam[0], h->nu, s));
            HIPCHK(h, launch_copy_state(h->Fv, lam[1], h->nv, s));
            HIPCHK(h, launch_copy_state(h->Fw, lam[2], h->nw, s));
            GroupDesc G;
            nsp_state muv{mu[0], mu[1], mu[2], h->adj_p};
            fill_group(G, h, muv, 0, 1, 0, 0, nullptr);
            st = run(hs, 1, &G, MODE_PROJECT, 0, 1.0, &po, s, nullptr, 0);
            if (st != NSP_OK) return st;
            // lam = mu + dt (dR/du)^T mu at the state of step m; lid adjoint
            const double *um = h->adj_segu + (long long)m * F3;
            const double *velm[3] = {um, um + h->nu, um + h->nu + h->nv};
            const double *muc[3] = {mu[0], mu[1], mu[2]};
            HIPCHK(h, launch_momentum_adjoint(A, velm, muc, lam, h->adj_glid, s));
        }
    }
    HIPCHK(h, launch_copy_state(grad.u, lam[0], h->nu, s));
    HIPCHK(h, launch_copy_state(grad.v, lam[1], h->nv, s));
    HIPCHK(h, launch_copy_state(grad.w, lam[2], h->nw, s));
    if (g_lid) HIPCHK(h, launch_copy_state(g_lid, h->adj_glid, (long long)h->nz * (h->nx + 1), s));
    HIPCHK(h, hipStreamSynchronize(s));
    return NSP_OK;
}

nsp_status nsp_momentum_adjoint(nsp_handle *h, nsp_state vel, nsp_state mu, nsp_state lam, double *g_lid, double dt,
                                void *stream) {
    if (!h) return NSP_ERR_ARG;
    if (!adj_size_ok(h)) return fail(h, NSP_ERR_UNSUPPORTED, "the adjoint takes grids of fewer than 2^31 faces");
    if (h->pz) return fail(h, NSP_ERR_UNSUPPORTED, "the adjoint is implemented for walls in z only");
    if (h->slip) return fail(h, NSP_ERR_UNSUPPORTED, "the adjoint is implemented for no-slip obstacles only");
    if (!(vel.u && vel.v && vel.w && mu.u && mu.v && mu.w && lam.u && lam.v && lam.w) || !(dt > 0))
        return fail(h, NSP_ERR_ARG, "bad momentum-adjoint arguments");
    const double *vp[3] = {vel.u, vel.v, vel.w}, *mp[3] = {mu.u, mu.v, mu.w};
    double *lp[3] = {lam.u, lam.v, lam.w};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (lp[a] == mp[b] || lp[a] == vp[b]) return fail(h, NSP_ERR_ARG, "lam must not alias vel or mu");
    HIPCHK(h, launch_momentum_adjoint(adj_params(h, dt), vp, mp, lp, g_lid, static_cast<hipStream_t>(stream)));
    return NSP_OK;
}

nsp_status nsp_fine_solve_adjoint(nsp_handle *h, nsp_state y0, int nsteps, double dt, int ckpt_every,
                                  const nsp_poisson_opts *o, nsp_state grad, double *g_lid, double *J, void *stream) {
    if (!h) return NSP_ERR_ARG;
    const bool want_grad = grad.u && grad.v && grad.w;
    unsigned long long tape = 0;
    nsp_status st = nsp_fine_solve_record(h, y0, nsteps, dt, ckpt_every, o, J, want_grad ? &tape : nullptr, stream);
    if (st != NSP_OK || !want_grad) return st;
    return nsp_fine_solve_reverse(h, tape, grad, g_lid, stream);
}

nsp_status nsp_lid_from_modes(nsp_handle *h, const double *coef, int nmodes, double *lid_dev, void *stream) {
    if (!h) return NSP_ERR_ARG;
    if (!coef || !lid_dev || nmodes < 0 || nmodes > 64) return fail(h, NSP_ERR_ARG, "bad lid-mode arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, launch_lid_synth(adj_params(h, 1.0), coef, nmodes, lid_dev, s));
    HIPCHK(h, hipStreamSynchronize(s));
    return NSP_OK;
}

nsp_status nsp_lid_modes_grad(nsp_handle *h, const double *g_lid, int nmodes, double *g_coef, void *stream) {
    if (!h) return NSP_ERR_ARG;
    if (!g_lid || !g_coef || nmodes < 1 || nmodes > 64) return fail(h, NSP_ERR_ARG, "bad lid-mode arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, launch_lid_project(adj_params(h, 1.0), g_lid, nmodes, g_coef, s));
    HIPCHK(h, hipStreamSynchronize(s));
    return NSP_OK;
}

nsp_status nsp_launch_stats_get(nsp_handle *h, nsp_launch_stats out[3], int reset) {
    if (!h) return NSP_ERR_ARG;
    for (int m = 0; m < 3; ++m) {
        if (out) out[m] = h->stats[m];
        if (reset) h->stats[m] = nsp_launch_stats{};
    }
    return NSP_OK;
}

nsp_status nsp_set_launch(nsp_handle *h, int workgroups) {
    if (!h || workgroups < 0) return fail(h, NSP_ERR_ARG, "bad workgroup count");
    h->fixed_wg = workgroups;
    return NSP_OK;
}

nsp_status nsp_last_launch_ms(const nsp_handle *h, double *ms) {
    if (!h || !ms) return NSP_ERR_ARG;
    *ms = h->last_ms;
    return NSP_OK;
}

nsp_status nsp_autotune(nsp_handle *h, int batch, nsp_precision prec, void *stream, int *chosen,
                        int *chosen_planes, int *chosen_items) {
    if (!h || batch < 1 || batch > h->max_batch) return fail(h, NSP_ERR_ARG, "bad autotune batch");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // synthetic right-hand side (made mean-free inside the solve); every
    // candidate shape runs the same 40 CG iterations from p = 0
    std::vector<double> hb((size_t)h->ncells);
    for (long long c = 0; c < h->ncells; ++c) hb[c] = std::sin(0.37 * (double)c) + std::cos(0.011 * (double)c);
    struct TrialBuffers {  // freed on every return path
        double *b = nullptr, *p = nullptr;
        ~TrialBuffers() {
            (void)hipFree(b);
            (void)hipFree(p);
        }
    } tb;
    HIPCHK(h, dalloc(&tb.b, (size_t)batch * h->ncells));
    HIPCHK(h, dalloc(&tb.p, (size_t)batch * h->ncells));
    double *const b = tb.b, *const p = tb.p;
    for (int i = 0; i < batch; ++i)
        HIPCHK(h, hipMemcpy(b + (long long)i * h->ncells, hb.data(), h->ncells * sizeof(double), hipMemcpyHostToDevice));
    nsp_poisson_opts o{0.0, 40, prec, 1e-30, 1};
    const int ntiles = batch * std::max(h->ntiles, h->cgtiles);
    std::vector<int> cands;
    for (int c : {h->max_wg, h->max_wg * 3 / 4, h->max_wg / 2, h->max_wg / 4, 512, 256, 128})
        if (c >= 1 && c <= std::min(h->max_wg, ntiles) &&
            std::find(cands.begin(), cands.end(), c) == cands.end())
            cands.push_back(c);
    if (cands.empty()) cands.push_back(std::min(h->max_wg, ntiles));
    GroupDesc G;
    nsp_state y{nullptr, nullptr, nullptr, p};
    fill_group(G, h, y, 0, batch, 0, 0, b);
    nsp_handle *hs[1] = {h};
    // column-tile depths in planes (from the grid's zsub up to 32); flat tiles have none
    std::vector<int> depths = {1}, itemss = {1};
    if (h->crb > 0) depths = h->zsh == 2 ? std::vector<int>{4, 8, 16, 32} : std::vector<int>{8, 16, 32};
    if (h->crb > 0 && prec != NSP_FP64 && h->cnb >= 2) itemss = {1, 2};
    nsp_launch_stats keep_stats[3];
    for (int m = 0; m < 3; ++m) keep_stats[m] = h->stats[m];  // the trial launches are not counted
    int best = cands[0], best_depth = depths[0], best_items = itemss[0];
    double best_ms = 1e30;
    for (int ni : itemss)
    for (int dep : depths)
        for (int c : cands) {
            double tot = 0;
            h->force_depth = dep;
            h->force_items = ni;
            for (int rep = 0; rep < 3; ++rep) {
                nsp_status st = NSP_OK;
                if (hipMemsetAsync(p, 0, (size_t)batch * h->ncells * sizeof(double), s) != hipSuccess)
                    st = fail(h, NSP_ERR_HIP, "autotune: memset failed");
                if (st == NSP_OK) st = run(hs, 1, &G, MODE_POISSON, 0, 1.0, &o, s, nullptr, c);
                if (st != NSP_OK && st != NSP_ERR_NOT_CONVERGED) {
                    h->force_depth = h->force_items = 0;
                    for (int m = 0; m < 3; ++m) h->stats[m] = keep_stats[m];
                    return st;
                }
                if (rep > 0) tot += h->last_ms;
            }
            if (tot < best_ms) { best_ms = tot; best = c; best_depth = dep; best_items = ni; }
        }
    h->force_depth = h->force_items = 0;
    for (int m = 0; m < 3; ++m) h->stats[m] = keep_stats[m];
    const int pr = prec != NSP_FP64 ? 1 : 0;
    const int keep_depth = h->crb > 0 ? best_depth : 0, keep_items = h->crb > 0 ? best_items : 0;
    bool found = false;
    for (TuneEntry &t : h->tuned)
        if (t.batch == batch && t.prec == pr) {
            t.workgroups = best;
            t.depth = keep_depth;
            t.items = keep_items;
            found = true;
        }
    if (!found) h->tuned.push_back(TuneEntry{batch, pr, best, keep_depth, keep_items});
    if (chosen) *chosen = best;
    if (chosen_planes) *chosen_planes = keep_depth;
    if (chosen_items) *chosen_items = keep_items;
    return NSP_OK;
}

}  // extern "C"

// ------------------------------------------------ allocation-free Poisson solve

namespace {

// Workspace of nsp_poisson_solve_noalloc: one file-scope device array, which
// every GPU the library runs on holds until the process ends.  Host code
// never uses the array's name as an address: the address on each device
// comes from hipGetSymbolAddress, taken once per device with that device
// current, and only that address is passed to kernels and copies.
constexpr size_t kScratchBytes = size_t(96) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_at[kMaxScratchDevices];  // scratch's address on each device (null: not yet taken)

nsp_status scratch_address(nsp_handle *h, unsigned char **out) {
    int dev = -1;
    HIPCHK(h, hipGetDevice(&dev));
    if (dev != h->device) return fail(h, NSP_ERR_ARG, "the current device is not the handle's device");
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(h, NSP_ERR_UNSUPPORTED, "device ordinal above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_at[dev]) {
        void *ptr = nullptr;
        HIPCHK(h, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(h, NSP_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_at[dev] = static_cast<unsigned char *>(ptr);
    }
    *out = g_scratch_at[dev];
    return NSP_OK;
}

// Hands out 256-byte-aligned pieces of [base, base + cap); `used` may exceed
// cap, which the caller checks before any piece is used.
struct Carve {
    unsigned char *base;
    size_t used = 0;
    template <class T>
    T *take(size_t n) {
        used = (used + 255) & ~size_t(255);
        T *p = reinterpret_cast<T *>(base + used);
        used += n * sizeof(T);
        return p;
    }
};

}  // namespace

extern "C" nsp_status nsp_poisson_solve_noalloc(nsp_handle *h, const double *b, double *p, int batch,
                                                const nsp_poisson_opts *o, void *stream, nsp_solve_info *info) {
    if (!h) return NSP_ERR_ARG;
    if (batch < 0 || batch > h->max_batch) return fail(h, NSP_ERR_ARG, "batch outside [0, max_batch]");
    if (!valid_opts(o)) return fail(h, NSP_ERR_ARG, "invalid Poisson options");
    if (batch == 0) return NSP_OK;
    if (!b || !p) return fail(h, NSP_ERR_ARG, "null pointer");
    if (o->solver != NSP_PCG && o->prec != NSP_FP64)
        return fail(h, NSP_ERR_UNSUPPORTED, "BiCGStab and single-reduction PCG run in FP64 only");
    if (batch > h->L.cap_slices) return fail(h, NSP_ERR_ARG, "batch above the handle's control-block capacity");
    unsigned char *base = nullptr;
    nsp_status st = scratch_address(h, &base);
    if (st != NSP_OK) return st;
    const size_t cells = (size_t)batch * (size_t)h->ncells;
    const int pstride = batch * std::max(h->ntiles, h->cgparts);
    Carve c{base};
    LaunchRes ws;
    ws.params = c.take<KParams>(1);
    ws.sync = c.take<SyncWords>(1);
    ws.ctl = c.take<SliceCtl>(batch);
    ws.part = c.take<double>((size_t)2 * kNQ * pstride);
    ws.params_host = h->L.params_host;
    ws.ctl_host = h->L.ctl_host;
    ws.cap_slices = batch;
    ws.cap_tiles = pstride;
    GroupDesc G;
    nsp_state y{nullptr, nullptr, nullptr, p};
    fill_group(G, h, y, 0, batch, 0, 0, b);
    G.b = c.take<double>(cells);
    G.r = c.take<double>(cells);
    G.d0 = c.take<double>(cells);
    G.d1 = c.take<double>(cells);
    G.e = c.take<float>(cells);
    G.q = c.take<double>(cells);
    G.bv0 = G.bv1 = G.brh = nullptr;
    if (o->solver != NSP_PCG) {
        G.bv0 = c.take<double>(cells);
        G.bv1 = c.take<double>(cells);
        G.brh = c.take<double>(cells);
    }
    if (c.used > kScratchBytes)
        return fail(h, NSP_ERR_ARG,
                    "the solve needs " + std::to_string(c.used) + " bytes of workspace, above the " +
                        std::to_string(kScratchBytes) + " bytes of the allocation-free solve");
    nsp_handle *hs[1] = {h};
    return run(hs, 1, &G, MODE_POISSON, 0, 1.0, o, static_cast<hipStream_t>(stream), info, 0, &ws);
}
