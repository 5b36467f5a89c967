// Internal data structures shared by the host side and the gfx950 kernels
// of libnsp.  Not part of the public C ABI (include/nsp.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace nsp {

constexpr int kBlock = 1024;     // threads per workgroup (16 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kMaxGroups = 4;    // grids per launch (uneven batch)
constexpr int kMaxSlices = 64;   // slices per launch
constexpr int kNQ = 4;           // partial sums per tile

// Per-cell flag byte: which of the six faces of the pressure cell are open,
// whether the cell is fluid, and whether the momentum stencil of the cell's
// low faces may touch a wall, an obstacle or the domain boundary (then the
// image-rule path is taken; otherwise every stencil point is an open face).
enum : uint8_t {
    FL_XM = 1, FL_XP = 2, FL_YM = 4, FL_YP = 8, FL_ZM = 16, FL_ZP = 32,
    FL_OPEN = 63, FL_FLUID = 64, FL_SLOW = 128
};

constexpr int kMaxBlk = 8;       // zsub-plane partial blocks per column tile (32 planes / 4)

// One grid and the batch of slices it carries in a launch.
struct GroupDesc {
    int nx, ny, nz;
    int ncells;            // nx*ny*nz
    int nu, nv, nw;        // faces per slice of u, v, w
    int tile;              // cells per tile (multiple of kBlock)
    int ntiles;            // tiles per slice
    int nslices;           // slices of this grid in the launch
    int slice0;            // first slice index of this grid in the launch
    int tile0;             // first tile index of this grid in the launch
    // CG tiles (phases of the CG loop).  Column tiles: full x rows, cby rows
    // in y, cbz planes in z (a multiple of zsub, chosen per launch); each
    // thread walks z carrying cni items (rows yy and yy + crb; cni = 2 only
    // in FP32 launches), so cby = cni * crb.  Partial sums are kept per crb
    // rows and zsub planes whatever cbz and cni are, so results depend on
    // neither.  cby == 0: the CG loop uses the flat tiles above (one partial
    // per tile).
    int cby, cbz;          // rows / planes per column tile
    int cny, cnz;          // column tiles along y / z
    int crb, cni, cnb;     // rows per partial block, items per thread, row blocks along y
    int zsh;               // log2 of zsub, the planes per partial block (8, or 4 on grids whose
                           // slice alone has fewer 8-plane column tiles than workgroups); fixed per grid
    int cgtiles;           // CG tiles per slice
    int cgtile0;           // first CG tile index of this grid in the launch
    int cgparts;           // CG partial sums per slice
    int cgpart0;           // first CG partial index of this grid in the launch
    double nfluid;         // number of fluid cells
    int pz;                // periodic in z: cell k = 0 neighbours k = nz - 1; the w plane at
                           // z = Lz repeats z = 0 (written equal)
    int slip;              // free-slip obstacle walls (domain walls stay no-slip)
    int upwind;            // donor-cell convective face values instead of SMART (coarse propagator)
    double ih[3], ih2[3];  // 1/h, 1/h^2 per direction
    float ih2f[3];
    double inv_re;
    const uint8_t *flags;  // [ncells]
    const double *lid;     // [nz][nx+1]
    const double *idiag;   // [64]: 1/diag(A) per open-face pattern
    const float *idiag32;  // [64]
    double *u, *v, *w, *p;         // state, slice 0 (slice stride nu/nv/nw/ncells)
    double *Fu, *Fv, *Fw, *b;      // predictor and right-hand side workspace
    double *r, *d0, *d1, *q;       // CG vectors (FP32 view in mixed mode); BiCGStab: p in d0/d1, t in q;
                                   // single-reduction CG: s in d0/d1, p in q
    double *bv0, *bv1, *brh;       // BiCGStab: v (two buffers) and the shadow residual; single-reduction
                                   // CG: w (two buffers) and the second residual buffer
    float *e;                      // FP32 defect correction
    const double *bin;             // Poisson mode: caller's right-hand side
    double *pprev;                 // KParams::extrap: the previous step's pressure per slice (slice stride ncells)
};

// Per-slice solver state, written by the reducing workgroup at barriers and
// read by every workgroup after them.
struct SliceCtl {
    double bnorm, rz, alpha, beta, r0, mean_b, mean_r, mean_p, rel_true, res_true;
    double omega;  // BiCGStab (rz holds rho = <r^, r>)
    int active;   // CG iterating
    int first;    // next search direction is the preconditioned residual
    int it;       // CG iterations of the current step
    int it_in;    // iterations of the current inner (FP32) solve
    int need;     // mixed: another defect-correction sweep is needed
    int zero;     // right-hand side is zero: solution is p = 0
    int cold;     // the warm start was worse than none: the solve restarts from p = 0
    int fresh;    // reliable update: the FP32 residual was just replaced (until the next phase A)
    int outer;    // restarts / sweeps of the current step
    int done;     // current solve finished for this slice
    int status;   // worst status over the call
    int step_status; // status of the current solve
    int tot_it, max_it, tot_outer;
};

// Grid-barrier words.  A barrier combines arrivals per XCD: every workgroup
// waits until its stores are acknowledged by its XCD's L2, then increments
// that XCD's counter with an L2 atomic; the XCD's last arriver writes the
// whole L2 back once (one release for all its workgroups, instead of one L2
// write-back per workgroup, which serialise per XCD) and stores the barrier
// epoch into the XCD's arrival word; every workgroup polls the eight arrival
// words.  Start-up uses a plain barrier over per-workgroup words, which also
// records each workgroup's XCD.
constexpr int kMaxWG = 2048;  // workgroups per launch
constexpr int kMaxXcd = 16;   // XCC_ID values
struct SyncWords {
    unsigned arrive[kMaxWG];        // start-up barrier, one word per workgroup
    unsigned xof[kMaxWG];           // XCD of each workgroup
    unsigned xarr[kMaxXcd];         // per-XCD arrival epochs (device scope)
    unsigned pad0[64 - kMaxXcd];
    unsigned xcnt[kMaxXcd * 64];    // per-XCD counters, 256 bytes apart; each is
                                    // only ever touched through its XCD's L2
    int abort;                      // set when a barrier wait exceeds its spin limit
    int pad[63];
};

// MODE_FINE: nsteps projection steps on the state; MODE_POISSON: solve
// A p = bin; MODE_PROJECT: state velocities = P(F workspace), the step's
// projection applied to a given face field (dt = 1), p the warm start.
enum Mode : int { MODE_FINE = 0, MODE_POISSON = 1, MODE_PROJECT = 2 };

struct KParams {
    GroupDesc g[kMaxGroups];
    int ngroups;
    int nslices;           // total slices in the launch
    int ntiles;            // total tiles in the launch
    int cgtiles;           // total CG tiles in the launch
    int pstride;           // max(flat tiles, CG partials): stride of the partial-sum rows
    int mode;
    int nsteps;
    int prec;              // 0 fp64, 1 mixed (restarted FP32 solves), 2 mixed with reliable updates
    int maxit, max_outer;
    int xcd_remap;         // contiguous tile ranges per XCD
    int solver;            // 0: Jacobi-PCG, 1: Jacobi-BiCGStab (FP64), 2: single-reduction Jacobi-PCG (FP64)
    int wt;                // CG outputs by write-through (device-scope) stores
    int rr;                // CG vectors held in registers: every group has column tiles of 4 or 8
                           // planes (one partial block deep, nz a multiple), one item per thread, and
                           // the launch has no more CG tiles than workgroups
    int extrap;            // MODE_FINE: warm start 2 p^s - p^(s-1) from the second step on (GroupDesc::pprev)
    double dt;
    double rtol, eta;
    SliceCtl *ctl;         // [nslices]
    double *part;          // [2][kNQ][pstride]: double-buffered by barrier parity
    SyncWords *sync;
};

// Launchers implemented in nsp_kernels.hip.
// P_dev: device copy of the parameters, valid until the launch completes
// rr: the instantiation that keeps the CG vectors in registers (KParams::rr)
hipError_t launch_persistent(const KParams *P_dev, int workgroups, bool rr, hipStream_t stream);
hipError_t max_coresident_workgroups(int device, int *out);
hipError_t launch_reset_sync(SyncWords *s, hipStream_t stream);
// zero nwords 32-bit words at p on the stream (a kernel, not a memset)
hipError_t launch_zero_words(void *p, long long nwords, hipStream_t stream);
// What a replayed graph keeps across its replays (cleared by the host):
// per slice the worst status, the most CG iterations of one step, and the
// sums of CG iterations and sweeps; whether a barrier wait was abandoned.
struct GraphFold {
    int status[kMaxSlices];
    int max_it[kMaxSlices];
    long long it[kMaxSlices];
    long long outer[kMaxSlices];
    int abort;
    int pad;
};
// Adds to `graph` the kernel nodes of one persistent launch: zero the
// control blocks, reset the barrier words, the persistent kernel (a
// cooperative node) and a fold of the slices' results and the abort flag
// into *fold, which the graph never clears.
hipError_t add_persistent_graph_nodes(hipGraph_t graph, const KParams *P_dev, int workgroups, bool rr,
                                      SliceCtl *ctl, int nslices, SyncWords *sync, GraphFold *fold);

struct UpdateSeg {
    double *y;          // slice-end state to overwrite (y^{k+1}_{n+1})
    const double *f;    // F(y^k_n)
    const double *g;    // G(y^{k+1}_n)
    double *gold;       // G(y^k_n), replaced by g
    long long n;        // elements
    int jslot;          // 0: velocity jump, 1: pressure jump
};
constexpr int kMaxSegs = 4 * kMaxGroups;
struct UpdateParams {
    UpdateSeg seg[kMaxSegs];
    int nseg;
    unsigned long long *jump;  // [2 * kMaxGroups] bit patterns of the max |y_new - y_old|
    int group_of_seg[kMaxSegs];
};
hipError_t launch_parareal_update(const UpdateParams &U, hipStream_t stream);

// Grid transfers between a fine grid and one with half its cells in every
// direction (nx, ny, nz of the fine grid, all even).  Component c = 0..3 is
// u, v, w, p; src/dst hold `batch` slices back to back.
struct TransferParams {
    int prolong;                    // 0: restrict fine -> coarse; 1: prolong coarse -> fine
    int nx, ny, nz;                 // fine grid
    int batch;
    const double *src[4];
    double *dst[4];
};
hipError_t launch_transfer(const TransferParams &T, hipStream_t stream);
hipError_t launch_copy_state(double *dst, const double *src, long long n, hipStream_t stream);

// Adjoint of the fine step (nsp_adjoint.hip).
struct AdjParams {
    int nx, ny, nz;
    double h[3], L[3], ih[3], ih2[3];
    double inv_re, dt;
    const uint8_t *flags;
    const double *lid;
};
constexpr int kSumBlocks = 256;
hipError_t launch_momentum_adjoint(const AdjParams &A, const double *const vel[3], const double *const mu[3],
                                   double *const lam[3], double *glid, hipStream_t s);
hipError_t launch_scale_open(const AdjParams &A, const double *const a[3], double scale, double *const out[3],
                             hipStream_t s);
hipError_t launch_sumsq_open(const AdjParams &A, const double *const a[3], double *part, double *out, hipStream_t s);
hipError_t launch_lid_synth(const AdjParams &A, const double *coef, int M, double *lid, hipStream_t s);
hipError_t launch_lid_project(const AdjParams &A, const double *glid, int M, double *gcoef, hipStream_t s);

}  // namespace nsp
