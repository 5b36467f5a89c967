// gfx950 kernels of libnsp: one persistent, cooperatively launched kernel
// that runs whole projection steps (or a Poisson solve) for a batch of
// slices of up to kMaxGroups grids, with the CG loop resident on the device.
//
// Method (Croce, Ruprecht & Krause, Sec. 2): forward-Euler Chorin-Temam
// projection on a uniform staggered grid.  One step:
//   MOM   predictor F = u + dt (Lap(u)/Re - Conv_SMART(u)) on open faces
//   RHS   b = -div(F)/dt on fluid cells, then b -= mean_fluid(b)
//   CG    Jacobi-preconditioned CG on A p = b, A = -D G (7-point, open faces)
//         [or: FP64 residual + FP32 inner CG + FP64 update, repeated]
//   CORR  u = F - dt G p on open faces, 0 on closed faces; p gauge-fixed
//
// Work is split into tiles of `tile` consecutive cells of one slice; each
// tile writes its own partial sums (fixed-order wave64 butterflies, then a
// fixed combination of the four waves), so every reduction result depends
// only on the grid, never on the launch shape or on the batch it shares.
// Between phases all workgroups meet at a grid barrier whose arrivals are
// combined per XCD (one L2 write-back per XCD and barrier, see SyncWords).
// After it every workgroup reads all the slices' partials and sums them
// itself, one wave per slice, in the same fixed order, then runs the CG
// scalar logic (alpha, beta, convergence, cold start) on its own LDS copy of
// each slice's state; identical inputs and order give every workgroup the
// same result, so no reducer workgroup and no second barrier are needed.
// Launches whose CG tiles fit one per workgroup keep x, r and the search
// direction in registers across the whole solve (the RR instantiation).
#include "nsp_internal.h"

namespace nsp {

namespace {

constexpr unsigned kSpinLimit = 1u << 23;

// Pointers taken from the parameter block are generic; accesses through them
// would be flat instructions (which also wait on LDS traffic).  Everything
// the kernels touch lives in device global memory, so cast first.
#define GAS __attribute__((address_space(1)))
#define LAS __attribute__((address_space(3)))
template <class T>
__device__ __forceinline__ GAS T *gp(T *p) { return (GAS T *)p; }
template <class T>
__device__ __forceinline__ const GAS T *gp(const T *p) { return (const GAS T *)p; }  // ~seconds: a wait this long means something is broken

enum Red : int {
    R_NONE = 0, R_MEANB, R_INIT, R_A, R_B, R_TRUE, R_OUT0, R_OUT, R_CAST, R_A32, R_B32, R_BG1, R_BG2, R_BG3,
    R_SR0, R_SR, R_CAST0RU, R_B32RU, R_OUTRU, R_CASTRU
};

// a * b + c with one rounding.  The library is compiled with
// -ffp-contract=off, so the compiler fuses nothing on its own; the CG
// kernels fuse explicitly, so every instantiation computes the same bits.
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// s_waitcnt operand (gfx9 encoding) for vmcnt(0) with expcnt/lgkmcnt untouched
constexpr unsigned kWaitVm0 = 0x0F70;

// Hardware XCD (accelerator complex die) index of the executing workgroup.
__device__ __forceinline__ unsigned hw_xcc_id() {
    unsigned x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    return x & (kMaxXcd - 1);
}

// v of the lane selected by the DPP control CTRL (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double read_lane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | lo);
}

// Sum over the 64 lanes of a full wave, in one fixed order (so every wave,
// workgroup and launch gets the same bits from the same values): pairs,
// quads, half rows and rows by DPP moves (a + b and b + a are the same
// double, so each group holds one value), then the four row sums as
// (r0 + r1) + (r2 + r3).  Returns the same value in every lane.
__device__ __forceinline__ double wave_sum(double v) {
    v = v + dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
    v = v + dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
    v = v + dpp_move<0x141>(v);  // row_half_mirror
    v = v + dpp_move<0x140>(v);  // row_mirror
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// ---------------------------------------------------------------- geometry

struct IJK { int i, j, k; };

__device__ __forceinline__ IJK decomp(const GAS GroupDesc &G, int c) {
    IJK r;
    int t = c / G.nx;
    r.i = c - t * G.nx;
    r.k = t / G.ny;
    r.j = t - r.k * G.ny;
    return r;
}

// extent of component C's face array along direction D
template <int C, int D>
__device__ __forceinline__ int fext(const GAS GroupDesc &G) {
    int n = D == 0 ? G.nx : (D == 1 ? G.ny : G.nz);
    return n + (C == D ? 1 : 0);
}

template <int C>
__device__ __forceinline__ long fidx(const GAS GroupDesc &G, int i, int j, int k) {
    return ((long)k * fext<C, 1>(G) + j) * fext<C, 0>(G) + i;
}

template <int C, int D>
__device__ __forceinline__ long fstride(const GAS GroupDesc &G) {
    return D == 0 ? 1L : (D == 1 ? (long)fext<C, 0>(G) : (long)fext<C, 0>(G) * fext<C, 1>(G));
}

__device__ __forceinline__ long cidx(const GAS GroupDesc &G, int i, int j, int k) {
    return ((long)k * G.ny + j) * G.nx + i;
}

// z position wrapped into [0, nz) on grids periodic in z; unchanged otherwise
__device__ __forceinline__ int wrapk(const GAS GroupDesc &G, int k) {
    if (!G.pz) return k;
    k %= G.nz;
    return k < 0 ? k + G.nz : k;
}

// Face of component C at (i,j,k) separates cells (i,j,k) - e_C and (i,j,k);
// it is open when both are fluid cells, which the cell's own "minus" bit
// records.  Positions outside the face array are not open.
template <int C>
__device__ __forceinline__ bool face_open(const GAS GroupDesc &G, int i, int j, int k) {
    k = wrapk(G, k);
    if (i < 0 || j < 0 || k < 0) return false;
    if (i >= G.nx || j >= G.ny || k >= G.nz) return false;  // includes the high boundary face
    const uint8_t bit = C == 0 ? FL_XM : (C == 1 ? FL_YM : FL_ZM);
    return (gp(G.flags)[cidx(G, i, j, k)] & bit) != 0;
}

// Wall value beyond the open face (i,j,k) of component C in direction D,
// sense S: only u sees the lid, across the top boundary.
template <int C, int D>
__device__ __forceinline__ double wall_value(const GAS GroupDesc &G, int i, int j, int k, int S) {
    if (C == 0 && D == 1 && S > 0 && j == G.ny - 1) return gp(G.lid)[(long)k * (G.nx + 1) + i];
    return 0.0;
}

// ------------------------------------------------------------------ SMART

// Normalised-variable SMART (Gaskell & Lau): phi_hat = (C-U)/(D-U); face
// value 3 phi_hat on (0,1/6), 3/4 phi_hat + 3/8 on [1/6,5/6), 1 on [5/6,1),
// first-order upwind elsewhere.
__device__ __forceinline__ double smart_face(double U, double C, double D) {
    double delta = D - U;
    if (delta == 0.0) return C;
    double ph = (C - U) / delta;
    double pf;
    if (ph > 0.0 && ph < 1.0 / 6.0) pf = 3.0 * ph;
    else if (ph >= 1.0 / 6.0 && ph < 5.0 / 6.0) pf = 0.75 * ph + 0.375;
    else if (ph >= 5.0 / 6.0 && ph < 1.0) pf = 1.0;
    else pf = ph;
    return U + pf * delta;
}

// ------------------------------------------------------- momentum stencil

// Values at offsets -2,-1,+1,+2 along D of the stencil of the open face
// (i,j,k) of component C.  FAST: every position is an open face.  Otherwise
// the image rule: along C's own axis a closed face holds 0 and the next
// position is the odd reflection -phi0; across it a closed neighbour is a
// wall half a cell away, image 2*wall - mirror (no-slip) or the mirror value
// (free-slip obstacle), with the mirror itself resolved first (one-cell gaps).
template <bool FAST, int C, int D>
__device__ __forceinline__ void line_values(const GAS GroupDesc &G, const GAS double *__restrict__ phi, int i, int j,
                                            int k, long id, double phi0, double &vm2, double &vm1, double &vp1,
                                            double &vp2) {
    const long s = fstride<C, D>(G);
    if (FAST) {
        vm2 = phi[id - 2 * s];
        vm1 = phi[id - s];
        vp1 = phi[id + s];
        vp2 = phi[id + 2 * s];
        return;
    }
    const int di = D == 0, dj = D == 1, dk = D == 2;
    // value at offset m along D (wrapped across the periodic z seam)
    auto at = [&](int m) -> double {
        if (D == 2 && G.pz) return phi[fidx<C>(G, i, j, wrapk(G, k + m))];
        return phi[id + m * s];
    };
    const bool om1 = face_open<C>(G, i - di, j - dj, k - dk);
    const bool op1 = face_open<C>(G, i + di, j + dj, k + dk);
    if (C == D) {
        vm1 = om1 ? at(-1) : 0.0;
        vp1 = op1 ? at(1) : 0.0;
        vm2 = !om1 ? -phi0 : (face_open<C>(G, i - 2 * di, j - 2 * dj, k - 2 * dk) ? at(-2) : 0.0);
        vp2 = !op1 ? -phi0 : (face_open<C>(G, i + 2 * di, j + 2 * dj, k + 2 * dk) ? at(2) : 0.0);
    } else {
        // a closed position inside the grid along D is closed by a solid
        // cell (an obstacle wall); with free-slip obstacles its image is the
        // mirror value itself instead of 2*wall - mirror
        const int pD = D == 0 ? i : (D == 1 ? j : k), nD = D == 0 ? G.nx : (D == 1 ? G.ny : G.nz);
        auto slip = [&](int m) { return G.slip && ((D == 2 && G.pz) || (pD + m >= 0 && pD + m < nD)); };
        const double wm = wall_value<C, D>(G, i, j, k, -1);
        const double wp = wall_value<C, D>(G, i, j, k, +1);
        vm1 = om1 ? at(-1) : (slip(-1) ? phi0 : 2.0 * wm - phi0);
        vp1 = op1 ? at(1) : (slip(1) ? phi0 : 2.0 * wp - phi0);
        if (!op1) vp2 = slip(1) ? vm1 : 2.0 * wp - vm1;
        else if (face_open<C>(G, i + 2 * di, j + 2 * dj, k + 2 * dk)) vp2 = at(2);
        else vp2 = slip(2) ? at(1) : 2.0 * wall_value<C, D>(G, i + di, j + dj, k + dk, +1) - at(1);
        if (!om1) vm2 = slip(-1) ? vp1 : 2.0 * wm - vp1;
        else if (face_open<C>(G, i - 2 * di, j - 2 * dj, k - 2 * dk)) vm2 = at(-2);
        else vm2 = slip(-2) ? at(-1) : 2.0 * wall_value<C, D>(G, i - di, j - dj, k - dk, -1) - at(-1);
    }
}

// real value of component D at face (i,j,k): closed faces hold 0
template <bool FAST, int D>
__device__ __forceinline__ double real_face(const GAS GroupDesc &G, const GAS double *__restrict__ a, int i, int j, int k) {
    if (FAST) return a[fidx<D>(G, i, j, k)];
    k = wrapk(G, k);
    return face_open<D>(G, i, j, k) ? a[fidx<D>(G, i, j, k)] : 0.0;
}

// Contribution of direction D to the convective and diffusive terms at the
// open face (i,j,k) of component C.
template <bool FAST, int C, int D>
__device__ __forceinline__ void dir_terms(const GAS GroupDesc &G, const GAS double *const *vel, int i, int j,
                                          int k, long id, double phi0, double &conv, double &lap) {
    const GAS double *phi = vel[C];
    double vm2, vm1, vp1, vp2;
    line_values<FAST, C, D>(G, phi, i, j, k, id, phi0, vm2, vm1, vp1, vp2);
    double ap, am;
    if (C == D) {
        ap = 0.5 * (phi0 + vp1);  // along the own axis the +-1 values are the real ones
        am = 0.5 * (vm1 + phi0);
    } else {
        // the two D-faces straddling the position of the face along C
        const int ci = C == 0, cj = C == 1, ck = C == 2;
        const int di = D == 0, dj = D == 1, dk = D == 2;
        ap = 0.5 * (real_face<FAST, D>(G, vel[D], i - ci + di, j - cj + dj, k - ck + dk) +
                    real_face<FAST, D>(G, vel[D], i + di, j + dj, k + dk));
        am = 0.5 * (real_face<FAST, D>(G, vel[D], i - ci, j - cj, k - ck) + real_face<FAST, D>(G, vel[D], i, j, k));
    }
    // face values: SMART of the upwind triple, or (donor cell) its central
    // node, the node on the face's upwind side
    double fp = 0.0, fm = 0.0;
    if (G.upwind) {
        if (ap != 0.0) fp = ap * (ap > 0.0 ? phi0 : vp1);
        if (am != 0.0) fm = am * (am > 0.0 ? vm1 : phi0);
    } else {
        if (ap != 0.0) fp = ap * (ap > 0.0 ? smart_face(vm1, phi0, vp1) : smart_face(vp2, vp1, phi0));
        if (am != 0.0) fm = am * (am > 0.0 ? smart_face(vm2, vm1, phi0) : smart_face(vp1, phi0, vm1));
    }
    conv += (fp - fm) * G.ih[D];
    lap += ((vp1 - 2.0 * phi0) + vm1) * G.ih2[D];
}

template <bool FAST, int C>
__device__ __forceinline__ double predictor(const GAS GroupDesc &G, const GAS double *const *vel, int i, int j,
                                            int k, double dt) {
    const long id = fidx<C>(G, i, j, k);
    const double phi0 = vel[C][id];
    double conv = 0.0, lap = 0.0;
    dir_terms<FAST, C, 0>(G, vel, i, j, k, id, phi0, conv, lap);
    dir_terms<FAST, C, 1>(G, vel, i, j, k, id, phi0, conv, lap);
    dir_terms<FAST, C, 2>(G, vel, i, j, k, id, phi0, conv, lap);
    return phi0 + dt * (lap * G.inv_re - conv);
}

// ------------------------------------------------------------ the runner

// RR: the kernel instantiation for launches whose CG vectors stay in
// registers (PCG only); the other holds the streaming CG, BiCGStab and the
// single-reduction CG.  Two instantiations keep each one's register
// allocation free of the other's code.
template <bool RR>
struct Runner {
    const GAS KParams &P;
    int tb, te, ts;        // my tiles: tb, tb + ts, ... < te
    int cb, ce, cs;        // my CG tiles, same scheme over the CG tile list
    LAS double *s_red;     // [kWaves * kNQ] wave partials
    const LAS double *s_idg;   // [kMaxGroups * 64]
    const LAS float *s_idg32;  // [kMaxGroups * 64]
    LAS double *s_plane;       // two buffers of (cby + 2) * nx: a column tile's plane with halo rows
    LAS SliceCtl *s_ctl;       // [nslices] this workgroup's copy of the slices' CG state
    const LAS double *s_nf;    // [nslices] fluid cells of the slice's grid
    const LAS int *s_pb;       // [nslices][2] first partial of the slice (flat, CG tiles)
    const LAS int *s_pn;       // [nslices][2] partials of the slice (flat, CG tiles)
    LAS double *s_sum;         // [nslices][kNQ] reduced sums of the last barrier
    const LAS unsigned *s_nx;  // [kMaxXcd] workgroups of this launch on each XCD
    unsigned xcc;              // this workgroup's XCD
    LAS double *s_blk;         // [kMaxBlk][kWaves][kNQ] wave partials of a column tile's plane blocks
    unsigned epoch = 0;        // barriers passed (uniform over the grid)

    __device__ __forceinline__ void locate(int t, int &gi, int &sl) const {
        gi = 0;
        while (gi + 1 < P.ngroups && t >= P.g[gi + 1].tile0) ++gi;
        sl = (t - P.g[gi].tile0) / P.g[gi].ntiles;
    }

    __device__ __forceinline__ void locate_cg(int t, int &gi, int &sl) const {
        gi = 0;
        while (gi + 1 < P.ngroups && t >= P.g[gi + 1].cgtile0) ++gi;
        sl = (t - P.g[gi].cgtile0) / P.g[gi].cgtiles;
    }

    // fixed pairwise tree over the per-wave sums of quantity q
    __device__ __forceinline__ double combine_waves(int q) const {
        double w[kWaves];
#pragma unroll
        for (int i = 0; i < kWaves; ++i) w[i] = s_red[i * kNQ + q];
#pragma unroll
        for (int span = 1; span < kWaves; span *= 2)
#pragma unroll
            for (int i = 0; i + span < kWaves; i += 2 * span) w[i] = w[i] + w[i + span];
        return w[0];
    }

    // Sum the NQ per-thread values over the workgroup in a fixed order and
    // store them as tile t's partials.
    template <int NQ>
    __device__ __forceinline__ void store_partials(double (&acc)[NQ], int t) {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double v = wave_sum(acc[q]);
            if (lane == 0) s_red[wv * kNQ + q] = v;
        }
        __syncthreads();
        if (threadIdx.x < NQ) {
            const int q = threadIdx.x;
            double v = combine_waves(q);
            // partials feed the next barrier (epoch + 1): buffer of its parity
            gp(P.part)[(long)(((epoch + 1) & 1) * kNQ + q) * P.pstride + t] = v;
        }
        __syncthreads();
    }

    // Loop over my tiles; `skip(G, gs)` is uniform per tile; `body(G, sl,
    // gs, c, acc)` handles cell c of local slice sl (global slice gs).
    template <int NQ, class Skip, class Body>
    __device__ __forceinline__ void tiles(Skip skip, Body body) {
        for (int t = tb; t < te; t += ts) {
            int gi, sl;
            locate(t, gi, sl);
            const GAS GroupDesc &G = P.g[gi];
            const int gs = G.slice0 + sl;
            if (skip(G, gs)) continue;
            constexpr int NA = NQ > 0 ? NQ : 1;
            double acc[NA];
#pragma unroll
            for (int q = 0; q < NA; ++q) acc[q] = 0.0;
            const int lt = t - G.tile0 - sl * G.ntiles;
            const int base = lt * G.tile;
            const int end = min(base + G.tile, G.ncells);
            for (int c = base + (int)threadIdx.x; c < end; c += kBlock) body(G, sl, gs, c, acc);
            if constexpr (NQ > 0) store_partials<NA>(acc, t);
        }
    }

    // ------------------------------------------------------- grid barrier


    __device__ __forceinline__ bool aborted() const {
        return __hip_atomic_load(&gp(P.sync)->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    }

    // Wave 0 only: spin until w[i] >= e for every i < n (all lanes load
    // their share each round, then vote); then one acquire fence for the
    // workgroup.  False if the launch was abandoned.
    __device__ __forceinline__ bool wave0_wait_all(const GAS unsigned *w, int n, unsigned e) const {
        const int lane = threadIdx.x & 63;
        unsigned spins = 0;
        bool ok = true;
        for (;;) {
            int mine = 1;
            for (int i = lane; i < n; i += 64)
                mine &= __hip_atomic_load(&w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= e;
            if (__all(mine)) break;
            __builtin_amdgcn_s_sleep(1);
            if ((++spins & 63u) == 0) {
                if (aborted()) { ok = false; break; }
                if (spins > kSpinLimit) {
                    __hip_atomic_store(&gp(P.sync)->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = false;
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        return ok;
    }

    __device__ __forceinline__ static int nq_of(int rid) {
        switch (rid) {
        case R_MEANB: case R_A: case R_A32: case R_BG1: return 1;
        case R_B: case R_B32: case R_CAST: case R_BG2: case R_BG3: case R_CAST0RU: case R_B32RU: case R_CASTRU:
            return 2;
        case R_OUTRU: return 3;
        case R_TRUE: case R_OUT: case R_SR0: case R_SR: return 3;
        case R_INIT: case R_OUT0: return 4;
        default: return 0;
        }
    }

    // Every workgroup reduces every slice's partials of the barrier just
    // passed, in one fixed order (wave w takes slices w, w + 16, ...; lane l
    // sums partials l, l + 64, ...; the wave butterfly combines the lanes), so
    // all workgroups obtain bit-identical sums.  Lanes of wave 0 then run the
    // CG scalar logic, one slice each, on this workgroup's copy of the
    // control blocks.  Returns the OR of the slices' flags.
    // one wave's lane sums of NQ quantities over partials t = lane, lane + 64,
    // ... of one slice, in that order; the loads of four consecutive terms
    // are issued together before they are added
    template <int NQ>
    __device__ __forceinline__ void lane_sums(const GAS double *pp, int nt, int lane, double (&v)[kNQ]) {
        constexpr int kRB = 4;
        for (int t0 = lane; t0 < nt; t0 += 64 * kRB) {
            double a[kRB][NQ];
#pragma unroll
            for (int j = 0; j < kRB; ++j)
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    a[j][q] = t0 + 64 * j < nt ? pp[(long)q * P.pstride + t0 + 64 * j] : 0.0;
#pragma unroll
            for (int j = 0; j < kRB; ++j)
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    if (t0 + 64 * j < nt) v[q] += a[j][q];
        }
    }

    __device__ __forceinline__ int reduce_all(int rid, int buf) {
        __shared__ int s_any;
        const int nq = nq_of(rid);
        const int cg = (rid == R_A || rid == R_B || rid == R_A32 || rid == R_B32 || rid == R_BG1 || rid == R_BG2 ||
                        rid == R_SR0 || rid == R_SR || rid == R_B32RU) ? 1 : 0;
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int s = wv; s < P.nslices; s += kWaves) {
            const GAS double *pp = gp(P.part) + (long)(buf * kNQ) * P.pstride + s_pb[2 * s + cg];
            const int nt = s_pn[2 * s + cg];
            double v[kNQ] = {0.0, 0.0, 0.0, 0.0};
            switch (nq) {
            case 1: lane_sums<1>(pp, nt, lane, v); break;
            case 2: lane_sums<2>(pp, nt, lane, v); break;
            case 3: lane_sums<3>(pp, nt, lane, v); break;
            case 4: lane_sums<4>(pp, nt, lane, v); break;
            default: break;
            }
#pragma unroll
            for (int q = 0; q < kNQ; ++q)
                if (q < nq) {
                    const double w = wave_sum(v[q]);
                    if (lane == 0) s_sum[s * kNQ + q] = w;
                }
        }
        __syncthreads();
        if (wv == 0) {
            int f = 0;
            if (lane < P.nslices) {
                double S[kNQ] = {0.0, 0.0, 0.0, 0.0};
                for (int q = 0; q < nq; ++q) S[q] = s_sum[lane * kNQ + q];
                f = control(rid, lane, S, s_nf[lane]);
            }
            // bit 0: some slice iterates; bit 1: some slice takes a cold start
            const int any = (__any(f & 1) ? 1 : 0) | (__any(f & 2) ? 2 : 0);
            if (lane == 0) s_any = any;
        }
        __syncthreads();
        return s_any;
    }

    // Start-up barrier: every workgroup records its XCD, releases, stores
    // epoch 1 into its own word and waits for all; then wave 0 counts the
    // workgroups per XCD.  Returns false if the launch was abandoned.
    __device__ __forceinline__ bool startup(LAS unsigned *nx) {
        __shared__ int s_ok0;
        GAS SyncWords *S = gp(P.sync);
        if (threadIdx.x == 0) {
            __hip_atomic_store(&S->xof[blockIdx.x], xcc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            __hip_atomic_store(&S->arrive[blockIdx.x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (threadIdx.x < 64) {
            const bool ok = wave0_wait_all(S->arrive, gridDim.x, 1u);
            unsigned cnt[kMaxXcd];
#pragma unroll
            for (int x = 0; x < kMaxXcd; ++x) cnt[x] = 0;
            for (int i = threadIdx.x; i < (int)gridDim.x; i += 64) {
                const unsigned x = __hip_atomic_load(&S->xof[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                for (int y = 0; y < kMaxXcd; ++y) cnt[y] += (x == (unsigned)y) ? 1u : 0u;
            }
#pragma unroll
            for (int y = 0; y < kMaxXcd; ++y) {
                unsigned v = cnt[y];
                for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
                if (threadIdx.x == 0) nx[y] = v;
            }
            if (threadIdx.x == 0) s_ok0 = ok;
        }
        __syncthreads();
        epoch = 1;
        return s_ok0;
    }

    // Grid barrier.  Returns the control word (the OR of the slices' flags
    // after the reduction rid; identical in every workgroup), or -1 if the
    // launch was abandoned.  Arrival: each wave waits for its own stores to
    // be acknowledged by the L2, the workgroup increments its XCD's counter
    // (an L2 atomic: every workgroup of the XCD shares that L2), and the
    // XCD's last arriver releases once for the XCD (write-back of the L2)
    // and publishes the epoch.  Departure: wave 0 polls the XCDs' words and
    // acquires.  Then every workgroup reduces the partials itself: one hop,
    // no master.  The partial buffers alternate with the barrier's parity: a
    // workgroup can run at most one barrier ahead of the slowest reader, so
    // the buffer it writes is never the one being read.
    __device__ __forceinline__ int sync(int rid) {
        __shared__ int s_ok;
        const unsigned e = ++epoch;
        GAS SyncWords *S = gp(P.sync);
        __builtin_amdgcn_s_waitcnt(kWaitVm0);  // this wave's stores are in the L2
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned old = __hip_atomic_fetch_add(&S->xcnt[xcc * 64], 1u, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old + 1u == (e - 1u) * s_nx[xcc]) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // release the whole XCD's results
                __hip_atomic_store(&S->xarr[xcc], e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            unsigned spins = 0;
            bool ok = true;
            for (;;) {
                int mine = 1;
                if (lane < kMaxXcd && s_nx[lane] > 0)
                    mine = __hip_atomic_load(&S->xarr[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= e;
                if (__all(mine)) break;
                __builtin_amdgcn_s_sleep(1);
                if ((++spins & 63u) == 0) {
                    if (aborted()) { ok = false; break; }
                    if (spins > kSpinLimit) {
                        __hip_atomic_store(&S->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = false;
                        break;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (lane == 0) s_ok = ok;
        }
        __syncthreads();
        if (!s_ok) return -1;
        if (rid == R_NONE) return 0;
        return reduce_all(rid, (int)(e & 1u));
    }

    __device__ __forceinline__ void finish_solve(LAS SliceCtl &c) {
        c.done = 1;
        c.status = max(c.status, c.step_status);
        c.tot_it += c.it;
        c.max_it = max(c.max_it, c.it);
        c.tot_outer += c.outer;
    }

    // CG scalar logic for one slice after reduction rid; returns this
    // slice's contribution to the control word.
    __device__ __forceinline__ int control(int rid, int s, const double *S, double nf) {
        LAS SliceCtl &c = s_ctl[s];
        switch (rid) {
        case R_MEANB:
            c.mean_b = S[0] / nf;
            return 0;
        case R_INIT: {
            // S0 = ||b||^2, S1 = ||r||^2, S2 = <r,z>, S3 = <b, M^-1 b>.  A warm
            // start worse than none (||r||^2 > ||b||^2) is dropped: the solve
            // starts from p = 0, r = b (written by phase_cold)
            c.bnorm = sqrt(S[0]);
            c.it = 0;
            c.outer = 0;
            c.done = 0;
            c.step_status = 0;
            c.first = 1;
            c.zero = (c.bnorm == 0.0);
            c.active = 0;
            c.cold = 0;
            if (c.zero) return 0;
            c.cold = S[1] > S[0] ? 1 : 0;
            const double rr = c.cold ? S[0] : S[1];
            c.rz = c.cold ? S[3] : S[2];
            if (P.solver == 1) {
                // BiCGStab: r^ = r0, so rho = <r^, r0> = ||r0||^2; alpha = omega = 1
                c.rz = rr;
                c.alpha = 1.0;
                c.omega = 1.0;
            }
            const double rn = sqrt(rr);
            if (!isfinite(rn)) c.step_status = 3;
            else if (rn > P.rtol * c.bnorm) c.active = (c.it < P.maxit) ? 1 : (c.step_status = 2, 0);
            return c.active | (c.cold << 1);
        }
        case R_A:
            if (c.active) c.alpha = c.rz / S[0];
            return 0;
        case R_B: {
            // S0 = <r,z>, S1 = ||r||^2
            if (!c.active) return 0;
            c.beta = S[0] / c.rz;
            c.rz = S[0];
            c.it += 1;
            c.first = 0;
            const double rn = sqrt(S[1]);
            if (!isfinite(rn)) { c.step_status = 3; c.active = 0; }
            else if (rn <= P.rtol * c.bnorm) c.active = 0;
            else if (c.it >= P.maxit) { c.step_status = 2; c.active = 0; }
            return c.active;
        }
        case R_TRUE: {
            // S0 = ||b - A p||^2, S1 = sum p, S2 = <r,z> of the true residual
            if (c.zero) {
                c.rel_true = 0.0;
                c.res_true = 0.0;
                if (!c.done) finish_solve(c);
                return 0;
            }
            if (c.done) return 0;
            c.res_true = sqrt(S[0]);
            c.rel_true = c.res_true / c.bnorm;
            c.mean_p = S[1] / nf;
            const bool ok = c.step_status == 0;
            if (ok && isfinite(c.rel_true) && c.rel_true > 2.0 * P.rtol && c.it < P.maxit) {
                if (P.solver == 1 && c.outer >= 16) {
                    // BiCGStab broke down repeatedly: give up
                    c.step_status = 2;
                    finish_solve(c);
                    return 0;
                }
                c.outer += 1;
                c.rz = S[2];
                if (P.solver == 1) {  // restart BiCGStab with r^ = r
                    c.rz = S[0];
                    c.alpha = 1.0;
                    c.omega = 1.0;
                }
                c.first = 1;
                c.active = 1;
                return 1;
            }
            if (!isfinite(c.rel_true)) c.step_status = 3;
            finish_solve(c);
            return 0;
        }
        case R_OUT0:
        case R_OUT: {
            // S0 = ||r||^2, S1 = sum r, S2 = sum p, S3 = ||b||^2 (first sweep)
            if (rid == R_OUT0) {
                c.bnorm = sqrt(S[3]);
                c.it = 0;
                c.outer = 0;
                c.done = 0;
                c.step_status = 0;
                c.zero = (c.bnorm == 0.0);
                c.need = 0;
                c.cold = 0;
            } else {
                c.cold = 0;
            }
            if (c.done) return 0;
            if (c.zero) {
                c.rel_true = 0.0;
                c.res_true = 0.0;
                finish_solve(c);
                return 0;
            }
            if (rid == R_OUT0 && S[0] > S[3]) {
                // the warm start is worse than none: p = 0 (phase_cold), then
                // the residual is evaluated again
                c.cold = 1;
                return 2;
            }
            c.res_true = sqrt(S[0]);
            c.rel_true = c.res_true / c.bnorm;
            c.mean_p = S[2] / nf;
            c.need = 0;
            if (!isfinite(c.res_true)) c.step_status = 3;
            else if (c.res_true <= P.rtol * c.bnorm) { /* converged */ }
            else if (c.outer >= P.max_outer) c.step_status = 2;
            else { c.need = 1; c.mean_r = S[1] / nf; }
            if (!c.need) finish_solve(c);
            return c.need;
        }
        case R_CAST: {
            // S0 = ||r32||^2, S1 = <r32, z32>
            if (!c.need) return 0;
            c.outer += 1;
            c.r0 = sqrt(S[0]);
            c.rz = S[1];
            c.it_in = 0;
            c.first = 1;
            c.active = (isfinite(c.r0) && c.r0 > P.eta * c.r0 && P.maxit > 0) ? 1 : 0;
            return c.active;
        }
        case R_A32:
            if (c.active) c.alpha = c.rz / S[0];
            c.fresh = 0;
            return 0;
        case R_B32: {
            if (!c.active) return 0;
            c.beta = S[0] / c.rz;
            c.rz = S[0];
            c.it_in += 1;
            c.it += 1;
            c.first = 0;
            const double rn = sqrt(S[1]);
            c.active = (rn > P.eta * c.r0 && c.it_in < P.maxit && isfinite(rn)) ? 1 : 0;
            return c.active;
        }
        case R_BG1: {
            // S0 = <r^, v>: alpha = rho / <r^, v> (zero: breakdown, restart)
            if (!c.active) return 0;
            if (S[0] == 0.0 || !isfinite(S[0])) { c.active = 0; return 0; }
            c.alpha = c.rz / S[0];
            return 0;
        }
        case R_BG2: {
            // S0 = <t, s>, S1 = <t, t>
            if (!c.active) return 0;
            c.omega = S[1] > 0.0 ? S[0] / S[1] : 0.0;
            return 0;
        }
        case R_BG3: {
            // S0 = <r^, r_new> (the next rho), S1 = ||r_new||^2
            if (!c.active) return 0;
            c.it += 1;
            c.first = 0;
            const double rn = sqrt(S[1]);
            if (!isfinite(rn)) { c.step_status = 3; c.active = 0; return 0; }
            if (rn <= P.rtol * c.bnorm) { c.active = 0; return 0; }
            if (c.it >= P.maxit) { c.step_status = 2; c.active = 0; return 0; }
            if (S[0] == 0.0 || c.omega == 0.0) { c.active = 0; return 0; }  // breakdown: restart
            c.beta = (S[0] / c.rz) * (c.alpha / c.omega);
            c.rz = S[0];
            return 1;
        }
        case R_CAST0RU: {
            // reliable updates, first FP32 residual: S0 = ||rt||^2, S1 = <rt, z>
            if (!c.need) return 0;
            c.need = 0;
            c.r0 = sqrt(S[0]);
            c.rz = S[1];
            c.it_in = 0;
            c.first = 1;
            c.active = (isfinite(c.r0) && c.r0 > 0.0 && P.maxit > 0) ? 1 : 0;
            if (!c.active) {
                // nothing to iterate on: the FP64 residual decides at once
                c.step_status = (P.maxit > 0 && isfinite(c.r0)) ? c.step_status : 2;
                finish_solve(c);
            }
            return c.active;
        }
        case R_B32RU: {
            // after an FP32 step: S0 = <rt, z>, S1 = ||rt||^2.  A reliable
            // update is due when the residual has fallen by eta since the last
            // one, below the tolerance, or at the iteration limit
            if (!c.active) return 0;
            c.it_in += 1;
            c.it += 1;
            const double rn = sqrt(S[1]);
            if (rn <= P.eta * c.r0 || rn <= P.rtol * c.bnorm || c.it >= P.maxit || !isfinite(rn)) {
                c.need = 1;
                return 3;
            }
            c.beta = S[0] / c.rz;
            c.rz = S[0];
            c.first = 0;
            return 1;
        }
        case R_OUTRU: {
            // FP64 residual after a reliable update: S0 = ||r||^2, S1 = sum r,
            // S2 = sum p
            if (!c.need) return c.active ? 1 : 0;
            c.outer += 1;
            c.res_true = sqrt(S[0]);
            c.rel_true = c.res_true / c.bnorm;
            c.mean_p = S[2] / nf;
            int stop = 0;
            if (!isfinite(c.res_true)) { c.step_status = 3; stop = 1; }
            else if (c.res_true <= P.rtol * c.bnorm) stop = 1;
            else if (c.outer >= P.max_outer || c.it >= P.maxit) { c.step_status = 2; stop = 1; }
            if (stop) {
                c.need = 0;
                c.active = 0;
                finish_solve(c);
                return 0;
            }
            c.mean_r = S[1] / nf;
            return 3;
        }
        case R_CASTRU: {
            // the new FP32 residual: S0 = ||rt||^2, S1 = <rt, z>; the search
            // direction is kept, beta from the new <rt, z>
            if (!c.need) return c.active ? 1 : 0;
            c.need = 0;
            c.fresh = 1;
            c.r0 = sqrt(S[0]);
            c.beta = S[1] / c.rz;
            c.rz = S[1];
            c.first = 0;
            return 1;
        }
        case R_SR0: {
            // start of a single-reduction CG run: S0 = gamma = <r,u>,
            // S1 = delta = <w,u>, S2 = ||r||^2; the first step has beta = 0
            if (!c.active) return 0;
            c.rz = S[0];
            c.alpha = S[0] / S[1];
            c.beta = 0.0;
            c.first = 1;
            return 1;
        }
        case R_SR: {
            // after a single-reduction step: S0 = gamma, S1 = delta, S2 = ||r||^2
            // of the new residual; the next step's beta and alpha
            if (!c.active) return 0;
            c.it += 1;
            c.first = 0;
            const double rn = sqrt(S[2]);
            if (!isfinite(rn)) { c.step_status = 3; c.active = 0; return 0; }
            if (rn <= P.rtol * c.bnorm) { c.active = 0; return 0; }
            if (c.it >= P.maxit) { c.step_status = 2; c.active = 0; return 0; }
            const double beta = S[0] / c.rz;
            c.alpha = S[0] / (S[1] - beta * S[0] / c.alpha);
            c.beta = beta;
            c.rz = S[0];
            return 1;
        }
        default:
            return 0;
        }
    }

    // ------------------------------------------------------------- phases

    __device__ __forceinline__ const LAS SliceCtl &ctl(int gs) const { return s_ctl[gs]; }

    // pressure after the gauge fix of the last solve
    __device__ __forceinline__ double p_eff(const LAS SliceCtl &c, double p, bool fluid) const {
        if (c.zero) return 0.0;
        return fluid ? p - c.mean_p : p;
    }

    __device__ __forceinline__ void phase_mom(bool gauge) {
        tiles<0>([](const GAS GroupDesc &, int) { return false; },
                 [&](const GAS GroupDesc &G, int sl, int gs, int c, double *) {
                     const IJK x = decomp(G, c);
                     const uint8_t fl = gp(G.flags)[c];
                     const GAS double *vel[3] = {gp(G.u) + (long)sl * G.nu, gp(G.v) + (long)sl * G.nv, gp(G.w) + (long)sl * G.nw};
                     double GAS *Fu = gp(G.Fu) + (long)sl * G.nu, *Fv = gp(G.Fv) + (long)sl * G.nv, *Fw = gp(G.Fw) + (long)sl * G.nw;
                     double fu = 0.0, fv = 0.0, fw = 0.0;
                     if (!(fl & FL_SLOW)) {
                         fu = predictor<true, 0>(G, vel, x.i, x.j, x.k, P.dt);
                         fv = predictor<true, 1>(G, vel, x.i, x.j, x.k, P.dt);
                         fw = predictor<true, 2>(G, vel, x.i, x.j, x.k, P.dt);
                     } else {
                         if (fl & FL_XM) fu = predictor<false, 0>(G, vel, x.i, x.j, x.k, P.dt);
                         if (fl & FL_YM) fv = predictor<false, 1>(G, vel, x.i, x.j, x.k, P.dt);
                         if (fl & FL_ZM) fw = predictor<false, 2>(G, vel, x.i, x.j, x.k, P.dt);
                     }
                     Fu[fidx<0>(G, x.i, x.j, x.k)] = fu;
                     Fv[fidx<1>(G, x.i, x.j, x.k)] = fv;
                     Fw[fidx<2>(G, x.i, x.j, x.k)] = fw;
                     if (x.i == G.nx - 1) Fu[fidx<0>(G, G.nx, x.j, x.k)] = 0.0;
                     if (x.j == G.ny - 1) Fv[fidx<1>(G, x.i, G.ny, x.k)] = 0.0;
                     // the w plane at z = Lz: a closed wall, or (periodic) the face at z = 0
                     if (!G.pz && x.k == G.nz - 1) Fw[fidx<2>(G, x.i, x.j, G.nz)] = 0.0;
                     if (G.pz && x.k == 0) Fw[fidx<2>(G, x.i, x.j, G.nz)] = fw;
                     if (P.extrap) {
                         // warm start of this step's solve: p^s after the gauge
                         // fix, then 2 p^s - p^(s-1) from the second step on
                         double GAS *p = gp(G.p) + (long)sl * G.ncells;
                         double GAS *pp = gp(G.pprev) + (long)sl * G.ncells;
                         const double ps = gauge ? p_eff(ctl(gs), p[c], fl & FL_FLUID) : p[c];
                         if (gauge) p[c] = 2.0 * ps - pp[c];
                         pp[c] = ps;
                     } else if (gauge) {
                         double GAS *p = gp(G.p) + (long)sl * G.ncells;
                         p[c] = p_eff(ctl(gs), p[c], fl & FL_FLUID);
                     }
                 });
    }

    __device__ __forceinline__ void phase_gauge() {
        tiles<0>([](const GAS GroupDesc &, int) { return false; },
                 [&](const GAS GroupDesc &G, int sl, int gs, int c, double *) {
                     double GAS *p = gp(G.p) + (long)sl * G.ncells;
                     p[c] = p_eff(ctl(gs), p[c], gp(G.flags)[c] & FL_FLUID);
                 });
    }

    __device__ __forceinline__ void phase_rhs() {
        tiles<1>([](const GAS GroupDesc &, int) { return false; },
                 [&](const GAS GroupDesc &G, int sl, int, int c, double *acc) {
                     double GAS *b = gp(G.b) + (long)sl * G.ncells;
                     if (!(gp(G.flags)[c] & FL_FLUID)) { b[c] = 0.0; return; }
                     const IJK x = decomp(G, c);
                     const double GAS *Fu = gp(G.Fu) + (long)sl * G.nu, *Fv = gp(G.Fv) + (long)sl * G.nv,
                                  *Fw = gp(G.Fw) + (long)sl * G.nw;
                     const long iu = fidx<0>(G, x.i, x.j, x.k), iv = fidx<1>(G, x.i, x.j, x.k),
                                iw = fidx<2>(G, x.i, x.j, x.k);
                     double div = (Fu[iu + 1] - Fu[iu]) * G.ih[0];
                     div += (Fv[iv + G.nx] - Fv[iv]) * G.ih[1];
                     div += (Fw[iw + (long)G.nx * G.ny] - Fw[iw]) * G.ih[2];
                     const double bv = -div / P.dt;
                     b[c] = bv;
                     acc[0] += bv;
                 });
    }

    // Poisson mode: mean of the caller's right-hand side
    __device__ __forceinline__ void phase_meanb_user() {
        tiles<1>([](const GAS GroupDesc &, int) { return false; },
                 [&](const GAS GroupDesc &G, int sl, int, int c, double *acc) {
                     if (gp(G.flags)[c] & FL_FLUID) acc[0] += gp(G.bin)[(long)sl * G.ncells + c];
                 });
    }

    // (A x)_c over the open faces of cell c, in the order x-,x+,y-,y+,z-,z+
    template <class T, class Get, class H>
    __device__ __forceinline__ T apply_A(const GAS GroupDesc &G, int c, uint8_t fl, T xc, Get get, const H &ih2) const {
        T s = T(0);
        const long sy = G.nx, sz = (long)G.nx * G.ny;
        if (fl & FL_XM) s += (xc - get(c - 1)) * ih2[0];
        if (fl & FL_XP) s += (xc - get(c + 1)) * ih2[0];
        if (fl & FL_YM) s += (xc - get(c - sy)) * ih2[1];
        if (fl & FL_YP) s += (xc - get(c + sy)) * ih2[1];
        // z neighbours wrap around the slice (used only where the bits are set)
        const long zm = c - sz < 0 ? c - sz + G.ncells : c - sz;
        const long zp = c + sz >= G.ncells ? c + sz - G.ncells : c + sz;
        if (fl & FL_ZM) s += (xc - get(zm)) * ih2[2];
        if (fl & FL_ZP) s += (xc - get(zp)) * ih2[2];
        return s;
    }


    __device__ __forceinline__ int group_index(const GAS GroupDesc &G) const { return (int)(&G - P.g); }

    // FP64 CG, initial residual: b -= mean_b (stored), r = b - A p.
    // partials: ||b||^2, ||r||^2, <r,z>, <b, M^-1 b>
    __device__ __forceinline__ void phase_init64(bool from_user) {
        tiles<4>([](const GAS GroupDesc &, int) { return false; },
                 [&](const GAS GroupDesc &G, int sl, int gs, int c, double *acc) {
                     const long off = (long)sl * G.ncells;
                     double GAS *b = gp(G.b) + off, *r = gp(G.r) + off;
                     const double GAS *p = gp(G.p) + off;
                     const uint8_t fl = gp(G.flags)[c];
                     if (!(fl & FL_FLUID)) { b[c] = 0.0; r[c] = 0.0; return; }
                     const double bsrc = from_user ? gp(G.bin)[off + c] : b[c];
                     const double bv = bsrc - ctl(gs).mean_b;
                     b[c] = bv;
                     const double ap = apply_A<double>(G, c, fl, p[c], [&](long n) { return p[n]; }, G.ih2);
                     const double rv = bv - ap;
                     r[c] = rv;
                     const double idg = s_idg[group_index(G) * 64 + (fl & FL_OPEN)];
                     acc[0] += bv * bv;
                     acc[1] += rv * rv;
                     acc[2] += rv * (rv * idg);
                     acc[3] += bv * (bv * idg);
                 });
    }

    // Cold start of the slices whose warm start was worse than none: p = 0
    // on every cell and, when with_r, r = b (the residual of p = 0).
    __device__ __forceinline__ void phase_cold(bool with_r) {
        tiles<0>([&](const GAS GroupDesc &, int gs) { return !ctl(gs).cold; },
                 [&](const GAS GroupDesc &G, int sl, int, int c, double *) {
                     const long off = (long)sl * G.ncells;
                     gp(G.p)[off + c] = 0.0;
                     if (with_r) gp(G.r)[off + c] = gp(G.b)[off + c];
                 });
    }

    // ------------------------------------------------------------ CG loop
    //
    // When the launch is small enough to stay in the Infinity Cache (P.wt),
    // the CG phases write their outputs with device-scope (write-through)
    // stores: the data then streams out during the phase, and the one L2
    // write-back per XCD at the next barrier finds no dirty CG data to flush
    // (measured: 4-7 % per iteration at 128^3 and 8 x 96^3).  HBM-bound
    // launches keep plain stores (write-through cost 3 % at 32 x 128^3).
    //
    // Per iteration two phases touch every cell once (bytes per cell, FP64 /
    // FP32 vectors, flags 1 byte):
    //   A: d_new = z + beta d_old, z = r/diag       read r, d_old  write d_new
    //      partial <d_new, A d_new>                 (A d_new from neighbours'
    //      d_new, recomputed from their r and d_old)
    //   B: q = A d_new; p += alpha d_new; r -= alpha q; partials <r,z>, <r,r>
    //                                                read p, d_new, r  write p, r
    // = 66 B (FP64) / 34 B (FP32) per cell per iteration; q is never stored.
    // Loads are unconditional (neighbour indices clamped into the slice) so
    // the two cells a thread handles per round have all their loads in
    // flight together; closed faces are masked afterwards.

    template <bool WT, class T>
    __device__ __forceinline__ void st_out(GAS T *p, T v) const {
        if constexpr (WT) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else *p = v;
    }

    template <class T>
    __device__ __forceinline__ T ih2_of(const GAS GroupDesc &G, int d) const {
        return sizeof(T) == 8 ? (T)G.ih2[d] : (T)G.ih2f[d];
    }

    template <class T>
    __device__ __forceinline__ T idg_of(int gb, uint8_t f) const {
        return sizeof(T) == 8 ? (T)s_idg[gb + (f & FL_OPEN)] : (T)s_idg32[gb + (f & FL_OPEN)];
    }

    // one tile of phase A; returns this thread's share of <d_new, A d_new>
    template <class T, bool FIRST, bool WT>
    __device__ __forceinline__ double tile_A(const GAS GroupDesc &G, const GAS uint8_t *__restrict__ fl, const GAS T *__restrict__ r,
                             const GAS T *__restrict__ dold, GAS T *__restrict__ dnew, T beta, int base, int end) {
        const int gb = group_index(G) * 64;
        const long sy = G.nx, sz = (long)G.nx * G.ny;
        const long last = G.ncells - 1;
        const long off[6] = {-1, 1, -sy, sy, -sz, sz};
        const T h2[3] = {ih2_of<T>(G, 0), ih2_of<T>(G, 1), ih2_of<T>(G, 2)};
        double acc = 0.0;
        for (int c0 = base + (int)threadIdx.x; c0 < end; c0 += 2 * kBlock) {
            const bool has1 = c0 + kBlock < end;
            const long cc[2] = {c0, has1 ? c0 + kBlock : c0};
            uint8_t f[2], fn[2][6];
            T rc[2], dc[2], rn[2][6], dn[2][6];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                f[u] = fl[cc[u]];
                rc[u] = r[cc[u]];
                dc[u] = FIRST ? T(0) : dold[cc[u]];
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    long n = cc[u] + off[k];
                    // wrap into the slice: z neighbours across a periodic seam;
                    // any other out-of-range neighbour is behind a closed face
                    n = n < 0 ? n + last + 1 : (n > last ? n - last - 1 : n);
                    fn[u][k] = fl[n];
                    rn[u][k] = r[n];
                    dn[u][k] = FIRST ? T(0) : dold[n];
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const T z0 = rc[u] * idg_of<T>(gb, f[u]);
                const T d0 = FIRST ? z0 : fmaT(beta, dc[u], z0);
                T q = T(0);
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    const T zk = rn[u][k] * idg_of<T>(gb, fn[u][k]);
                    const T dk = FIRST ? zk : fmaT(beta, dn[u][k], zk);
                    if (f[u] & (1 << k)) q = fmaT(d0 - dk, h2[k >> 1], q);
                }
                if (u == 0 || has1) {
                    st_out<WT>(&dnew[cc[u]], d0);
                    acc = fmaT((double)d0, (double)q, acc);
                }
            }
        }
        return acc;
    }

    // ---------------------------------------------------- column tiles
    //
    // A column tile covers full x rows, rows [y0, y1) and planes [z0, z1) of
    // one slice.  Thread tid owns (x, y) = (tid % nx, y0 + tid / nx) and
    // walks z keeping d at planes k-1, k, k+1 in registers (loads for the
    // next plane are issued one step ahead); the plane k values go to LDS
    // for the x/y neighbours; the rows just outside [y0, y1) are loaded by
    // the edge-row threads.  Each cell's r, d, flags are read once.

    // The LDS plane holds rows y0-1 .. y1 of plane k (row y0-1 first); the
    // halo rows y0-1 and y1 are computed by threads 0 .. 2nx-1 as a second
    // item (whole waves, since column tiles need nx % 32 == 0 and 2nx <= the
    // workgroup size).  Halo rows outside the domain are never read (their
    // faces are closed) and are filled from a valid cell.
    // A thread carries NI items of a column tile: rows yy and yy + crb (NI =
    // 2, FP32 launches with enough tiles) of the x position tid % nx.  Partial
    // sums are kept per block of crb rows and zsub planes whatever NI and
    // the tile depth are, so neither changes a result.
    template <int NI>
    struct ColPos {
        bool act[NI];   // item inside the tile
        bool halo;      // this thread also computes one halo item
        long c0[NI];    // index of the item at z0; clamped to a valid cell when idle
        long h0;        // index of the halo item at z0 (valid cell)
        int slot[NI];   // LDS slot of the item
        int hslot;      // LDS slot of the halo item
    };

    template <int NI>
    __device__ __forceinline__ ColPos<NI> col_pos(const GAS GroupDesc &G, int y0, int y1, int z0) const {
        ColPos<NI> p;
        const int tid = threadIdx.x, nx = G.nx, R = G.crb;
        const int x = tid % nx, yy = tid / nx;
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            const int row = yy + u * R, y = y0 + row;
            p.act[u] = yy < R && row < G.cby && y < y1;
            p.c0[u] = ((long)z0 * G.ny + (p.act[u] ? y : y0)) * nx + x;
            p.slot[u] = (p.act[u] ? row + 1 : 1) * nx + x;
        }
        p.halo = tid < 2 * nx;
        const bool upper = tid >= nx;
        int yh = upper ? y1 : y0 - 1;
        yh = yh < 0 ? 0 : (yh >= G.ny ? G.ny - 1 : yh);
        p.h0 = ((long)z0 * G.ny + yh) * nx + x;
        p.hslot = upper ? (y1 - y0 + 1) * nx + x : x;
        return p;
    }

    template <class T, int NI>
    struct PlaneLoad {
        uint8_t f[NI], fh;
        T a[NI], b[NI], c[NI], ah, bh;
    };

    // Column-tile partials.  At the end of each zsub-plane block every wave
    // sums its lanes' NI x NQ values (wave_sum) into the block's LDS slots;
    // at the end of the tile one workgroup barrier, then each of the tile's
    // blocks x NI x NQ sums is combined over the waves in the fixed tree of
    // combine_waves and stored as partial pbase + (first block + b) * cnb +
    // row block (rows beyond the grid in the last tile are not stored).  The
    // next write to the slots follows at least one plane step, whose barrier
    // every thread of the combine has passed.
    template <int NQ, int NI>
    __device__ __forceinline__ void stage_block(double (&acc)[NI][NQ], int blk) {
        static_assert(NQ * NI <= kNQ, "wave partial slots");
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < NI; ++u)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const double v = wave_sum(acc[u][q]);
                if (lane == 0) s_blk[(blk * kWaves + wv) * kNQ + u * NQ + q] = v;
                acc[u][q] = 0.0;
            }
        __builtin_amdgcn_sched_barrier(0);
    }

    template <int NQ, int NI>
    __device__ __forceinline__ void flush_blocks(const GAS GroupDesc &G, int nblk, int z0, int pbase, int yb) {
        __syncthreads();
        for (int x = threadIdx.x; x < nblk * NI * NQ; x += kBlock) {
            const int b = x / (NI * NQ), u = (x / NQ) % NI, q = x % NQ;
            const LAS double *L = s_blk + b * kWaves * kNQ + u * NQ + q;
            // the pairwise tree of combine_waves over the 16 waves, written out
            static_assert(kWaves == 16, "wave tree");
            auto l = [&](int i) { return L[i * kNQ]; };
            const double v = (((l(0) + l(1)) + (l(2) + l(3))) + ((l(4) + l(5)) + (l(6) + l(7)))) +
                             (((l(8) + l(9)) + (l(10) + l(11))) + ((l(12) + l(13)) + (l(14) + l(15))));
            const int rb = yb * G.cni + u;
            if (rb < G.cnb) {
                const int t = pbase + ((z0 >> G.zsh) + b) * G.cnb + rb;
                gp(P.part)[(long)(((epoch + 1) & 1) * kNQ + q) * P.pstride + t] = v;
            }
        }
    }

    // phase A over one column tile; stores <d_new, A d_new> per crb rows and
    // zsub planes as partials pbase + (k / zsub) * cnb + row block.  Loads
    // run two planes ahead: two PlaneLoad sets alternate (the loop is
    // unrolled by two so that no register copy waits for a load in flight).
    template <class T, bool FIRST, bool WT, int NI>
    __device__ void col_A(const GAS GroupDesc &G, const GAS uint8_t *__restrict__ fl, const GAS T *__restrict__ r,
                          const GAS T *__restrict__ dold, GAS T *__restrict__ dnew, T beta, int y0, int y1, int z0,
                          int z1, int pbase, int yb) {
        const int gb = group_index(G) * 64;
        const long sz = (long)G.nx * G.ny;
        const int nx = G.nx, nz = G.nz;
        const T hx = ih2_of<T>(G, 0), hy = ih2_of<T>(G, 1), hz = ih2_of<T>(G, 2);
        const ColPos<NI> P0 = col_pos<NI>(G, y0, y1, z0);
        LAS T *plane = reinterpret_cast<LAS T *>(s_plane);
        const int pst = (G.cby + 2) * nx;  // one plane buffer
        auto dn = [&](uint8_t f, T rv, T dv) -> T {
            const T z = rv * idg_of<T>(gb, f);
            return FIRST ? z : fmaT(beta, dv, z);
        };
        // planes beyond nz wrap to the bottom (a periodic seam; with walls the
        // values are masked by the closed faces)
        auto load = [&](int k, PlaneLoad<T, NI> &L) {
            const long o = (long)(k % nz - z0) * sz;
#pragma unroll
            for (int u = 0; u < NI; ++u) {
                L.f[u] = fl[P0.c0[u] + o];
                L.a[u] = r[P0.c0[u] + o];
                if (!FIRST) L.b[u] = dold[P0.c0[u] + o];
            }
            if (P0.halo) {
                L.fh = fl[P0.h0 + o];
                L.ah = r[P0.h0 + o];
                if (!FIRST) L.bh = dold[P0.h0 + o];
            }
        };
        // every prologue load is issued before any of them is used
        PlaneLoad<T, NI> L0{}, LA{}, LB{};
        load(z0, L0);
        load(z0 + 1, LA);
        load(z0 + 2, LB);
        T dm[NI], dc[NI];
        uint8_t fc[NI];
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            const long cm = z0 > 0 ? P0.c0[u] - sz : P0.c0[u] + (long)(nz - 1) * sz;
            const uint8_t fm = fl[cm];
            const T rm = r[cm], om = FIRST ? T(0) : dold[cm];
            dm[u] = dn(fm, rm, om);
            dc[u] = dn(L0.f[u], L0.a[u], L0.b[u]);
            fc[u] = L0.f[u];
        }
        T hc = dn(L0.fh, L0.ah, L0.bh);
        double acc[NI][1];
#pragma unroll
        for (int u = 0; u < NI; ++u) acc[u][0] = 0.0;
        int buf = 0;
        auto step = [&](int k, PlaneLoad<T, NI> &Lk1) {
            T dp[NI];
            uint8_t fp[NI];
#pragma unroll
            for (int u = 0; u < NI; ++u) {
                dp[u] = dn(Lk1.f[u], Lk1.a[u], Lk1.b[u]);
                fp[u] = Lk1.f[u];
            }
            const T hn = dn(Lk1.fh, Lk1.ah, Lk1.bh);
            load(k + 3, Lk1);
            LAS T *pl = plane + buf * pst;
#pragma unroll
            for (int u = 0; u < NI; ++u)
                if (P0.act[u]) pl[P0.slot[u]] = dc[u];
            if (P0.halo) pl[P0.hslot] = hc;
            __syncthreads();
#pragma unroll
            for (int u = 0; u < NI; ++u) {
                const int sl = P0.slot[u];
                const uint8_t f = fc[u];
                const T d0 = dc[u];
                T q = T(0);
                q = (f & FL_XM) ? fmaT(d0 - pl[sl - 1], hx, q) : q;
                q = (f & FL_XP) ? fmaT(d0 - pl[sl + 1], hx, q) : q;
                q = (f & FL_YM) ? fmaT(d0 - pl[sl - nx], hy, q) : q;
                q = (f & FL_YP) ? fmaT(d0 - pl[sl + nx], hy, q) : q;
                q = (f & FL_ZM) ? fmaT(d0 - dm[u], hz, q) : q;
                q = (f & FL_ZP) ? fmaT(d0 - dp[u], hz, q) : q;
                if (P0.act[u]) st_out<WT>(&dnew[P0.c0[u] + (long)(k - z0) * sz], d0);
                acc[u][0] = P0.act[u] ? fmaT((double)d0, (double)q, acc[u][0]) : acc[u][0];
                dm[u] = d0;
                dc[u] = dp[u];
                fc[u] = fp[u];
            }
            hc = hn;
            buf ^= 1;
            if (((k + 1) & ((1 << G.zsh) - 1)) == 0 || k + 1 == z1) stage_block<1, NI>(acc, (k - z0) >> G.zsh);
        };
        for (int k = z0; k < z1; k += 2) {
            step(k, LA);
            if (k + 1 < z1) step(k + 1, LB);
        }
        flush_blocks<1, NI>(G, (z1 - z0 + (1 << G.zsh) - 1) >> G.zsh, z0, pbase, yb);
    }

    // phase B over one column tile: q = A d from d's planes; x += alpha d,
    // r -= alpha q; partials <r,z>, <r,r> per crb rows and zsub planes as in
    // col_A.  Loads and halos as in col_A.
    template <class T, bool WT, int NI>
    __device__ void col_B(const GAS GroupDesc &G, const GAS uint8_t *__restrict__ fl, const GAS T *__restrict__ d,
                          GAS T *__restrict__ x, GAS T *__restrict__ r, T alpha, int y0, int y1, int z0, int z1,
                          int pbase, int yb) {
        double acc[NI][2];
#pragma unroll
        for (int u = 0; u < NI; ++u) acc[u][0] = acc[u][1] = 0.0;
        const int gb = group_index(G) * 64;
        const long sz = (long)G.nx * G.ny;
        const int nx = G.nx, nz = G.nz;
        const T hx = ih2_of<T>(G, 0), hy = ih2_of<T>(G, 1), hz = ih2_of<T>(G, 2);
        const ColPos<NI> P0 = col_pos<NI>(G, y0, y1, z0);
        LAS T *plane = reinterpret_cast<LAS T *>(s_plane);
        const int pst = (G.cby + 2) * nx;
        // plane k: f, a = d, b = x, c = r; ah = halo d
        auto load = [&](int k, PlaneLoad<T, NI> &L) {
            const long o = (long)(k % nz - z0) * sz;
#pragma unroll
            for (int u = 0; u < NI; ++u) {
                L.f[u] = fl[P0.c0[u] + o];
                L.a[u] = d[P0.c0[u] + o];
                L.b[u] = x[P0.c0[u] + o];
                L.c[u] = r[P0.c0[u] + o];
            }
            if (P0.halo) L.ah = d[P0.h0 + o];
        };
        // every prologue load is issued before any of them is used
        PlaneLoad<T, NI> L0{}, LA{}, LB{};
        load(z0, L0);
        load(z0 + 1, LA);
        load(z0 + 2, LB);
        T dm[NI], dc[NI], xc[NI], rc[NI];
        uint8_t fc[NI];
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            dm[u] = d[z0 > 0 ? P0.c0[u] - sz : P0.c0[u] + (long)(nz - 1) * sz];
            dc[u] = L0.a[u];
            xc[u] = L0.b[u];
            rc[u] = L0.c[u];
            fc[u] = L0.f[u];
        }
        T hc = L0.ah;
        int buf = 0;
        auto step = [&](int k, PlaneLoad<T, NI> &Lk1) {
            T dp[NI], xn[NI], rn[NI];
            uint8_t fp[NI];
#pragma unroll
            for (int u = 0; u < NI; ++u) {
                dp[u] = Lk1.a[u];
                xn[u] = Lk1.b[u];
                rn[u] = Lk1.c[u];
                fp[u] = Lk1.f[u];
            }
            const T hn = Lk1.ah;
            load(k + 3, Lk1);
            LAS T *pl = plane + buf * pst;
#pragma unroll
            for (int u = 0; u < NI; ++u)
                if (P0.act[u]) pl[P0.slot[u]] = dc[u];
            if (P0.halo) pl[P0.hslot] = hc;
            __syncthreads();
#pragma unroll
            for (int u = 0; u < NI; ++u) {
                const int sl = P0.slot[u];
                const uint8_t f = fc[u];
                const T d0 = dc[u];
                T q = T(0);
                q = (f & FL_XM) ? fmaT(d0 - pl[sl - 1], hx, q) : q;
                q = (f & FL_XP) ? fmaT(d0 - pl[sl + 1], hx, q) : q;
                q = (f & FL_YM) ? fmaT(d0 - pl[sl - nx], hy, q) : q;
                q = (f & FL_YP) ? fmaT(d0 - pl[sl + nx], hy, q) : q;
                q = (f & FL_ZM) ? fmaT(d0 - dm[u], hz, q) : q;
                q = (f & FL_ZP) ? fmaT(d0 - dp[u], hz, q) : q;
                const T xv = fmaT(alpha, d0, xc[u]);
                const T rv = fmaT(-alpha, q, rc[u]);
                const T z = rv * idg_of<T>(gb, f);
                const bool live = P0.act[u] && (f & FL_FLUID);
                const long c = P0.c0[u] + (long)(k - z0) * sz;
                if (live) {
                    st_out<WT>(&x[c], xv);
                    st_out<WT>(&r[c], rv);
                }
                acc[u][0] = live ? fmaT((double)rv, (double)z, acc[u][0]) : acc[u][0];
                acc[u][1] = live ? fmaT((double)rv, (double)rv, acc[u][1]) : acc[u][1];
                dm[u] = d0;
                dc[u] = dp[u];
                fc[u] = fp[u];
                xc[u] = xn[u];
                rc[u] = rn[u];
            }
            hc = hn;
            buf ^= 1;
            if (((k + 1) & ((1 << G.zsh) - 1)) == 0 || k + 1 == z1) stage_block<2, NI>(acc, (k - z0) >> G.zsh);
        };
        for (int k = z0; k < z1; k += 2) {
            step(k, LA);
            if (k + 1 < z1) step(k + 1, LB);
        }
        flush_blocks<2, NI>(G, (z1 - z0 + (1 << G.zsh) - 1) >> G.zsh, z0, pbase, yb);
    }

    template <class T, int NI>
    __device__ __forceinline__ void col_A_ni(const GAS GroupDesc &G, bool first, const GAS T *r, const GAS T *dold,
                                             GAS T *dnew, T beta, int y0, int y1, int z0, int z1, int pbase, int yb) {
        if (P.wt) {
            if (first) col_A<T, true, true, NI>(G, gp(G.flags), r, dold, dnew, beta, y0, y1, z0, z1, pbase, yb);
            else col_A<T, false, true, NI>(G, gp(G.flags), r, dold, dnew, beta, y0, y1, z0, z1, pbase, yb);
        } else {
            if (first) col_A<T, true, false, NI>(G, gp(G.flags), r, dold, dnew, beta, y0, y1, z0, z1, pbase, yb);
            else col_A<T, false, false, NI>(G, gp(G.flags), r, dold, dnew, beta, y0, y1, z0, z1, pbase, yb);
        }
    }

    __device__ __forceinline__ void cg_tile_bounds(const GAS GroupDesc &G, int lt, int &y0, int &y1, int &z0,
                                                   int &z1, int &yb) const {
        yb = lt % G.cny;
        const int zb = lt / G.cny;
        y0 = yb * G.cby;
        y1 = min(y0 + G.cby, G.ny);
        z0 = zb * G.cbz;
        z1 = min(z0 + G.cbz, G.nz);
    }

    template <class T>
    __device__ __forceinline__ void phase_A(int par) {
        for (int t = cb; t < ce; t += cs) {
            int gi, sl;
            locate_cg(t, gi, sl);
            const GAS GroupDesc &G = P.g[gi];
            const LAS SliceCtl &cs_ = ctl(G.slice0 + sl);
            if (!cs_.active) continue;
            const long off = (long)sl * G.ncells;
            const GAS T *r = gp(reinterpret_cast<const T *>(G.r)) + off;
            const GAS T *dold = gp(reinterpret_cast<const T *>(par ? G.d1 : G.d0)) + off;
            GAS T *dnew = gp(reinterpret_cast<T *>(par ? G.d0 : G.d1)) + off;
            const int lt = t - G.cgtile0 - sl * G.cgtiles;
            const bool first = cs_.first;
            const T beta = first ? T(0) : (T)cs_.beta;
            const int pbase = G.cgpart0 + sl * G.cgparts;
            if (G.cby > 0) {
                int y0, y1, z0, z1, yb;
                cg_tile_bounds(G, lt, y0, y1, z0, z1, yb);
                if constexpr (sizeof(T) == 4) {
                    if (G.cni == 2) {
                        col_A_ni<T, 2>(G, first, r, dold, dnew, beta, y0, y1, z0, z1, pbase, yb);
                        continue;
                    }
                }
                col_A_ni<T, 1>(G, first, r, dold, dnew, beta, y0, y1, z0, z1, pbase, yb);
            } else {
                const int base = lt * G.tile, end = min(base + G.tile, G.ncells);
                double acc[1];
                if (P.wt)
                    acc[0] = first ? tile_A<T, true, true>(G, gp(G.flags), r, dold, dnew, beta, base, end)
                                   : tile_A<T, false, true>(G, gp(G.flags), r, dold, dnew, beta, base, end);
                else
                    acc[0] = first ? tile_A<T, true, false>(G, gp(G.flags), r, dold, dnew, beta, base, end)
                                   : tile_A<T, false, false>(G, gp(G.flags), r, dold, dnew, beta, base, end);
                store_partials<1>(acc, pbase + lt);
            }
        }
    }

    // one tile of phase B: x is p (FP64) or e (FP32)
    template <class T, bool WT>
    __device__ __forceinline__ void tile_B(const GAS GroupDesc &G, const GAS uint8_t *__restrict__ fl, const GAS T *__restrict__ d,
                           GAS T *__restrict__ x, GAS T *__restrict__ r, T alpha, int base, int end, double (&acc)[2]) {
        const int gb = group_index(G) * 64;
        const long sy = G.nx, sz = (long)G.nx * G.ny;
        const long last = G.ncells - 1;
        const long off[6] = {-1, 1, -sy, sy, -sz, sz};
        const T h2[3] = {ih2_of<T>(G, 0), ih2_of<T>(G, 1), ih2_of<T>(G, 2)};
        for (int c0 = base + (int)threadIdx.x; c0 < end; c0 += 2 * kBlock) {
            const bool has1 = c0 + kBlock < end;
            const long cc[2] = {c0, has1 ? c0 + kBlock : c0};
            uint8_t f[2];
            T dc[2], xc[2], rc[2], dn[2][6];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                f[u] = fl[cc[u]];
                dc[u] = d[cc[u]];
                xc[u] = x[cc[u]];
                rc[u] = r[cc[u]];
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    long n = cc[u] + off[k];
                    // wrap into the slice: z neighbours across a periodic seam;
                    // any other out-of-range neighbour is behind a closed face
                    n = n < 0 ? n + last + 1 : (n > last ? n - last - 1 : n);
                    dn[u][k] = d[n];
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                T q = T(0);
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    if (f[u] & (1 << k)) q = fmaT(dc[u] - dn[u][k], h2[k >> 1], q);
                const T xv = fmaT(alpha, dc[u], xc[u]);
                const T rv = fmaT(-alpha, q, rc[u]);
                const T z = rv * idg_of<T>(gb, f[u]);
                if (u == 0 || has1) {
                    st_out<WT>(&x[cc[u]], xv);
                    st_out<WT>(&r[cc[u]], rv);
                    acc[0] = fmaT((double)rv, (double)z, acc[0]);
                    acc[1] = fmaT((double)rv, (double)rv, acc[1]);
                }
            }
        }
    }

    // ------------------------------------------- register-resident CG
    //
    // When a launch has no more CG column tiles than workgroups, every
    // workgroup owns at most one tile for the whole solve, and the tile's
    // vectors x, r and d stay in registers across iterations (thread (x, y)
    // holds its column's K planes).  Per iteration only tile-boundary values
    // (rows y0 and y1 - 1, planes z0 and z1 - 1) go through memory: phase B
    // publishes z = M^-1 r there, phase A publishes d (two buffers by
    // iteration parity).  Phase A forms the halo d = z + beta d_prev from the
    // neighbouring tiles' published z and previous d, phase B reads the halo
    // d the neighbours published in phase A.  Every value is computed by the
    // formulas of col_A and col_B from the same inputs (q is formed again in
    // phase B, as col_B does) and the partials are kept per the same row and
    // plane blocks, so the results equal the streaming phases' bit for bit.
    // The loop writes x back when every slice of the launch is done.
    template <class T, int K>
    struct RRState {
        T r[K], x[K], d[K];
        unsigned long long f;  // flags of the column's K cells, byte k for plane k
    };

    template <class T, int K>
    __device__ __forceinline__ uint8_t rr_flag(const RRState<T, K> &S, int k) const {
        return (uint8_t)((S.f >> (8 * k)) & 0xFF);
    }

    // Stage d of the tile's K planes and of its halo rows (dh, halo threads)
    // in the LDS, plane k at offset k (cby + 2) nx, then one workgroup
    // barrier; the plane buffer of the register-resident instantiation holds
    // all K planes.  The previous reads of the buffer are a grid barrier back.
    template <class T, int K>
    __device__ __forceinline__ void rr_stage(const GAS GroupDesc &G, const ColPos<1> &P0, const RRState<T, K> &S,
                                             const T *dh) {
        LAS T *pl = reinterpret_cast<LAS T *>(s_plane);
        const int pst = (G.cby + 2) * G.nx;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (P0.act[0]) pl[k * pst + P0.slot[0]] = S.d[k];
            if (P0.halo) pl[k * pst + P0.hslot] = dh[k];
        }
        __syncthreads();
    }

    // q = A d at plane k of the column from the staged planes, z neighbours
    // from registers; the order of col_A
    template <class T, int K>
    __device__ __forceinline__ T rr_q(const GAS GroupDesc &G, const ColPos<1> &P0, const RRState<T, K> &S, int k,
                                      T dzm, T dzp, T hx, T hy, T hz) const {
        const LAS T *pl = reinterpret_cast<const LAS T *>(s_plane) + k * (G.cby + 2) * G.nx;
        const int sl = P0.slot[0], nx = G.nx;
        const uint8_t f = rr_flag(S, k);
        const T d0 = S.d[k];
        const T dm = k > 0 ? S.d[k > 0 ? k - 1 : 0] : dzm;
        const T dp = k < K - 1 ? S.d[k < K - 1 ? k + 1 : 0] : dzp;
        T q = T(0);
        q = (f & FL_XM) ? fmaT(d0 - pl[sl - 1], hx, q) : q;
        q = (f & FL_XP) ? fmaT(d0 - pl[sl + 1], hx, q) : q;
        q = (f & FL_YM) ? fmaT(d0 - pl[sl - nx], hy, q) : q;
        q = (f & FL_YP) ? fmaT(d0 - pl[sl + nx], hy, q) : q;
        q = (f & FL_ZM) ? fmaT(d0 - dm, hz, q) : q;
        q = (f & FL_ZP) ? fmaT(d0 - dp, hz, q) : q;
        return q;
    }

    // cells below and above the column's planes (wrapped into the slice)
    template <int K>
    __device__ __forceinline__ void rr_zcells(const GAS GroupDesc &G, const ColPos<1> &P0, int z0, long &cm,
                                              long &cp) const {
        const long sz = (long)G.nx * G.ny;
        cm = z0 > 0 ? P0.c0[0] - sz : P0.c0[0] + (long)(G.nz - 1) * sz;
        cp = P0.c0[0] + (long)((z0 + K) % G.nz - z0) * sz;
    }

    // phase A: d = z + beta d (own cells and halo), publish the boundary d,
    // q = A d, partial <d, q>
    template <class T, int K, bool WT>
    __device__ __forceinline__ void rr_phase_A(const GAS GroupDesc &G, const ColPos<1> &P0, RRState<T, K> &S,
                                               bool first, bool fresh, T beta, const GAS T *__restrict__ rg,
                                               const GAS T *__restrict__ pubz, const GAS T *__restrict__ dprev,
                                               GAS T *__restrict__ dcur, bool edge, int z0, int pbase, int yb) {
        const int gb = group_index(G) * 64;
        const long sz = (long)G.nx * G.ny;
        const GAS uint8_t *fl = gp(G.flags);
        // a neighbouring tile's d: at a (re)start z formed from r as the
        // streaming phase does, else beta d_prev + z from the published values
        // (z from r in memory right after a reliable update replaced r)
        auto dat = [&](long c) -> T {
            if (first) return rg[c] * idg_of<T>(gb, fl[c]);
            return fmaT(beta, dprev[c], fresh ? rg[c] * idg_of<T>(gb, fl[c]) : pubz[c]);
        };
        long cm, cp;
        rr_zcells<K>(G, P0, z0, cm, cp);
        const T dzm = dat(cm), dzp = dat(cp);
        T dh[K];
        if (P0.halo) {
#pragma unroll
            for (int k = 0; k < K; ++k) dh[k] = dat(P0.h0 + (long)k * sz);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const T z = S.r[k] * idg_of<T>(gb, rr_flag(S, k));
            S.d[k] = first ? z : fmaT(beta, S.d[k], z);
            if (P0.act[0] && (edge || k == 0 || k == K - 1)) st_out<WT>(&dcur[P0.c0[0] + (long)k * sz], S.d[k]);
        }
        const T hx = ih2_of<T>(G, 0), hy = ih2_of<T>(G, 1), hz = ih2_of<T>(G, 2);
        rr_stage<T, K>(G, P0, S, dh);
        double acc[1][1] = {{0.0}};
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const T q = rr_q<T, K>(G, P0, S, k, dzm, dzp, hx, hy, hz);
            acc[0][0] = P0.act[0] ? fmaT((double)S.d[k], (double)q, acc[0][0]) : acc[0][0];
        }
        stage_block<1, 1>(acc, 0);
        flush_blocks<1, 1>(G, 1, z0, pbase, yb);
    }

    // phase B: q = A d again (halo d as published in phase A), x += alpha d,
    // r -= alpha q on live cells, partials <r,z>, ||r||^2; publish z of the
    // tile's boundary cells
    template <class T, int K, bool WT>
    __device__ __forceinline__ void rr_phase_B(const GAS GroupDesc &G, const ColPos<1> &P0, RRState<T, K> &S,
                                               T alpha, GAS T *__restrict__ pubz, const GAS T *__restrict__ dcur,
                                               bool edge, int z0, int pbase, int yb) {
        const int gb = group_index(G) * 64;
        const long sz = (long)G.nx * G.ny;
        long cm, cp;
        rr_zcells<K>(G, P0, z0, cm, cp);
        const T dzm = dcur[cm], dzp = dcur[cp];
        T dh[K];
        if (P0.halo) {
#pragma unroll
            for (int k = 0; k < K; ++k) dh[k] = dcur[P0.h0 + (long)k * sz];
        }
        const T hx = ih2_of<T>(G, 0), hy = ih2_of<T>(G, 1), hz = ih2_of<T>(G, 2);
        rr_stage<T, K>(G, P0, S, dh);
        double acc[1][2] = {{0.0, 0.0}};
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const T q = rr_q<T, K>(G, P0, S, k, dzm, dzp, hx, hy, hz);
            const uint8_t f = rr_flag(S, k);
            const T xv = fmaT(alpha, S.d[k], S.x[k]);
            const T rv = fmaT(-alpha, q, S.r[k]);
            const T z = rv * idg_of<T>(gb, f);
            const bool live = P0.act[0] && (f & FL_FLUID);
            if (live) {
                S.x[k] = xv;
                S.r[k] = rv;
            }
            acc[0][0] = live ? fmaT((double)rv, (double)z, acc[0][0]) : acc[0][0];
            acc[0][1] = live ? fmaT((double)rv, (double)rv, acc[0][1]) : acc[0][1];
            if (P0.act[0] && (edge || k == 0 || k == K - 1))
                st_out<WT>(&pubz[P0.c0[0] + (long)k * sz], S.r[k] * idg_of<T>(gb, f));
        }
        stage_block<2, 1>(acc, 0);
        flush_blocks<2, 1>(G, 1, z0, pbase, yb);
    }

    // The CG loop of a launch whose CG tiles fit one per workgroup, with this
    // workgroup's tile (if any) of K planes held in registers.  ra / rb: the
    // reductions after phases A and B (FP64 or FP32 inner CG).  Published
    // boundary values: z in d0; d in d1 and q by iteration parity.  x is
    // written back after the loop, followed by a grid barrier.  Returns the
    // control word after the loop, or -1 if the launch was abandoned.
    template <class T, int K, bool WT>
    __device__ __forceinline__ int rr_loop(int any, int ra, int rb) {
        const bool has = cb < ce;
        int gi = 0, sl = 0;
        if (has) locate_cg(cb, gi, sl);
        const GAS GroupDesc &G = P.g[gi];
        const int gs = G.slice0 + sl;
        const long off = (long)sl * G.ncells;
        const int lt = has ? cb - G.cgtile0 - sl * G.cgtiles : 0;
        int y0 = 0, y1 = 0, z0 = 0, z1 = 0, yb = 0;
        cg_tile_bounds(G, lt, y0, y1, z0, z1, yb);
        const int pbase = G.cgpart0 + sl * G.cgparts;
        const ColPos<1> P0 = col_pos<1>(G, y0, y1, z0);
        const int yrow = (int)((P0.c0[0] / G.nx) % G.ny);
        const bool edge = yrow == y0 || yrow == y1 - 1;
        const GAS T *rg = gp(reinterpret_cast<const T *>(G.r)) + off;
        GAS T *xg = gp(sizeof(T) == 8 ? reinterpret_cast<T *>(G.p) : reinterpret_cast<T *>(G.e)) + off;
        GAS T *pubz = gp(reinterpret_cast<T *>(G.d0)) + off;
        GAS T *pubd[2] = {gp(reinterpret_cast<T *>(G.d1)) + off, gp(reinterpret_cast<T *>(G.q)) + off};
        const long sz = (long)G.nx * G.ny;
        RRState<T, K> S;
        S.f = 0;
        if (has) {
            const GAS uint8_t *fl = gp(G.flags);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const long c = P0.c0[0] + (long)k * sz;
                S.f |= (unsigned long long)fl[c] << (8 * k);
                S.r[k] = rg[c];
                S.x[k] = xg[c];
            }
        }
        int iter = 0;
        while (any > 0) {
            const LAS SliceCtl &c = ctl(gs);
            const bool run = has && c.active;
            GAS T *dcur = pubd[iter & 1];
            const GAS T *dprev = pubd[(iter + 1) & 1];
            if (run)
                rr_phase_A<T, K, WT>(G, P0, S, c.first, c.fresh, c.first ? T(0) : (T)c.beta, rg, pubz, dprev, dcur,
                                     edge, z0, pbase, yb);
            if (sync(ra) < 0) return -1;
            if (run) rr_phase_B<T, K, WT>(G, P0, S, (T)c.alpha, pubz, dcur, edge, z0, pbase, yb);
            any = sync(rb);
            if (any < 0) return -1;
            ++iter;
            if (rb == R_B32RU && (any & 2)) {
                // reliable update of the slices that asked for one: their e to
                // memory, the FP64 phases, then the new FP32 residual into the
                // registers; d stays
                if (has && c.need) {
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        if (P0.act[0] && (rr_flag(S, k) & FL_FLUID)) xg[P0.c0[0] + (long)k * sz] = S.x[k];
                }
                if (sync(R_NONE) < 0) return -1;
                phase_update();
                if (sync(R_NONE) < 0) return -1;
                phase_out(false, false, true);
                any = sync(R_OUTRU);
                if (any < 0) return -1;
                if (any & 2) {
                    phase_cast();
                    any = sync(R_CASTRU);
                    if (any < 0) return -1;
                }
                if (has && c.fresh) {
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        S.r[k] = rg[P0.c0[0] + (long)k * sz];
                        S.x[k] = T(0);
                    }
                }
            }
        }
        if (has) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (P0.act[0] && (rr_flag(S, k) & FL_FLUID)) xg[P0.c0[0] + (long)k * sz] = S.x[k];
        }
        // the phases after the loop read x at other tiles' cells: every
        // workgroup's write-back must be done first
        if (sync(R_NONE) < 0) return -1;
        return any;
    }

    // register-resident CG loop: the tile's depth K is 4 or 8 planes
    template <class T>
    __device__ __forceinline__ int rr_cg(int any, int ra, int rb) {
        int k8 = 0;
        if (cb < ce) {
            int gi, sl;
            locate_cg(cb, gi, sl);
            k8 = P.g[gi].cbz == 8;
        }
        if (P.wt) return k8 ? rr_loop<T, 8, true>(any, ra, rb) : rr_loop<T, 4, true>(any, ra, rb);
        return k8 ? rr_loop<T, 8, false>(any, ra, rb) : rr_loop<T, 4, false>(any, ra, rb);
    }

    // FP64: p += alpha d; r -= alpha A d.  partials <r,z>, ||r||^2
    // FP32 (inner solve of the mixed path): e += alpha d; r -= alpha A d.
    template <class T>
    __device__ __forceinline__ void phase_B(int par) {
        for (int t = cb; t < ce; t += cs) {
            int gi, sl;
            locate_cg(t, gi, sl);
            const GAS GroupDesc &G = P.g[gi];
            const LAS SliceCtl &cs_ = ctl(G.slice0 + sl);
            if (!cs_.active) continue;
            const long off = (long)sl * G.ncells;
            const GAS T *d = gp(reinterpret_cast<const T *>(par ? G.d0 : G.d1)) + off;
            GAS T *x = gp(sizeof(T) == 8 ? reinterpret_cast<T *>(G.p) : reinterpret_cast<T *>(G.e)) + off;
            GAS T *r = gp(reinterpret_cast<T *>(G.r)) + off;
            const int lt = t - G.cgtile0 - sl * G.cgtiles;
            const int pbase = G.cgpart0 + sl * G.cgparts;
            if (G.cby > 0) {
                int y0, y1, z0, z1, yb;
                cg_tile_bounds(G, lt, y0, y1, z0, z1, yb);
                const T al = (T)cs_.alpha;
                if constexpr (sizeof(T) == 4) {
                    if (G.cni == 2) {
                        if (P.wt) col_B<T, true, 2>(G, gp(G.flags), d, x, r, al, y0, y1, z0, z1, pbase, yb);
                        else col_B<T, false, 2>(G, gp(G.flags), d, x, r, al, y0, y1, z0, z1, pbase, yb);
                        continue;
                    }
                }
                if (P.wt) col_B<T, true, 1>(G, gp(G.flags), d, x, r, al, y0, y1, z0, z1, pbase, yb);
                else col_B<T, false, 1>(G, gp(G.flags), d, x, r, al, y0, y1, z0, z1, pbase, yb);
            } else {
                const int base = lt * G.tile, end = min(base + G.tile, G.ncells);
                double acc[2] = {0.0, 0.0};
                if (P.wt) tile_B<T, true>(G, gp(G.flags), d, x, r, (T)cs_.alpha, base, end, acc);
                else tile_B<T, false>(G, gp(G.flags), d, x, r, (T)cs_.alpha, base, end, acc);
                store_partials<2>(acc, pbase + lt);
            }
        }
    }

    // --------------------------------------------- single-reduction CG
    //
    // Chronopoulos & Gear's CG: one phase and one grid barrier per
    // iteration.  Besides x and r it carries u = M^-1 r, w = A u, the search
    // direction p and s = A p.  Iteration i, with alpha and beta from the
    // last barrier, in one pass over each column tile:
    //   s = w + beta s_old,  p = u + beta p_old  (beta = 0 on the first step)
    //   x += alpha p,  r_new = r - alpha s,  u_new = M^-1 r_new,  w_new = A u_new
    //   partials <r_new, u_new>, <w_new, u_new>, ||r_new||^2
    // w_new needs u_new at the six neighbours: each thread forms r_new of its
    // own cell (and of one halo cell) from r, w, s_old and puts u_new into the
    // LDS plane; z neighbours stay in registers, as in col_A.  r, w and s are
    // read at neighbours while they are written, so they alternate between
    // two buffers by iteration parity; p and x are pointwise and stay in
    // place.  Start of a run (SR_W0): w = A M^-1 r and the same partials.
    // Bytes per cell and iteration (FP64): reads r, w, s, p, x, flags; writes
    // r, w, s, p, x: 81 B.
    enum SrMode : int { SR_W0 = 0, SR_FIRST = 1, SR_NEXT = 2 };

    template <class T>
    struct SrLoad {
        uint8_t f, fh;
        T r, w, s, p, x, rh, wh, sh;
    };

    template <class T, int MODE, bool WT>
    __device__ void col_SR(const GAS GroupDesc &G, const GAS uint8_t *__restrict__ fl, const GAS T *__restrict__ r,
                           const GAS T *__restrict__ w, const GAS T *__restrict__ sold, GAS T *__restrict__ pv,
                           GAS T *__restrict__ x, GAS T *__restrict__ rout, GAS T *__restrict__ wout,
                           GAS T *__restrict__ sout, T alpha, T beta, int y0, int y1, int z0, int z1, int pbase,
                           int yb) {
        const int gb = group_index(G) * 64;
        const long sz = (long)G.nx * G.ny;
        const int nx = G.nx, nz = G.nz;
        const T hx = ih2_of<T>(G, 0), hy = ih2_of<T>(G, 1), hz = ih2_of<T>(G, 2);
        const ColPos<1> P0 = col_pos<1>(G, y0, y1, z0);
        LAS T *plane = reinterpret_cast<LAS T *>(s_plane);
        const int pst = (G.cby + 2) * nx;
        // s_i and r_{i+1} from the loaded r_i, w_i and s_{i-1}
        auto snew = [&](T wv, T sv) -> T { return MODE == SR_FIRST ? wv : fmaT(beta, sv, wv); };
        auto rnew = [&](T rv, T wv, T sv) -> T {
            if (MODE == SR_W0) return rv;
            return fmaT(-alpha, snew(wv, sv), rv);
        };
        auto load = [&](int k, SrLoad<T> &L) {
            const long o = (long)(k % nz - z0) * sz;
            const long c0 = P0.c0[0] + o;
            L.f = fl[c0];
            L.r = r[c0];
            if (MODE != SR_W0) {
                L.w = w[c0];
                L.x = x[c0];
                if (MODE == SR_NEXT) {
                    L.s = sold[c0];
                    L.p = pv[c0];
                }
            }
            if (P0.halo) {
                const long h0 = P0.h0 + o;
                L.fh = fl[h0];
                L.rh = r[h0];
                if (MODE != SR_W0) {
                    L.wh = w[h0];
                    if (MODE == SR_NEXT) L.sh = sold[h0];
                }
            }
        };
        SrLoad<T> L0{}, LA{}, LB{};
        load(z0, L0);
        load(z0 + 1, LA);
        load(z0 + 2, LB);
        // the centre plane's new values: u_new, r_new, s, p, x_new
        T uc, rc, sc = T(0), pc = T(0), xc = T(0), um;
        uint8_t fc;
        auto centre = [&](const SrLoad<T> &L, T &u, T &rn, T &sv, T &pp, T &xn) {
            rn = rnew(L.r, L.w, L.s);
            u = rn * idg_of<T>(gb, L.f);
            if (MODE != SR_W0) {
                sv = snew(L.w, L.s);
                const T uo = L.r * idg_of<T>(gb, L.f);
                pp = MODE == SR_FIRST ? uo : fmaT(beta, L.p, uo);
                xn = fmaT(alpha, pp, L.x);
            }
        };
        {
            const long cm = z0 > 0 ? P0.c0[0] - sz : P0.c0[0] + (long)(nz - 1) * sz;
            const uint8_t fm = fl[cm];
            const T rm = r[cm];
            const T wm = MODE != SR_W0 ? w[cm] : T(0), sm = MODE == SR_NEXT ? sold[cm] : T(0);
            um = rnew(rm, wm, sm) * idg_of<T>(gb, fm);
            centre(L0, uc, rc, sc, pc, xc);
            fc = L0.f;
        }
        T hc = rnew(L0.rh, L0.wh, L0.sh) * idg_of<T>(gb, L0.fh);
        double acc[1][3] = {{0.0, 0.0, 0.0}};
        int buf = 0;
        auto step = [&](int k, SrLoad<T> &Lk1) {
            T up, rp, sp = T(0), pp = T(0), xp = T(0);
            centre(Lk1, up, rp, sp, pp, xp);
            const uint8_t fp = Lk1.f;
            const T hn = rnew(Lk1.rh, Lk1.wh, Lk1.sh) * idg_of<T>(gb, Lk1.fh);
            load(k + 3, Lk1);
            LAS T *pl = plane + buf * pst;
            if (P0.act[0]) pl[P0.slot[0]] = uc;
            if (P0.halo) pl[P0.hslot] = hc;
            __syncthreads();
            const int sl = P0.slot[0];
            const uint8_t f = fc;
            T q = T(0);
            q = (f & FL_XM) ? fmaT(uc - pl[sl - 1], hx, q) : q;
            q = (f & FL_XP) ? fmaT(uc - pl[sl + 1], hx, q) : q;
            q = (f & FL_YM) ? fmaT(uc - pl[sl - nx], hy, q) : q;
            q = (f & FL_YP) ? fmaT(uc - pl[sl + nx], hy, q) : q;
            q = (f & FL_ZM) ? fmaT(uc - um, hz, q) : q;
            q = (f & FL_ZP) ? fmaT(uc - up, hz, q) : q;
            const bool live = P0.act[0] && (f & FL_FLUID);
            if (live) {
                const long c = P0.c0[0] + (long)(k - z0) * sz;
                st_out<WT>(&wout[c], q);
                if (MODE != SR_W0) {
                    st_out<WT>(&rout[c], rc);
                    st_out<WT>(&sout[c], sc);
                    st_out<WT>(&pv[c], pc);
                    st_out<WT>(&x[c], xc);
                }
            }
            acc[0][0] = live ? fmaT((double)rc, (double)uc, acc[0][0]) : acc[0][0];
            acc[0][1] = live ? fmaT((double)q, (double)uc, acc[0][1]) : acc[0][1];
            acc[0][2] = live ? fmaT((double)rc, (double)rc, acc[0][2]) : acc[0][2];
            um = uc;
            uc = up;
            rc = rp;
            sc = sp;
            pc = pp;
            xc = xp;
            fc = fp;
            hc = hn;
            buf ^= 1;
            if (((k + 1) & ((1 << G.zsh) - 1)) == 0 || k + 1 == z1) stage_block<3, 1>(acc, (k - z0) >> G.zsh);
        };
        for (int k = z0; k < z1; k += 2) {
            step(k, LA);
            if (k + 1 < z1) step(k + 1, LB);
        }
        flush_blocks<3, 1>(G, (z1 - z0 + (1 << G.zsh) - 1) >> G.zsh, z0, pbase, yb);
    }

    // the single-reduction step over one flat tile (grids without column
    // tiles): each thread forms u_new of its cell and of its six neighbours
    // from their r, w and s_old; partials as col_SR
    template <class T, int MODE, bool WT>
    __device__ __forceinline__ void tile_SR(const GAS GroupDesc &G, const GAS uint8_t *__restrict__ fl,
                                            const GAS T *__restrict__ r, const GAS T *__restrict__ w,
                                            const GAS T *__restrict__ sold, GAS T *__restrict__ pv,
                                            GAS T *__restrict__ x, GAS T *__restrict__ rout,
                                            GAS T *__restrict__ wout, GAS T *__restrict__ sout, T alpha, T beta,
                                            int base, int end, double (&acc)[3]) {
        const int gb = group_index(G) * 64;
        const long sy = G.nx, sz = (long)G.nx * G.ny;
        const long last = G.ncells - 1;
        const long off[6] = {-1, 1, -sy, sy, -sz, sz};
        const T h2[3] = {ih2_of<T>(G, 0), ih2_of<T>(G, 1), ih2_of<T>(G, 2)};
        auto snew = [&](T wv, T sv) -> T { return MODE == SR_FIRST ? wv : fmaT(beta, sv, wv); };
        auto rnew_at = [&](long n) -> T {
            const T rv = r[n];
            if (MODE == SR_W0) return rv;
            return fmaT(-alpha, snew(w[n], MODE == SR_NEXT ? sold[n] : T(0)), rv);
        };
        for (int c = base + (int)threadIdx.x; c < end; c += kBlock) {
            const uint8_t f = fl[c];
            const T rn = rnew_at(c);
            const T u = rn * idg_of<T>(gb, f);
            T q = T(0);
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                if (!(f & (1 << k))) continue;
                long n = c + off[k];
                // wrap into the slice: z neighbours across a periodic seam
                n = n < 0 ? n + last + 1 : (n > last ? n - last - 1 : n);
                const T un = rnew_at(n) * idg_of<T>(gb, fl[n]);
                q = fmaT(u - un, h2[k >> 1], q);
            }
            if (!(f & FL_FLUID)) continue;
            st_out<WT>(&wout[c], q);
            if (MODE != SR_W0) {
                const T wv = w[c];
                const T sv = snew(wv, MODE == SR_NEXT ? sold[c] : T(0));
                const T uo = r[c] * idg_of<T>(gb, f);
                const T pp = MODE == SR_FIRST ? uo : fmaT(beta, pv[c], uo);
                st_out<WT>(&rout[c], rn);
                st_out<WT>(&sout[c], sv);
                st_out<WT>(&pv[c], pp);
                st_out<WT>(&x[c], fmaT(alpha, pp, x[c]));
            }
            acc[0] = fmaT((double)rn, (double)u, acc[0]);
            acc[1] = fmaT((double)q, (double)u, acc[1]);
            acc[2] = fmaT((double)rn, (double)rn, acc[2]);
        }
    }

    template <class T, int MODE>
    __device__ __forceinline__ void sr_tile(const GAS GroupDesc &G, const LAS SliceCtl &cs, long off, int lt,
                                            int pbase, int par) {
        const GAS T *r = gp(reinterpret_cast<const T *>(par ? G.brh : G.r)) + off;
        const GAS T *w = gp(reinterpret_cast<const T *>(par ? G.bv1 : G.bv0)) + off;
        const GAS T *sold = gp(reinterpret_cast<const T *>(par ? G.d1 : G.d0)) + off;
        GAS T *rout = gp(reinterpret_cast<T *>(par ? G.r : G.brh)) + off;
        GAS T *wout = gp(reinterpret_cast<T *>(MODE == SR_W0 ? (par ? G.bv1 : G.bv0) : (par ? G.bv0 : G.bv1))) + off;
        GAS T *sout = gp(reinterpret_cast<T *>(par ? G.d0 : G.d1)) + off;
        GAS T *pv = gp(reinterpret_cast<T *>(G.q)) + off;
        GAS T *x = gp(reinterpret_cast<T *>(G.p)) + off;
        const T al = (T)cs.alpha, be = (T)cs.beta;
        if (G.cby > 0) {
            int y0, y1, z0, z1, yb;
            cg_tile_bounds(G, lt, y0, y1, z0, z1, yb);
            if (P.wt) col_SR<T, MODE, true>(G, gp(G.flags), r, w, sold, pv, x, rout, wout, sout, al, be, y0, y1, z0, z1, pbase, yb);
            else col_SR<T, MODE, false>(G, gp(G.flags), r, w, sold, pv, x, rout, wout, sout, al, be, y0, y1, z0, z1, pbase, yb);
        } else {
            const int base = lt * G.tile, end = min(base + G.tile, G.ncells);
            double acc[3] = {0.0, 0.0, 0.0};
            if (P.wt) tile_SR<T, MODE, true>(G, gp(G.flags), r, w, sold, pv, x, rout, wout, sout, al, be, base, end, acc);
            else tile_SR<T, MODE, false>(G, gp(G.flags), r, w, sold, pv, x, rout, wout, sout, al, be, base, end, acc);
            store_partials<3>(acc, pbase + lt);
        }
    }

    // one single-reduction phase over the active slices' CG tiles; w0: the
    // start of a run (w = A M^-1 r), else an iteration with parity par
    __device__ __forceinline__ void phase_SR(bool w0, int par) {
        for (int t = cb; t < ce; t += cs) {
            int gi, sl;
            locate_cg(t, gi, sl);
            const GAS GroupDesc &G = P.g[gi];
            const LAS SliceCtl &cs_ = ctl(G.slice0 + sl);
            if (!cs_.active) continue;
            const long off = (long)sl * G.ncells;
            const int lt = t - G.cgtile0 - sl * G.cgtiles;
            const int pbase = G.cgpart0 + sl * G.cgparts;
            if (w0) sr_tile<double, SR_W0>(G, cs_, off, lt, pbase, par);
            else if (cs_.first) sr_tile<double, SR_FIRST>(G, cs_, off, lt, pbase, par);
            else sr_tile<double, SR_NEXT>(G, cs_, off, lt, pbase, par);
        }
    }

    // FP64 true residual r = b - A p (stored for a restart).
    // partials ||r||^2, sum p, <r,z>
    __device__ __forceinline__ void phase_true64() {
        tiles<3>([&](const GAS GroupDesc &, int gs) { return ctl(gs).zero || ctl(gs).done; },
                 [&](const GAS GroupDesc &G, int sl, int gs, int c, double *acc) {
                     const uint8_t fl = gp(G.flags)[c];
                     if (!(fl & FL_FLUID)) return;
                     const long off = (long)sl * G.ncells;
                     const double GAS *p = gp(G.p) + off, *b = gp(G.b) + off;
                     double GAS *r = gp(G.r) + off;
                     const double ap = apply_A<double>(G, c, fl, p[c], [&](long n) { return p[n]; }, G.ih2);
                     const double rv = b[c] - ap;
                     r[c] = rv;
                     const double z = rv * s_idg[group_index(G) * 64 + (fl & FL_OPEN)];
                     acc[0] += rv * rv;
                     acc[1] += p[c];
                     acc[2] += rv * z;
                 });
    }

    // ------------------------------------------------------- BiCGStab
    //
    // The paper's solver (Sec. 2), Jacobi right-preconditioned, FP64, flat
    // tiles; three phases per iteration (bytes per cell: 49, 25, 65):
    //   BG1: p = r + beta (p - omega v), v = A M^-1 p    partial <r^, v>
    //   BG2: s = r - alpha v, t = A M^-1 s               partials <t,s>, <t,t>
    //   BG3: x += alpha M^-1 p + omega M^-1 s, r = s - omega t
    //                                                    partials <r^, r>, ||r||^2
    // p and v alternate between two buffers (par), since neighbours read the
    // old values while the new ones are written; s is recomputed, never
    // stored.  After a (re)start (first) the old p and v are zero and r^ = r.

    __device__ __forceinline__ double bg_idg(const GAS GroupDesc &G, uint8_t f) const {
        return s_idg[group_index(G) * 64 + (f & FL_OPEN)];
    }

    // The CG tiles of the launch: column tiles of a grid go to col(G, sl, gs,
    // y0, y1, z0, z1, pbase, yb), which stores its own partials; flat tiles
    // run body(G, sl, gs, c, acc) on each cell and store NQ partials at
    // pbase + tile.
    template <int NQ, class Skip, class Col, class Body>
    __device__ __forceinline__ void cg_tiles(Skip skip, Col col, Body body) {
        for (int t = cb; t < ce; t += cs) {
            int gi, sl;
            locate_cg(t, gi, sl);
            const GAS GroupDesc &G = P.g[gi];
            const int gs = G.slice0 + sl;
            if (skip(G, gs)) continue;
            const int lt = t - G.cgtile0 - sl * G.cgtiles;
            const int pbase = G.cgpart0 + sl * G.cgparts;
            if (G.cby > 0) {
                int y0, y1, z0, z1, yb;
                cg_tile_bounds(G, lt, y0, y1, z0, z1, yb);
                col(G, sl, gs, y0, y1, z0, z1, pbase, yb);
            } else {
                double acc[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
                const int base = lt * G.tile, end = min(base + G.tile, G.ncells);
                for (int c = base + (int)threadIdx.x; c < end; c += kBlock) body(G, sl, gs, c, acc);
                store_partials<NQ>(acc, pbase + lt);
            }
        }
    }

    struct BGLoad {
        uint8_t f, fh;
        double a, b, c, e, ah, bh, ch;
    };

    // BiCGStab phases 1 and 2 over one column tile (FP64, one column per
    // thread), on the plan of col_A: the value y = M^-1 w of each plane is
    // staged in the LDS plane with its halo rows, z neighbours in registers.
    //   MODE 1: w = p = r (first) or r + beta (p_old - omega v_old); stores
    //           p and v = A y; r^ = r on the first iteration; partial <r^, v>.
    //   MODE 2: w = s = r - alpha v; stores t = A y; partials <t, s>, <t, t>.
    template <int MODE, bool WT>
    __device__ void col_BG(const GAS GroupDesc &G, const GAS uint8_t *__restrict__ fl, const GAS double *__restrict__ r,
                           const GAS double *__restrict__ b_in, const GAS double *__restrict__ c_in,
                           GAS double *__restrict__ out0, GAS double *__restrict__ out1, GAS double *__restrict__ rh,
                           bool first, double beta, double omega, double alpha, int y0, int y1, int z0, int z1,
                           int pbase, int yb) {
        constexpr int NQ = MODE == 1 ? 1 : 2;
        const int gb = group_index(G) * 64;
        const long sz = (long)G.nx * G.ny;
        const int nx = G.nx, nz = G.nz;
        const double hx = G.ih2[0], hy = G.ih2[1], hz = G.ih2[2];
        const ColPos<1> P0 = col_pos<1>(G, y0, y1, z0);
        LAS double *plane = reinterpret_cast<LAS double *>(s_plane);
        const int pst = (G.cby + 2) * nx;
        const bool useb = MODE == 2 || !first;
        // w from the loaded values (a = r, b = p_old or v, c = v_old)
        auto wv = [&](double a, double bb, double cc) -> double {
            if (MODE == 1) return first ? a : a + beta * (bb - omega * cc);
            return a - alpha * bb;
        };
        auto load = [&](int k, BGLoad &L) {
            const long o = (long)(k % nz - z0) * sz;
            const long c0 = P0.c0[0] + o;
            L.f = fl[c0];
            L.a = r[c0];
            if (useb) L.b = b_in[c0];
            if (MODE == 1 && !first) L.c = c_in[c0];
            if (MODE == 1 && !first) L.e = rh[c0];
            if (P0.halo) {
                const long h0 = P0.h0 + o;
                L.fh = fl[h0];
                L.ah = r[h0];
                if (useb) L.bh = b_in[h0];
                if (MODE == 1 && !first) L.ch = c_in[h0];
            }
        };
        BGLoad L0{}, LA{}, LB{};
        load(z0, L0);
        load(z0 + 1, LA);
        load(z0 + 2, LB);
        double ym, wc, yc;
        uint8_t fc;
        double ac = L0.a, ec = L0.e;
        {
            const long cm = z0 > 0 ? P0.c0[0] - sz : P0.c0[0] + (long)(nz - 1) * sz;
            const uint8_t fm = fl[cm];
            const double am = r[cm], bm = useb ? b_in[cm] : 0.0, cm_ = (MODE == 1 && !first) ? c_in[cm] : 0.0;
            ym = idg_of<double>(gb, fm) * wv(am, bm, cm_);
            wc = wv(L0.a, L0.b, L0.c);
            yc = idg_of<double>(gb, L0.f) * wc;
            fc = L0.f;
        }
        double hc = idg_of<double>(gb, L0.fh) * wv(L0.ah, L0.bh, L0.ch);
        double acc[1][NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[0][q] = 0.0;
        int buf = 0;
        auto step = [&](int k, BGLoad &Lk1) {
            const double wp = wv(Lk1.a, Lk1.b, Lk1.c);
            const double yp = idg_of<double>(gb, Lk1.f) * wp;
            const uint8_t fp = Lk1.f;
            const double ap = Lk1.a, ep = Lk1.e;
            const double hn = idg_of<double>(gb, Lk1.fh) * wv(Lk1.ah, Lk1.bh, Lk1.ch);
            load(k + 3, Lk1);
            LAS double *pl = plane + buf * pst;
            if (P0.act[0]) pl[P0.slot[0]] = yc;
            if (P0.halo) pl[P0.hslot] = hc;
            __syncthreads();
            const int sl = P0.slot[0];
            const uint8_t f = fc;
            double q = 0.0;
            q = (f & FL_XM) ? fmaT(yc - pl[sl - 1], hx, q) : q;
            q = (f & FL_XP) ? fmaT(yc - pl[sl + 1], hx, q) : q;
            q = (f & FL_YM) ? fmaT(yc - pl[sl - nx], hy, q) : q;
            q = (f & FL_YP) ? fmaT(yc - pl[sl + nx], hy, q) : q;
            q = (f & FL_ZM) ? fmaT(yc - ym, hz, q) : q;
            q = (f & FL_ZP) ? fmaT(yc - yp, hz, q) : q;
            if (P0.act[0]) {
                const long c = P0.c0[0] + (long)(k - z0) * sz;
                if (MODE == 1) {
                    st_out<WT>(&out0[c], wc);
                    st_out<WT>(&out1[c], q);
                    const double rhc = first ? ac : ec;
                    if (first) st_out<WT>(&rh[c], ac);
                    acc[0][0] = fmaT(rhc, q, acc[0][0]);
                } else {
                    st_out<WT>(&out0[c], q);
                    acc[0][0] = fmaT(q, wc, acc[0][0]);
                    acc[0][NQ - 1] = fmaT(q, q, acc[0][NQ - 1]);
                }
            }
            ym = yc;
            yc = yp;
            wc = wp;
            fc = fp;
            ac = ap;
            ec = ep;
            hc = hn;
            buf ^= 1;
            if (((k + 1) & ((1 << G.zsh) - 1)) == 0 || k + 1 == z1) stage_block<NQ, 1>(acc, (k - z0) >> G.zsh);
        };
        for (int k = z0; k < z1; k += 2) {
            step(k, LA);
            if (k + 1 < z1) step(k + 1, LB);
        }
        flush_blocks<NQ, 1>(G, (z1 - z0 + (1 << G.zsh) - 1) >> G.zsh, z0, pbase, yb);
    }

    __device__ __forceinline__ void phase_bg1(int par) {
        auto skip = [&](const GAS GroupDesc &, int gs) { return !ctl(gs).active; };
        auto col = [&](const GAS GroupDesc &G, int sl, int gs, int y0, int y1, int z0, int z1, int pbase, int yb) {
            const LAS SliceCtl &cs = ctl(gs);
            const long off = (long)sl * G.ncells;
            const double GAS *r = gp(G.r) + off;
            const double GAS *pold = gp(par ? G.d1 : G.d0) + off, *vold = gp(par ? G.bv1 : G.bv0) + off;
            double GAS *pnew = gp(par ? G.d0 : G.d1) + off, *vnew = gp(par ? G.bv0 : G.bv1) + off;
            double GAS *rh = gp(G.brh) + off;
            if (P.wt)
                col_BG<1, true>(G, gp(G.flags), r, pold, vold, pnew, vnew, rh, cs.first, cs.beta, cs.omega, 0.0, y0,
                                y1, z0, z1, pbase, yb);
            else
                col_BG<1, false>(G, gp(G.flags), r, pold, vold, pnew, vnew, rh, cs.first, cs.beta, cs.omega, 0.0, y0,
                                 y1, z0, z1, pbase, yb);
        };
        cg_tiles<1>(skip, col, [&](const GAS GroupDesc &G, int sl, int gs, int c, double *acc) {
            const LAS SliceCtl &cs = ctl(gs);
            const long off = (long)sl * G.ncells;
            const GAS uint8_t *fl = gp(G.flags);
            const double GAS *r = gp(G.r) + off;
            const double GAS *pold = gp(par ? G.d1 : G.d0) + off, *vold = gp(par ? G.bv1 : G.bv0) + off;
            double GAS *pnew = gp(par ? G.d0 : G.d1) + off, *vnew = gp(par ? G.bv0 : G.bv1) + off;
            double GAS *rh = gp(G.brh) + off;
            const bool first = cs.first;
            const double beta = cs.beta, omega = cs.omega;
            auto pval = [&](long n) { return first ? r[n] : r[n] + beta * (pold[n] - omega * vold[n]); };
            const uint8_t f = fl[c];
            const double pc = pval(c);
            const double yc = bg_idg(G, f) * pc;
            const double vc = apply_A<double>(G, c, f, yc, [&](long n) { return bg_idg(G, fl[n]) * pval(n); }, G.ih2);
            pnew[c] = pc;
            vnew[c] = vc;
            double rhc;
            if (first) { rhc = r[c]; rh[c] = rhc; }
            else rhc = rh[c];
            acc[0] += rhc * vc;
        });
    }

    __device__ __forceinline__ void phase_bg2(int par) {
        auto skip = [&](const GAS GroupDesc &, int gs) { return !ctl(gs).active; };
        auto col = [&](const GAS GroupDesc &G, int sl, int gs, int y0, int y1, int z0, int z1, int pbase, int yb) {
            const LAS SliceCtl &cs = ctl(gs);
            const long off = (long)sl * G.ncells;
            const double GAS *r = gp(G.r) + off, *v = gp(par ? G.bv0 : G.bv1) + off;
            double GAS *t = gp(G.q) + off;
            if (P.wt)
                col_BG<2, true>(G, gp(G.flags), r, v, nullptr, t, nullptr, nullptr, false, 0.0, 0.0, cs.alpha, y0, y1,
                                z0, z1, pbase, yb);
            else
                col_BG<2, false>(G, gp(G.flags), r, v, nullptr, t, nullptr, nullptr, false, 0.0, 0.0, cs.alpha, y0, y1,
                                 z0, z1, pbase, yb);
        };
        cg_tiles<2>(skip, col, [&](const GAS GroupDesc &G, int sl, int gs, int c, double *acc) {
            const LAS SliceCtl &cs = ctl(gs);
            const long off = (long)sl * G.ncells;
            const GAS uint8_t *fl = gp(G.flags);
            const double GAS *r = gp(G.r) + off, *v = gp(par ? G.bv0 : G.bv1) + off;
            double GAS *t = gp(G.q) + off;
            const double alpha = cs.alpha;
            const uint8_t f = fl[c];
            const double sc = r[c] - alpha * v[c];
            const double zc = bg_idg(G, f) * sc;
            const double tc =
                apply_A<double>(G, c, f, zc, [&](long n) { return bg_idg(G, fl[n]) * (r[n] - alpha * v[n]); }, G.ih2);
            t[c] = tc;
            acc[0] += tc * sc;
            acc[1] += tc * tc;
        });
    }

    __device__ __forceinline__ void phase_bg3(int par) {
        tiles<2>([&](const GAS GroupDesc &, int gs) { return !ctl(gs).active; },
                 [&](const GAS GroupDesc &G, int sl, int gs, int c, double *acc) {
                     const LAS SliceCtl &cs = ctl(gs);
                     const long off = (long)sl * G.ncells;
                     const uint8_t f = gp(G.flags)[c];
                     const double GAS *p = gp(par ? G.d0 : G.d1) + off, *v = gp(par ? G.bv0 : G.bv1) + off;
                     const double GAS *t = gp(G.q) + off, *rh = gp(G.brh) + off;
                     double GAS *x = gp(G.p) + off, *r = gp(G.r) + off;
                     const double alpha = cs.alpha, omega = cs.omega, idg = bg_idg(G, f);
                     const double sc = r[c] - alpha * v[c];
                     x[c] = x[c] + alpha * (idg * p[c]) + omega * (idg * sc);
                     const double rn = sc - omega * t[c];
                     r[c] = rn;
                     acc[0] += rh[c] * rn;
                     acc[1] += rn * rn;
                 });
    }

    // Mixed: FP64 residual r = b - A p.  First sweep also makes b mean-free.
    // partials ||r||^2, sum r, sum p, ||b||^2.  need_only: the slices with a
    // reliable update pending.
    __device__ __forceinline__ void phase_out(bool first, bool from_user, bool need_only = false) {
        tiles<4>([&](const GAS GroupDesc &, int gs) {
                     if (need_only) return !ctl(gs).need;
                     return !first && (ctl(gs).done || ctl(gs).zero);
                 },
                 [&](const GAS GroupDesc &G, int sl, int gs, int c, double *acc) {
                     const long off = (long)sl * G.ncells;
                     double GAS *b = gp(G.b) + off;
                     const double GAS *p = gp(G.p) + off;
                     const uint8_t fl = gp(G.flags)[c];
                     if (!(fl & FL_FLUID)) { if (first) b[c] = 0.0; return; }
                     double bv;
                     if (first) {
                         const double bsrc = from_user ? gp(G.bin)[off + c] : b[c];
                         bv = bsrc - ctl(gs).mean_b;
                         b[c] = bv;
                     } else {
                         bv = b[c];
                     }
                     const double ap = apply_A<double>(G, c, fl, p[c], [&](long n) { return p[n]; }, G.ih2);
                     const double rv = bv - ap;
                     acc[0] += rv * rv;
                     acc[1] += rv;
                     acc[2] += p[c];
                     acc[3] += bv * bv;
                 });
    }

    // Mixed: r32 = fp32(r - mean r), e = 0.  partials ||r32||^2, <r32,z32>
    __device__ __forceinline__ void phase_cast() {
        tiles<2>([&](const GAS GroupDesc &, int gs) { return !ctl(gs).need; },
                 [&](const GAS GroupDesc &G, int sl, int gs, int c, double *acc) {
                     const long off = (long)sl * G.ncells;
                     float GAS *r32 = gp(reinterpret_cast<float *>(G.r)) + off;
                     float GAS *e = gp(G.e) + off;
                     const uint8_t fl = gp(G.flags)[c];
                     e[c] = 0.0f;
                     if (!(fl & FL_FLUID)) { r32[c] = 0.0f; return; }
                     const double GAS *p = gp(G.p) + off, *b = gp(G.b) + off;
                     const double ap = apply_A<double>(G, c, fl, p[c], [&](long n) { return p[n]; }, G.ih2);
                     const double rv = b[c] - ap;
                     const float rf = (float)(rv - ctl(gs).mean_r);
                     r32[c] = rf;
                     const float z = rf * s_idg32[group_index(G) * 64 + (fl & FL_OPEN)];
                     acc[0] += (double)rf * (double)rf;
                     acc[1] += (double)rf * (double)z;
                 });
    }

    // Mixed: p += fp64(e)
    __device__ __forceinline__ void phase_update() {
        tiles<0>([&](const GAS GroupDesc &, int gs) { return !ctl(gs).need; },
                 [&](const GAS GroupDesc &G, int sl, int, int c, double *) {
                     if (!(gp(G.flags)[c] & FL_FLUID)) return;
                     const long off = (long)sl * G.ncells;
                     gp(G.p)[off + c] += (double)gp(G.e)[off + c];
                 });
    }

    // u = F - dt G p_eff on open faces, 0 on closed faces
    __device__ __forceinline__ void phase_corr() {
        tiles<0>([](const GAS GroupDesc &, int) { return false; },
                 [&](const GAS GroupDesc &G, int sl, int gs, int c, double *) {
                     const IJK x = decomp(G, c);
                     const uint8_t fl = gp(G.flags)[c];
                     const LAS SliceCtl &cs = ctl(gs);
                     const long off = (long)sl * G.ncells;
                     const double GAS *p = gp(G.p) + off;
                     double GAS *u = gp(G.u) + (long)sl * G.nu, *v = gp(G.v) + (long)sl * G.nv, *w = gp(G.w) + (long)sl * G.nw;
                     const double GAS *Fu = gp(G.Fu) + (long)sl * G.nu, *Fv = gp(G.Fv) + (long)sl * G.nv,
                                  *Fw = gp(G.Fw) + (long)sl * G.nw;
                     const long iu = fidx<0>(G, x.i, x.j, x.k), iv = fidx<1>(G, x.i, x.j, x.k),
                                iw = fidx<2>(G, x.i, x.j, x.k);
                     const double pc = p_eff(cs, p[c], true);
                     u[iu] = (fl & FL_XM) ? Fu[iu] - P.dt * ((pc - p_eff(cs, p[c - 1], true)) * G.ih[0]) : 0.0;
                     v[iv] = (fl & FL_YM) ? Fv[iv] - P.dt * ((pc - p_eff(cs, p[c - G.nx], true)) * G.ih[1]) : 0.0;
                     const long czm = x.k > 0 ? c - (long)G.nx * G.ny : c - (long)G.nx * G.ny + G.ncells;
                     const double wv = (fl & FL_ZM) ? Fw[iw] - P.dt * ((pc - p_eff(cs, p[czm], true)) * G.ih[2]) : 0.0;
                     w[iw] = wv;
                     if (x.i == G.nx - 1) u[fidx<0>(G, G.nx, x.j, x.k)] = 0.0;
                     if (x.j == G.ny - 1) v[fidx<1>(G, x.i, G.ny, x.k)] = 0.0;
                     if (!G.pz && x.k == G.nz - 1) w[fidx<2>(G, x.i, x.j, G.nz)] = 0.0;
                     if (G.pz && x.k == 0) w[fidx<2>(G, x.i, x.j, G.nz)] = wv;
                 });
    }

    // ---------------------------------------------------------- programs

    // returns false on abort
    // after the initial residual: cold-start the slices that need it
    __device__ __forceinline__ int after_init(int any, bool with_r) {
        if (any < 0) return -1;
        if (any & 2) {
            phase_cold(with_r);
            if (sync(R_NONE) < 0) return -1;
        }
        return any & 1;
    }

    __device__ __forceinline__ bool solve64(bool from_user) {
        phase_init64(from_user);
        int any = after_init(sync(R_INIT), true);
        if (any < 0) return false;
        int iter = 0;
        for (;;) {
            if constexpr (RR) {
                any = rr_cg<double>(any, R_A, R_B);
                if (any < 0) return false;
            } else {
                while (any > 0) {
                    const int par = iter & 1;
                    phase_A<double>(par);
                    if (sync(R_A) < 0) return false;
                    phase_B<double>(par);
                    any = sync(R_B);
                    if (any < 0) return false;
                    ++iter;
                }
            }
            phase_true64();
            any = sync(R_TRUE);
            if (any < 0) return false;
            if (!any) break;
        }
        return true;
    }

    // single-reduction CG: each (re)start begins with w = A M^-1 r (R_SR0),
    // then one phase and one barrier per iteration; r, w, s alternate
    // between two buffers by iteration parity, starting from r in G.r
    __device__ __forceinline__ bool solve_sr(bool from_user) {
        phase_init64(from_user);
        int any = after_init(sync(R_INIT), true);
        if (any < 0) return false;
        for (;;) {
            if (any > 0) {
                phase_SR(true, 0);
                any = sync(R_SR0);
                if (any < 0) return false;
                int iter = 0;
                while (any > 0) {
                    phase_SR(false, iter & 1);
                    any = sync(R_SR);
                    if (any < 0) return false;
                    ++iter;
                }
            }
            phase_true64();
            any = sync(R_TRUE);
            if (any < 0) return false;
            if (!any) break;
        }
        return true;
    }

    // the FP64 solve of the selected solver
    __device__ __forceinline__ bool solve_fp64(bool from_user) {
        if constexpr (!RR) {
            if (P.solver == 1) return solve_bicg(from_user);
            if (P.solver == 2) return solve_sr(from_user);
        }
        return solve64(from_user);
    }

    __device__ __forceinline__ bool solve_bicg(bool from_user) {
        phase_init64(from_user);
        int any = after_init(sync(R_INIT), true);
        if (any < 0) return false;
        int par = 0;
        for (;;) {
            while (any > 0) {
                phase_bg1(par);
                if (sync(R_BG1) < 0) return false;
                phase_bg2(par);
                if (sync(R_BG2) < 0) return false;
                phase_bg3(par);
                any = sync(R_BG3);
                if (any < 0) return false;
                par ^= 1;
            }
            phase_true64();
            any = sync(R_TRUE);
            if (any < 0) return false;
            if (!any) break;
        }
        return true;
    }

    __device__ __forceinline__ bool solve_mixed(bool from_user) {
        phase_out(true, from_user);
        int any = sync(R_OUT0);
        if (any < 0) return false;
        if (any & 2) {
            // cold starts: p = 0, then every unfinished slice's residual again
            phase_cold(false);
            if (sync(R_NONE) < 0) return false;
            phase_out(false, false);
            any = sync(R_OUT);
            if (any < 0) return false;
        }
        int iter = 0;
        while (any > 0) {
            phase_cast();
            int act = sync(R_CAST);
            if (act < 0) return false;
            if constexpr (RR) {
                act = rr_cg<float>(act, R_A32, R_B32);
                if (act < 0) return false;
            } else {
                while (act > 0) {
                    const int par = iter & 1;
                    phase_A<float>(par);
                    if (sync(R_A32) < 0) return false;
                    phase_B<float>(par);
                    act = sync(R_B32);
                    if (act < 0) return false;
                    ++iter;
                }
            }
            phase_update();
            if (sync(R_NONE) < 0) return false;
            phase_out(false, false);
            any = sync(R_OUT);
            if (any < 0) return false;
        }
        return true;
    }

    // Mixed precision with reliable updates: one FP32 CG run per solve whose
    // search direction survives the updates (FP64 residual, fold of e into
    // p, new FP32 residual), in the streaming phases
    __device__ __forceinline__ bool solve_mixed_ru(bool from_user) {
        phase_out(true, from_user);
        int any = sync(R_OUT0);
        if (any < 0) return false;
        if (any & 2) {
            phase_cold(false);
            if (sync(R_NONE) < 0) return false;
            phase_out(false, false);
            any = sync(R_OUT);
            if (any < 0) return false;
        }
        if (!(any & 1)) return true;
        phase_cast();
        int act = sync(R_CAST0RU);
        if (act < 0) return false;
        if constexpr (RR) {
            return rr_cg<float>(act, R_A32, R_B32RU) >= 0;
        } else {
            int iter = 0;
            while (act > 0) {
                const int par = iter & 1;
                phase_A<float>(par);
                if (sync(R_A32) < 0) return false;
                phase_B<float>(par);
                act = sync(R_B32RU);
                if (act < 0) return false;
                ++iter;
                if (act & 2) {
                    phase_update();
                    if (sync(R_NONE) < 0) return false;
                    phase_out(false, false, true);
                    act = sync(R_OUTRU);
                    if (act < 0) return false;
                    if (act & 2) {
                        phase_cast();
                        act = sync(R_CASTRU);
                        if (act < 0) return false;
                    }
                }
            }
            return true;
        }
    }

    __device__ __forceinline__ bool solve_prec(bool from_user) {
        if (P.prec == 0) return solve_fp64(from_user);
        if (P.prec == 2) return solve_mixed_ru(from_user);
        return solve_mixed(from_user);
    }

    __device__ __forceinline__ void run() {
        if (P.mode == MODE_POISSON) {
            phase_meanb_user();
            if (sync(R_MEANB) < 0) return;
            const bool ok = solve_prec(true);
            if (!ok) return;
            phase_gauge();
            return;
        }
        if (P.mode == MODE_PROJECT) {
            phase_rhs();
            if (sync(R_MEANB) < 0) return;
            if (!solve_fp64(false)) return;
            phase_corr();
            if (sync(R_NONE) < 0) return;
            phase_gauge();
            return;
        }
        for (int step = 0; step < P.nsteps; ++step) {
            phase_mom(step > 0);
            if (sync(R_NONE) < 0) return;
            phase_rhs();
            if (sync(R_MEANB) < 0) return;
            const bool ok = solve_prec(false);
            if (!ok) return;
            phase_corr();
            // the correction reads neighbouring pressures: no cell may be
            // gauge-shifted before every workgroup has finished it
            if (sync(R_NONE) < 0) return;
        }
        if (P.nsteps > 0) phase_gauge();
    }
};

// The launch parameters live in device memory (one block per handle): a
// by-value parameter block of this size would be copied to scratch.
// At most 128 VGPRs (4 waves per SIMD): the CG phases need the occupancy;
// the image-rule momentum path may spill instead.
template <bool RR>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_persistent(const KParams *__restrict__ Pp) {
    const GAS KParams &P = *gp(Pp);
    __shared__ double s_red[kWaves * kNQ];
    __shared__ double s_blk[kMaxBlk * kWaves * kNQ];
    // (cby + 2) * nx <= kBlock + 2 nx <= 2 kBlock: two planes streaming, K <= 8
    // planes in the register-resident instantiation
    __shared__ double s_plane[(RR ? 8 : 2) * 2 * kBlock];
    __shared__ double s_idg[kMaxGroups * 64];
    __shared__ float s_idg32[kMaxGroups * 64];
    for (int x = threadIdx.x; x < P.ngroups * 64; x += kBlock) {
        s_idg[x] = P.g[x / 64].idiag[x % 64];
        s_idg32[x] = P.g[x / 64].idiag32[x % 64];
    }
    __syncthreads();
    // Tile schedule.  Workgroups are dispatched to the eight XCDs round-robin
    // (hardware index modulo 8).  Each XCD owns one contiguous range of
    // tiles, and its workgroups take that range's tiles in turn (stride =
    // workgroups on the XCD), so at any moment they sweep a narrow window of
    // consecutive tiles whose neighbouring planes are still in the XCD's L2.
    // The CG tiles are scheduled the same way over their own list.
    const int nb = gridDim.x, b = blockIdx.x;
    int sched[2][3];
    const int totals[2] = {P.ntiles, P.cgtiles};
    for (int w = 0; w < 2; ++w) {
        const int T = totals[w];
        sched[w][0] = b;
        sched[w][1] = T;
        sched[w][2] = nb;
        if (P.xcd_remap && nb >= 8) {
            const int x = b & 7, q = nb >> 3, rm = nb & 7;
            const int first = x * q + min(x, rm), count = q + (x < rm ? 1 : 0);
            sched[w][0] = (int)((long)first * T / nb) + (b >> 3);
            sched[w][1] = (int)((long)(first + count) * T / nb);
            sched[w][2] = count;
        }
    }
    // per-slice tables and this workgroup's copy of the control blocks
    __shared__ SliceCtl s_ctl[kMaxSlices];
    __shared__ double s_nf[kMaxSlices];
    __shared__ int s_pb[2 * kMaxSlices], s_pn[2 * kMaxSlices];
    __shared__ double s_sum[kMaxSlices * kNQ];
    constexpr int kCtlWords = sizeof(SliceCtl) / sizeof(int);
    static_assert(sizeof(SliceCtl) % sizeof(int) == 0, "SliceCtl is copied as words");
    {
        const GAS int *src = reinterpret_cast<const GAS int *>(gp(P.ctl));
        LAS int *dst = reinterpret_cast<LAS int *>((LAS SliceCtl *)s_ctl);
        for (int x = threadIdx.x; x < P.nslices * kCtlWords; x += kBlock) dst[x] = src[x];
        for (int sl = threadIdx.x; sl < P.nslices; sl += kBlock) {
            int gi = 0;
            while (gi + 1 < P.ngroups && sl >= P.g[gi + 1].slice0) ++gi;
            const GAS GroupDesc &G = P.g[gi];
            s_nf[sl] = G.nfluid;
            s_pb[2 * sl] = G.tile0 + (sl - G.slice0) * G.ntiles;
            s_pn[2 * sl] = G.ntiles;
            s_pb[2 * sl + 1] = G.cgpart0 + (sl - G.slice0) * G.cgparts;
            s_pn[2 * sl + 1] = G.cgparts;
        }
    }
    __syncthreads();
    __shared__ unsigned s_nx[kMaxXcd];
    Runner<RR> R{P, sched[0][0], sched[0][1], sched[0][2], sched[1][0], sched[1][1], sched[1][2], (LAS double *)s_red,
             (const LAS double *)s_idg, (const LAS float *)s_idg32, (LAS double *)s_plane, (LAS SliceCtl *)s_ctl,
             (const LAS double *)s_nf, (const LAS int *)s_pb, (const LAS int *)s_pn, (LAS double *)s_sum,
             (const LAS unsigned *)s_nx, hw_xcc_id(), (LAS double *)s_blk};
    if (R.startup((LAS unsigned *)s_nx)) R.run();
    // every workgroup holds the same control blocks: workgroup 0 returns them
    __syncthreads();
    if (blockIdx.x == 0) {
        GAS int *dst = reinterpret_cast<GAS int *>(gp(P.ctl));
        const LAS int *src = reinterpret_cast<const LAS int *>((LAS SliceCtl *)s_ctl);
        for (int x = threadIdx.x; x < P.nslices * kCtlWords; x += kBlock) dst[x] = src[x];
    }
}

// zero n 32-bit words (a kernel rather than a memset node, so that the
// launch sequence stays valid under stream capture)
// one replay's slice results folded into what the graph keeps across replays
__global__ void k_fold_status(const SliceCtl *ctl, const SyncWords *sync, int nslices, GraphFold *f) {
    const int s = threadIdx.x;
    if (s < nslices) {
        const SliceCtl &c = ctl[s];
        if (c.status > f->status[s]) f->status[s] = c.status;
        if (c.max_it > f->max_it[s]) f->max_it[s] = c.max_it;
        f->it[s] += c.tot_it;
        f->outer[s] += c.tot_outer;
    }
    if (s == 0 && sync->abort) f->abort = 1;
}

__global__ void k_zero_words(unsigned *w, long long n) {
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (long long)gridDim.x * blockDim.x)
        w[x] = 0u;
}

// Restriction (coarse output element) or prolongation (fine output element)
// between a fine MAC grid and the grid with half its cells per direction:
// fine cell (k, j, i) lies in coarse cell (k/2, j/2, i/2).  Restriction
// averages the four fine faces tiling a coarse face, summed (a + b) + (c + d)
// with a, b the pair at the lower index of the slower direction, and the
// eight fine cells of a coarse cell (two such four-sums, lower z first).
// Prolongation copies a coarse face to the fine faces inside it and averages
// the two coarse faces around a fine face halfway between them; pressure is
// copied to the eight fine cells.
__global__ void k_transfer(TransferParams T) {
    const long nx = T.nx, ny = T.ny, nz = T.nz, cx = nx / 2, cy = ny / 2, cz = nz / 2;
    // per-slice element counts of the fine and coarse components
    const long fn[4] = {(nx + 1) * ny * nz, nx * (ny + 1) * nz, nx * ny * (nz + 1), nx * ny * nz};
    const long cn[4] = {(cx + 1) * cy * cz, cx * (cy + 1) * cz, cx * cy * (cz + 1), cx * cy * cz};
    for (int c = 0; c < 4; ++c) {
        const long on = T.prolong ? fn[c] : cn[c];  // output elements per slice
        const long total = on * T.batch;
        const double *src = T.src[c];
        double *dst = T.dst[c];
        for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
            const long sl = e / on, r = e - sl * on;
            if (!T.prolong) {
                const double *f = src + sl * fn[c];
                double out;
                if (c == 0) {  // coarse u (K, J, I) of [cz][cy][cx+1]; fine u of [nz][ny][nx+1]
                    const long I = r % (cx + 1), J = (r / (cx + 1)) % cy, K = r / ((cx + 1) * cy);
                    auto at = [&](long k, long j) { return f[(k * ny + j) * (nx + 1) + 2 * I]; };
                    out = 0.25 * ((at(2 * K, 2 * J) + at(2 * K, 2 * J + 1)) + (at(2 * K + 1, 2 * J) + at(2 * K + 1, 2 * J + 1)));
                } else if (c == 1) {  // coarse v of [cz][cy+1][cx]; fine v of [nz][ny+1][nx]
                    const long I = r % cx, J = (r / cx) % (cy + 1), K = r / (cx * (cy + 1));
                    auto at = [&](long k, long i) { return f[(k * (ny + 1) + 2 * J) * nx + i]; };
                    out = 0.25 * ((at(2 * K, 2 * I) + at(2 * K, 2 * I + 1)) + (at(2 * K + 1, 2 * I) + at(2 * K + 1, 2 * I + 1)));
                } else if (c == 2) {  // coarse w of [cz+1][cy][cx]; fine w of [nz+1][ny][nx]
                    const long I = r % cx, J = (r / cx) % cy, K = r / (cx * cy);
                    auto at = [&](long j, long i) { return f[(2 * K * ny + j) * nx + i]; };
                    out = 0.25 * ((at(2 * J, 2 * I) + at(2 * J, 2 * I + 1)) + (at(2 * J + 1, 2 * I) + at(2 * J + 1, 2 * I + 1)));
                } else {  // coarse p of [cz][cy][cx]
                    const long I = r % cx, J = (r / cx) % cy, K = r / (cx * cy);
                    auto at = [&](long k, long j, long i) { return f[(k * ny + j) * nx + i]; };
                    const double z0 = (at(2 * K, 2 * J, 2 * I) + at(2 * K, 2 * J, 2 * I + 1)) +
                                      (at(2 * K, 2 * J + 1, 2 * I) + at(2 * K, 2 * J + 1, 2 * I + 1));
                    const double z1 = (at(2 * K + 1, 2 * J, 2 * I) + at(2 * K + 1, 2 * J, 2 * I + 1)) +
                                      (at(2 * K + 1, 2 * J + 1, 2 * I) + at(2 * K + 1, 2 * J + 1, 2 * I + 1));
                    out = 0.125 * (z0 + z1);
                }
                dst[e] = out;
            } else {
                const double *g = src + sl * cn[c];
                double out;
                if (c == 0) {  // fine u (k, j, i) of [nz][ny][nx+1]
                    const long i = r % (nx + 1), j = (r / (nx + 1)) % ny, k = r / ((nx + 1) * ny);
                    const long b = ((k / 2) * cy + j / 2) * (cx + 1);
                    out = (i & 1) ? 0.5 * (g[b + i / 2] + g[b + i / 2 + 1]) : g[b + i / 2];
                } else if (c == 1) {  // fine v of [nz][ny+1][nx]
                    const long i = r % nx, j = (r / nx) % (ny + 1), k = r / (nx * (ny + 1));
                    const long b = (k / 2) * (cy + 1) * cx + i / 2;
                    out = (j & 1) ? 0.5 * (g[b + (j / 2) * cx] + g[b + (j / 2 + 1) * cx]) : g[b + (j / 2) * cx];
                } else if (c == 2) {  // fine w of [nz+1][ny][nx]
                    const long i = r % nx, j = (r / nx) % ny, k = r / (nx * ny);
                    const long b = (j / 2) * cx + i / 2, pl = cy * cx;
                    out = (k & 1) ? 0.5 * (g[b + (k / 2) * pl] + g[b + (k / 2 + 1) * pl]) : g[b + (k / 2) * pl];
                } else {
                    const long i = r % nx, j = (r / nx) % ny, k = r / (nx * ny);
                    out = g[((k / 2) * cy + j / 2) * cx + i / 2];
                }
                dst[e] = out;
            }
        }
    }
}

// Eq. (6) on the segments: y <- f + (g - gold), gold <- g, and the max of
// |y_new - y_old| per jump slot.  The max is taken over the block (wave
// shuffles, then LDS) and only then merged into the slot with one 64-bit
// atomic max of the non-negative bit pattern per block and slot (segments of
// one slot are consecutive), so a launch issues a few hundred atomics, not
// one per wave; the max does not depend on the order.
__global__ void __launch_bounds__(kBlock) k_parareal_update(UpdateParams U) {
    __shared__ double s_m[kWaves];
    double m = 0.0;
    for (int si = 0; si < U.nseg; ++si) {
        const UpdateSeg &S = U.seg[si];
        for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < S.n;
             x += (long long)gridDim.x * blockDim.x) {
            const double g = S.g[x];
            const double y = S.f[x] + (g - S.gold[x]);
            const double d = fabs(y - S.y[x]);
            m = (d > m || d != d) ? d : m;
            S.y[x] = y;
            S.gold[x] = g;
        }
        const bool flush = si + 1 == U.nseg || U.group_of_seg[si + 1] != U.group_of_seg[si] ||
                           U.seg[si + 1].jslot != S.jslot;
        if (!flush) continue;
        for (int o = 32; o >= 1; o >>= 1) {
            const double t = __shfl_xor(m, o, 64);
            m = (t > m || t != t) ? t : m;
        }
        if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            double mm = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mm = (s_m[w] > mm || s_m[w] != s_m[w]) ? s_m[w] : mm;
            if (mm != 0.0) {
                const unsigned long long bits = __double_as_longlong(mm);
                const int slot = 2 * U.group_of_seg[si] + S.jslot;
                __hip_atomic_fetch_max(&U.jump[slot], bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
        m = 0.0;
    }
}

__global__ void k_copy(double *__restrict__ dst, const double *__restrict__ src, long long n) {
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (long long)gridDim.x * blockDim.x)
        dst[x] = src[x];
}

}  // namespace

hipError_t launch_persistent(const KParams *P_dev, int workgroups, bool rr, hipStream_t stream) {
    const KParams *arg = P_dev;
    void *args[] = {&arg};
    const void *fn = rr ? reinterpret_cast<const void *>(&k_persistent<true>)
                        : reinterpret_cast<const void *>(&k_persistent<false>);
    return hipLaunchCooperativeKernel(fn, dim3(workgroups), dim3(kBlock), args, 0, stream);
}

hipError_t max_coresident_workgroups(int device, int *out) {
    int per_cu = 0, per_cu_rr = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(&k_persistent<false>), kBlock, 0);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_rr, reinterpret_cast<const void *>(&k_persistent<true>),
                                                     kBlock, 0);
    if (e != hipSuccess) return e;
    per_cu = per_cu < per_cu_rr ? per_cu : per_cu_rr;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return e;
    *out = per_cu * prop.multiProcessorCount;
    return hipSuccess;
}

hipError_t launch_zero_words(void *p, long long nwords, hipStream_t stream) {
    if (nwords <= 0) return hipSuccess;
    long long blocks = (nwords + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(256), 0, stream, reinterpret_cast<unsigned *>(p),
                       nwords);
    return hipGetLastError();
}

hipError_t launch_reset_sync(SyncWords *s, hipStream_t stream) {
    return launch_zero_words(s, (long long)(sizeof(SyncWords) / sizeof(unsigned)), stream);
}

hipError_t add_persistent_graph_nodes(hipGraph_t graph, const KParams *P_dev, int workgroups, bool rr,
                                      SliceCtl *ctl, int nslices, SyncWords *sync, GraphFold *fold) {
    if (nslices <= 0 || nslices > kMaxSlices) return hipErrorInvalidValue;
    // node 1: zero the control blocks; node 2: reset the barrier words
    unsigned *cw = reinterpret_cast<unsigned *>(ctl);
    long long cn = (long long)nslices * (long long)(sizeof(SliceCtl) / sizeof(unsigned));
    unsigned *sw = reinterpret_cast<unsigned *>(sync);
    long long sn = (long long)(sizeof(SyncWords) / sizeof(unsigned));
    void *a1[] = {&cw, &cn};
    void *a2[] = {&sw, &sn};
    hipKernelNodeParams k1{}, k2{}, k3{}, k4{};
    k1.func = reinterpret_cast<void *>(&k_zero_words);
    k1.gridDim = dim3((unsigned)((cn + 255) / 256));
    k1.blockDim = dim3(256);
    k1.kernelParams = a1;
    k2.func = reinterpret_cast<void *>(&k_zero_words);
    k2.gridDim = dim3((unsigned)((sn + 255) / 256 > 1024 ? 1024 : (sn + 255) / 256));
    k2.blockDim = dim3(256);
    k2.kernelParams = a2;
    // node 3: the persistent kernel, a cooperative launch
    const KParams *arg = P_dev;
    void *a3[] = {&arg};
    k3.func = rr ? reinterpret_cast<void *>(&k_persistent<true>) : reinterpret_cast<void *>(&k_persistent<false>);
    k3.gridDim = dim3((unsigned)workgroups);
    k3.blockDim = dim3(kBlock);
    k3.kernelParams = a3;
    // node 4: fold this replay's slice results and the abort flag into what
    // the graph keeps across replays
    const SliceCtl *cc = ctl;
    const SyncWords *sc = sync;
    int ns = nslices;
    void *a4[] = {&cc, &sc, &ns, &fold};
    k4.func = reinterpret_cast<void *>(&k_fold_status);
    k4.gridDim = dim3(1);
    k4.blockDim = dim3(64);
    k4.kernelParams = a4;
    hipGraphNode_t n1, n2, n3, n4;
    hipError_t e = hipGraphAddKernelNode(&n1, graph, nullptr, 0, &k1);
    if (e != hipSuccess) return e;
    if ((e = hipGraphAddKernelNode(&n2, graph, &n1, 1, &k2)) != hipSuccess) return e;
    if ((e = hipGraphAddKernelNode(&n3, graph, &n2, 1, &k3)) != hipSuccess) return e;
    hipKernelNodeAttrValue coop{};
    coop.cooperative = 1;
    if ((e = hipGraphKernelNodeSetAttribute(n3, hipKernelNodeAttributeCooperative, &coop)) != hipSuccess) return e;
    return hipGraphAddKernelNode(&n4, graph, &n3, 1, &k4);
}

hipError_t launch_parareal_update(const UpdateParams &U, hipStream_t stream) {
    long long nmax = 0;
    for (int i = 0; i < U.nseg; ++i) nmax = U.seg[i].n > nmax ? U.seg[i].n : nmax;
    // two 1024-thread blocks per CU stream the arrays at full rate
    long long blocks = (nmax + kBlock - 1) / kBlock;
    if (blocks > 512) blocks = 512;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_parareal_update, dim3((unsigned)blocks), dim3(kBlock), 0, stream, U);
    return hipGetLastError();
}

hipError_t launch_transfer(const TransferParams &T, hipStream_t stream) {
    const long long n = (long long)(T.nx + 1) * (T.ny + 1) * (T.nz + 1) * T.batch;
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_transfer, dim3((unsigned)blocks), dim3(256), 0, stream, T);
    return hipGetLastError();
}

hipError_t launch_copy_state(double *dst, const double *src, long long n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, stream, dst, src, n);
    return hipGetLastError();
}

}  // namespace nsp
