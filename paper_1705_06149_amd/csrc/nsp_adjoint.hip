// gfx950 kernels for the adjoint of the fine step, the kinetic-energy
// objective and the lid sine basis.
//
// One forward step is u' = P(M(u)), M(u) = u + dt R(u) on open faces, R the
// momentum right-hand side (central diffusion, SMART convection, image rule
// at walls and obstacles, lid on the top face), P the orthogonal projector
// onto discretely divergence-free fields (Chorin-Temam projection, Sec. 2 of
// Croce, Ruprecht & Krause).  Its adjoint: mu = P lam' (P symmetric; done by
// the persistent kernel in projection mode), then
//     lam = mu + dt (dR/du)^T mu,   g_lid += dt (dR/dlid)^T mu,
// which k_mom_adjoint computes by scattering each open face's local
// Jacobian-transpose contributions with FP64 atomic adds.  SMART is
// piecewise linear in (U, C, D): the adjoint uses the slopes of the branch
// the forward step took; a zero transport velocity gives a zero flux and no
// contribution.
#include "nsp_internal.h"

namespace nsp {

namespace {

// A stencil value as a linear form in face values of one component plus a
// multiple of one lid value.
struct Form {
    int n;
    long idx[4];
    double coef[4];
    double lcoef;
    long lidx;
};

struct AdjGrid {
    int nx, ny, nz;
    double ih[3], ih2[3];
    double inv_re, dt;
    const uint8_t *flags;
    const double *lid;
};

__device__ __forceinline__ int ext(const AdjGrid &G, int c, int d) {
    const int n = d == 0 ? G.nx : (d == 1 ? G.ny : G.nz);
    return n + (c == d ? 1 : 0);
}

__device__ __forceinline__ long face_index(const AdjGrid &G, int c, const int p[3]) {
    return ((long)p[2] * ext(G, c, 1) + p[1]) * ext(G, c, 0) + p[0];
}

// open face of component c at p: both adjacent cells fluid (the cell's own
// "minus" open bit); outside the array or on the high boundary: closed
__device__ __forceinline__ bool open_face(const AdjGrid &G, int c, const int p[3]) {
    if (p[0] < 0 || p[1] < 0 || p[2] < 0 || p[0] >= G.nx || p[1] >= G.ny || p[2] >= G.nz) return false;
    const uint8_t bit = c == 0 ? FL_XM : (c == 1 ? FL_YM : FL_ZM);
    return (G.flags[((long)p[2] * G.ny + p[1]) * G.nx + p[0]] & bit) != 0;
}

__device__ __forceinline__ bool lid_wall(const AdjGrid &G, int c, const int p[3], int d, int s) {
    return c == 0 && d == 1 && s > 0 && p[1] == G.ny - 1;
}

__device__ __forceinline__ void add_term(Form &F, long idx, double coef) {
    F.idx[F.n] = idx;
    F.coef[F.n] = coef;
    ++F.n;
}

// value at offset +-1 (one = true) or +-2 along d, sense s, of the stencil
// of open face f: own axis -> closed face 0, next position -phi0; across ->
// wall half a cell away, image 2*wall - mirror (mirror resolved first)
__device__ void form_of(const AdjGrid &G, int c, const int f[3], int d, int s, bool one, Form &F) {
    int f1[3] = {f[0], f[1], f[2]}, f2[3] = {f[0], f[1], f[2]};
    f1[d] += s;
    f2[d] += 2 * s;
    const long i0 = face_index(G, c, f);
    F.n = 0;
    F.lcoef = 0.0;
    F.lidx = (long)f[2] * (G.nx + 1) + f[0];
    const bool o1 = open_face(G, c, f1);
    if (c == d) {
        if (!o1) { if (!one) add_term(F, i0, -1.0); return; }
        if (one) { add_term(F, face_index(G, c, f1), 1.0); return; }
        if (open_face(G, c, f2)) add_term(F, face_index(G, c, f2), 1.0);
        return;
    }
    if (!o1) {
        if (lid_wall(G, c, f, d, s)) F.lcoef += 2.0;
        if (one) { add_term(F, i0, -1.0); return; }
        // 2 wall - (value at offset 1 on the other side)
        int g1[3] = {f[0], f[1], f[2]};
        g1[d] -= s;
        if (open_face(G, c, g1)) {
            add_term(F, face_index(G, c, g1), -1.0);
        } else {
            if (lid_wall(G, c, f, d, -s)) F.lcoef -= 2.0;
            add_term(F, i0, 1.0);
        }
        return;
    }
    if (one) { add_term(F, face_index(G, c, f1), 1.0); return; }
    if (!open_face(G, c, f2)) {
        if (lid_wall(G, c, f1, d, s)) F.lcoef += 2.0;
        add_term(F, face_index(G, c, f1), -1.0);
        return;
    }
    add_term(F, face_index(G, c, f2), 1.0);
}

__device__ __forceinline__ double form_value(const Form &F, const double *phi, const double *lid) {
    double v = 0.0;
    for (int q = 0; q < F.n; ++q) v += F.coef[q] * phi[F.idx[q]];
    return v + F.lcoef * lid[F.lidx];
}

__device__ __forceinline__ void scatter(const Form &F, double wgt, double *lam, double *glid) {
    for (int q = 0; q < F.n; ++q) atomicAdd(&lam[F.idx[q]], wgt * F.coef[q]);
    if (F.lcoef != 0.0) atomicAdd(&glid[F.lidx], wgt * F.lcoef);
}

// SMART face value and its slopes with respect to U, C, D on the branch taken
__device__ __forceinline__ double smart_and_slopes(double U, double C, double D, double s[3]) {
    const double delta = D - U;
    s[0] = 0.0; s[1] = 1.0; s[2] = 0.0;
    if (delta == 0.0) return C;
    const double ph = (C - U) / delta;
    double pf;
    if (ph > 0.0 && ph < 1.0 / 6.0) { pf = 3.0 * ph; s[0] = -2.0; s[1] = 3.0; }
    else if (ph >= 1.0 / 6.0 && ph < 5.0 / 6.0) { pf = 0.75 * ph + 0.375; s[0] = -0.125; s[1] = 0.75; s[2] = 0.375; }
    else if (ph >= 5.0 / 6.0 && ph < 1.0) { pf = 1.0; s[1] = 0.0; s[2] = 1.0; }
    else pf = ph;
    return U + pf * delta;
}

// lam = masked mu (closed faces 0); one thread per face of component c
__global__ void k_adj_init(AdjGrid G, int c, const double *__restrict__ mu, double *__restrict__ lam, long n) {
    for (long x = (long)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (long)gridDim.x * blockDim.x) {
        const int e0 = ext(G, c, 0), e1 = ext(G, c, 1);
        const int p[3] = {(int)(x % e0), (int)((x / e0) % e1), (int)(x / ((long)e0 * e1))};
        lam[x] = open_face(G, c, p) ? mu[x] : 0.0;
    }
}

// dt (dR/du)^T mu and dt (dR/dlid)^T mu for the open faces of component c
__global__ void k_mom_adjoint(AdjGrid G, int c, const double *__restrict__ u, const double *__restrict__ v,
                              const double *__restrict__ w, const double *__restrict__ muc, double *lu, double *lv,
                              double *lw, double *glid, long n) {
    const double *vel[3] = {u, v, w};
    double *lam[3] = {lu, lv, lw};
    for (long x = (long)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (long)gridDim.x * blockDim.x) {
        const int e0 = ext(G, c, 0), e1 = ext(G, c, 1);
        const int f[3] = {(int)(x % e0), (int)((x / e0) % e1), (int)(x / ((long)e0 * e1))};
        if (!open_face(G, c, f)) continue;
        const double m0 = muc[x];
        if (m0 == 0.0) continue;
        const double *phi = vel[c];
        for (int d = 0; d < 3; ++d) {
            Form Vm2, Vm1, Vp1, Vp2, Self;
            form_of(G, c, f, d, -1, false, Vm2);
            form_of(G, c, f, d, -1, true, Vm1);
            form_of(G, c, f, d, +1, true, Vp1);
            form_of(G, c, f, d, +1, false, Vp2);
            Self.n = 0;
            Self.lcoef = 0.0;
            Self.lidx = 0;
            add_term(Self, x, 1.0);
            // diffusion
            const double wd = G.dt * m0 * G.inv_re * G.ih2[d];
            scatter(Vp1, wd, lam[c], glid);
            scatter(Vm1, wd, lam[c], glid);
            atomicAdd(&lam[c][x], -2.0 * wd);
            // convection: -(flux(+) - flux(-)) / h
            for (int s = -1; s <= 1; s += 2) {
                int ac;
                long ai[2];
                bool ao[2];
                if (d == c) {
                    int f1[3] = {f[0], f[1], f[2]};
                    f1[d] += s;
                    ac = c;
                    ai[0] = x;
                    ao[0] = true;
                    ao[1] = open_face(G, c, f1);
                    ai[1] = ao[1] ? face_index(G, c, f1) : 0;
                } else {
                    int q1[3] = {f[0], f[1], f[2]}, q2[3] = {f[0], f[1], f[2]};
                    if (s > 0) { q1[d] += 1; q2[d] += 1; }
                    q1[c] -= 1;
                    ac = d;
                    ao[0] = open_face(G, d, q1);
                    ao[1] = open_face(G, d, q2);
                    ai[0] = ao[0] ? face_index(G, d, q1) : 0;
                    ai[1] = ao[1] ? face_index(G, d, q2) : 0;
                }
                const double a1 = ao[0] ? vel[ac][ai[0]] : 0.0;
                const double a2 = ao[1] ? vel[ac][ai[1]] : 0.0;
                const double abar = 0.5 * (a1 + a2);
                if (abar == 0.0) continue;
                const Form *U, *C, *D;
                if (s > 0) {
                    if (abar > 0.0) { U = &Vm1; C = &Self; D = &Vp1; }
                    else { U = &Vp2; C = &Vp1; D = &Self; }
                } else {
                    if (abar > 0.0) { U = &Vm2; C = &Vm1; D = &Self; }
                    else { U = &Vp1; C = &Self; D = &Vm1; }
                }
                double sl[3];
                const double phis = smart_and_slopes(form_value(*U, phi, G.lid), form_value(*C, phi, G.lid),
                                                     form_value(*D, phi, G.lid), sl);
                const double wc = -(double)s * G.dt * m0 * G.ih[d];
                if (ao[0]) atomicAdd(&lam[ac][ai[0]], wc * 0.5 * phis);
                if (ao[1]) atomicAdd(&lam[ac][ai[1]], wc * 0.5 * phis);
                scatter(*U, wc * abar * sl[0], lam[c], glid);
                scatter(*C, wc * abar * sl[1], lam[c], glid);
                scatter(*D, wc * abar * sl[2], lam[c], glid);
            }
        }
    }
}

// out = scale * a on open faces of component c, 0 on closed faces
__global__ void k_scale_open(AdjGrid G, int c, const double *__restrict__ a, double scale, double *__restrict__ out,
                             long n) {
    for (long x = (long)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (long)gridDim.x * blockDim.x) {
        const int e0 = ext(G, c, 0), e1 = ext(G, c, 1);
        const int p[3] = {(int)(x % e0), (int)((x / e0) % e1), (int)(x / ((long)e0 * e1))};
        out[x] = open_face(G, c, p) ? scale * a[x] : 0.0;
    }
}

// per-block sums of squares over open faces (fixed order: grid-stride
// per thread, wave butterfly, fixed four-wave combine)
__global__ void k_sumsq_open(AdjGrid G, int c, const double *__restrict__ a, long n, double *__restrict__ part) {
    __shared__ double s[4];
    double acc = 0.0;
    for (long x = (long)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (long)gridDim.x * blockDim.x) {
        const int e0 = ext(G, c, 0), e1 = ext(G, c, 1);
        const int p[3] = {(int)(x % e0), (int)((x / e0) % e1), (int)(x / ((long)e0 * e1))};
        if (open_face(G, c, p)) acc += a[x] * a[x];
    }
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
}

__global__ void k_sum_parts(const double *__restrict__ part, int n, double *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        *out = s;
    }
}

// lid(i,k) = 1 + sum_{m,n} coef[m][n] sin(m pi x_i/lx) sin(n pi z_k/lz),
// x_i = i hx, z_k = (k + 1/2) hz; coef is M x M, modes 1..M
__global__ void k_lid_synth(int nx, int nz, double hx, double hz, double lx, double lz, const double *__restrict__ coef,
                            int M, double *__restrict__ lid) {
    const long n = (long)nz * (nx + 1);
    for (long x = (long)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (long)gridDim.x * blockDim.x) {
        const int i = (int)(x % (nx + 1)), k = (int)(x / (nx + 1));
        const double X = i * hx, Z = (k + 0.5) * hz;
        double v = 1.0;
        for (int a = 0; a < M; ++a) {
            const double sx = sin(M_PI * (a + 1) * X / lx);
            for (int b = 0; b < M; ++b) v += coef[a * M + b] * sx * sin(M_PI * (b + 1) * Z / lz);
        }
        lid[x] = v;
    }
}

// g_coef[m][n] = sum_{k,i} g_lid(i,k) sin(m pi x_i/lx) sin(n pi z_k/lz), fixed order
__global__ void k_lid_project(int nx, int nz, double hx, double hz, double lx, double lz,
                              const double *__restrict__ glid, int M, double *__restrict__ gcoef) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * M) return;
    const int a = t / M, b = t % M;
    double s = 0.0;
    for (int k = 0; k < nz; ++k) {
        const double sz = sin(M_PI * (b + 1) * (k + 0.5) * hz / lz);
        for (int i = 0; i <= nx; ++i) s += glid[(long)k * (nx + 1) + i] * sin(M_PI * (a + 1) * i * hx / lx) * sz;
    }
    gcoef[t] = s;
}

unsigned blocks_for(long n) {
    long b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    return (unsigned)(b < 1 ? 1 : b);
}

AdjGrid adj_grid(const AdjParams &A) {
    AdjGrid G;
    G.nx = A.nx;
    G.ny = A.ny;
    G.nz = A.nz;
    for (int d = 0; d < 3; ++d) {
        G.ih[d] = A.ih[d];
        G.ih2[d] = A.ih2[d];
    }
    G.inv_re = A.inv_re;
    G.dt = A.dt;
    G.flags = A.flags;
    G.lid = A.lid;
    return G;
}

}  // namespace

hipError_t launch_momentum_adjoint(const AdjParams &A, const double *const vel[3], const double *const mu[3],
                                   double *const lam[3], double *glid, hipStream_t s) {
    const AdjGrid G = adj_grid(A);
    const long nf[3] = {(long)(A.nx + 1) * A.ny * A.nz, (long)A.nx * (A.ny + 1) * A.nz, (long)A.nx * A.ny * (A.nz + 1)};
    for (int c = 0; c < 3; ++c)
        hipLaunchKernelGGL(k_adj_init, dim3(blocks_for(nf[c])), dim3(256), 0, s, G, c, mu[c], lam[c], nf[c]);
    for (int c = 0; c < 3; ++c)
        hipLaunchKernelGGL(k_mom_adjoint, dim3(blocks_for(nf[c])), dim3(256), 0, s, G, c, vel[0], vel[1], vel[2],
                           mu[c], lam[0], lam[1], lam[2], glid, nf[c]);
    return hipGetLastError();
}

hipError_t launch_scale_open(const AdjParams &A, const double *const a[3], double scale, double *const out[3],
                             hipStream_t s) {
    const AdjGrid G = adj_grid(A);
    const long nf[3] = {(long)(A.nx + 1) * A.ny * A.nz, (long)A.nx * (A.ny + 1) * A.nz, (long)A.nx * A.ny * (A.nz + 1)};
    for (int c = 0; c < 3; ++c)
        hipLaunchKernelGGL(k_scale_open, dim3(blocks_for(nf[c])), dim3(256), 0, s, G, c, a[c], scale, out[c], nf[c]);
    return hipGetLastError();
}

// sum of squares of (u, v, w) over open faces into out[0] (device); part
// needs 3 * kSumBlocks doubles
hipError_t launch_sumsq_open(const AdjParams &A, const double *const a[3], double *part, double *out, hipStream_t s) {
    const AdjGrid G = adj_grid(A);
    const long nf[3] = {(long)(A.nx + 1) * A.ny * A.nz, (long)A.nx * (A.ny + 1) * A.nz, (long)A.nx * A.ny * (A.nz + 1)};
    for (int c = 0; c < 3; ++c)
        hipLaunchKernelGGL(k_sumsq_open, dim3(kSumBlocks), dim3(256), 0, s, G, c, a[c], nf[c], part + c * kSumBlocks);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, part, 3 * kSumBlocks, out);
    return hipGetLastError();
}

hipError_t launch_lid_synth(const AdjParams &A, const double *coef, int M, double *lid, hipStream_t s) {
    const long n = (long)A.nz * (A.nx + 1);
    hipLaunchKernelGGL(k_lid_synth, dim3(blocks_for(n)), dim3(256), 0, s, A.nx, A.nz, A.h[0], A.h[2], A.L[0], A.L[2],
                       coef, M, lid);
    return hipGetLastError();
}

hipError_t launch_lid_project(const AdjParams &A, const double *glid, int M, double *gcoef, hipStream_t s) {
    hipLaunchKernelGGL(k_lid_project, dim3((M * M + 63) / 64), dim3(64), 0, s, A.nx, A.nz, A.h[0], A.h[2], A.L[0],
                       A.L[2], glid, M, gcoef);
    return hipGetLastError();
}

}  // namespace nsp
