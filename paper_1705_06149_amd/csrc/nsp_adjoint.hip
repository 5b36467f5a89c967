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
// which k_mom_adjoint gathers face by face: every face sums, in a fixed
// order, the transposed contributions of the interfaces whose fluxes read
// it, so the result has no atomics and repeats bitwise.  SMART is piecewise
// linear in (U, C, D): the adjoint uses the slopes of the branch the forward
// step took; a zero transport velocity gives a zero flux and no
// contribution.
#include "nsp_internal.h"

namespace nsp {

namespace {

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

// open face of component c at (i,j,k): both adjacent cells fluid (the
// cell's own "minus" open bit); outside the array or on the high boundary:
// closed
__device__ __forceinline__ bool open_face(const AdjGrid &G, int c, int i, int j, int k) {
    if (i < 0 || j < 0 || k < 0 || i >= G.nx || j >= G.ny || k >= G.nz) return false;
    const uint8_t bit = c == 0 ? FL_XM : (c == 1 ? FL_YM : FL_ZM);
    return (G.flags[((long)k * G.ny + j) * G.nx + i] & bit) != 0;
}

template <int C>
__device__ __forceinline__ long fid(const AdjGrid &G, int i, int j, int k) {
    return ((long)k * ext(G, C, 1) + j) * ext(G, C, 0) + i;
}

// distance in the array of component C between neighbours along D
template <int C, int D>
__device__ __forceinline__ long fstride(const AdjGrid &G) {
    return D == 0 ? 1 : (D == 1 ? (long)ext(G, C, 0) : (long)ext(G, C, 0) * ext(G, C, 1));
}

// ------------------------------------------------------------ interfaces
//
// The momentum right-hand side of an open face is a sum over the six
// interfaces around it (one per side and direction) of a diffusive flux
// (the difference of the two values across the interface) and a convective
// flux (transport velocity times the SMART value upwind of the
// interface).  Between two open faces both of them see the same flux, with
// the same image values, so the step is conservative and its transpose can
// be taken interface by interface:
//     R(L) += nu/h^2 Delta - Phi/h,   R(L + e) += -nu/h^2 Delta + Phi/h
// for the interface between face L of a component and the next face L + e
// along a direction.  An interface with only one open side enters that
// side alone.  Its values at L - e, L, L + e, L + 2e, after the image rule
// (a closed face of the component's own axis holds 0 and the next position
// its odd reflection; across, a closed neighbour is a wall half a cell away
// with image 2 wall - mirror; the lid is the wall above the top row of u),
// are X[0..3]; Delta = X2 - X1; Phi = a (a > 0: SMART(X0, X1, X2), else
// SMART(X3, X2, X1)), a the mean of the two faces of the transport component
// that straddle the interface (own axis: of X1 and X2).

struct Line {
    bool oL, oU, om, o2;   // open: L, L + e, L - e, L + 2e
    bool lidL, lidU;       // the lid is the wall above L / above L + e
    double X[4];
};

// image-resolved values of the line of interface (C, D, L = (i,j,k));
// false when neither L nor L + e is open
template <int C, int D>
__device__ __forceinline__ bool line_of(const AdjGrid &G, const double *__restrict__ phi, int i, int j, int k,
                                        Line &Ln) {
    constexpr int di = D == 0, dj = D == 1, dk = D == 2;
    Ln.oL = open_face(G, C, i, j, k);
    Ln.oU = open_face(G, C, i + di, j + dj, k + dk);
    if (!Ln.oL && !Ln.oU) return false;
    Ln.om = open_face(G, C, i - di, j - dj, k - dk);
    Ln.o2 = open_face(G, C, i + 2 * di, j + 2 * dj, k + 2 * dk);
    Ln.lidL = C == 0 && D == 1 && j == G.ny - 1;
    Ln.lidU = C == 0 && D == 1 && j + 1 == G.ny - 1;
    const double lv = (Ln.lidL || Ln.lidU) ? G.lid[(long)k * (G.nx + 1) + i] : 0.0;
    const double wL = Ln.lidL ? lv : 0.0, wU = Ln.lidU ? lv : 0.0;
    const long id = fid<C>(G, i, j, k), s = fstride<C, D>(G);
    if (Ln.oL) {
        const double P0 = phi[id];
        Ln.X[1] = P0;
        if (C == D) {
            Ln.X[0] = Ln.om ? phi[id - s] : 0.0;
            Ln.X[2] = Ln.oU ? phi[id + s] : 0.0;
            Ln.X[3] = !Ln.oU ? -P0 : (Ln.o2 ? phi[id + 2 * s] : 0.0);
        } else {
            Ln.X[0] = Ln.om ? phi[id - s] : 2.0 * 0.0 - P0;
            Ln.X[2] = Ln.oU ? phi[id + s] : 2.0 * wL - P0;
            Ln.X[3] = !Ln.oU ? 2.0 * wL - Ln.X[0] : (Ln.o2 ? phi[id + 2 * s] : 2.0 * wU - Ln.X[2]);
        }
    } else {
        const double P1 = phi[id + s];
        Ln.X[2] = P1;
        if (C == D) {
            Ln.X[1] = 0.0;
            Ln.X[0] = -P1;
            Ln.X[3] = Ln.o2 ? phi[id + 2 * s] : 0.0;
        } else {
            Ln.X[1] = 2.0 * 0.0 - P1;
            Ln.X[3] = Ln.o2 ? phi[id + 2 * s] : 2.0 * wU - P1;
            Ln.X[0] = 2.0 * 0.0 - Ln.X[3];
        }
    }
    return true;
}

// derivatives of X[0..3] with respect to the value at position L + (POS-1) e
// (cx) and to the lid beside L (lx)
template <int C, int D, int POS>
__device__ __forceinline__ void coefs_of(const Line &Ln, double cx[4], double lx[4]) {
    const double p0 = POS == 0, p1 = POS == 1, p2 = POS == 2, p3 = POS == 3;
    lx[0] = lx[1] = lx[2] = lx[3] = 0.0;
    if (Ln.oL) {
        cx[1] = p1;
        if (C == D) {
            cx[0] = Ln.om ? p0 : 0.0;
            cx[2] = Ln.oU ? p2 : 0.0;
            cx[3] = !Ln.oU ? -p1 : (Ln.o2 ? p3 : 0.0);
        } else {
            cx[0] = Ln.om ? p0 : -p1;
            cx[2] = Ln.oU ? p2 : -p1;
            cx[3] = !Ln.oU ? -cx[0] : (Ln.o2 ? p3 : -cx[2]);
            lx[2] = (!Ln.oU && Ln.lidL) ? 2.0 : 0.0;
            lx[3] = !Ln.oU ? (Ln.lidL ? 2.0 : 0.0) : ((!Ln.o2 && Ln.lidU) ? 2.0 : 0.0);
        }
    } else {
        cx[2] = p2;
        if (C == D) {
            cx[1] = 0.0;
            cx[0] = -p2;
            cx[3] = Ln.o2 ? p3 : 0.0;
        } else {
            cx[1] = -p2;
            cx[3] = Ln.o2 ? p3 : -p2;
            cx[0] = -cx[3];
            lx[3] = (!Ln.o2 && Ln.lidU) ? 2.0 : 0.0;
            lx[0] = -lx[3];
        }
    }
}

// value of the transport component D at its face (i,j,k); closed: 0
template <int D>
__device__ __forceinline__ double real_face(const AdjGrid &G, const double *__restrict__ a, int i, int j, int k) {
    return open_face(G, D, i, j, k) ? a[fid<D>(G, i, j, k)] : 0.0;
}

// SMART (normalised variable, Gaskell & Lau) face value of the upwind
// triple (U, C, D) and its slopes on the branch taken
__device__ __forceinline__ double smart_slopes(double U, double C, double D, double &sU, double &sC, double &sD) {
    const double delta = D - U;
    sU = 0.0; sC = 1.0; sD = 0.0;
    if (delta == 0.0) return C;
    const double ph = (C - U) / delta;
    double pf;
    if (ph > 0.0 && ph < 1.0 / 6.0) { pf = 3.0 * ph; sU = -2.0; sC = 3.0; }
    else if (ph >= 1.0 / 6.0 && ph < 5.0 / 6.0) { pf = 0.75 * ph + 0.375; sU = -0.125; sC = 0.75; sD = 0.375; }
    else if (ph >= 5.0 / 6.0 && ph < 1.0) { pf = 1.0; sC = 0.0; sD = 1.0; }
    else pf = ph;
    return U + pf * delta;
}

// The linearised fluxes of interface (C, D, L = (i,j,k)) with their adjoint
// weights: wphi = dt/h (mu(L+e) - mu(L)), wdel = dt nu/h^2 (mu(L) - mu(L+e)),
// closed faces taking mu = 0.
struct Flux {
    double wphi, wdel;
    double a;              // transport velocity
    double S, sU, sC, sD;  // SMART value and slopes (a != 0)
};

template <int C, int D>
__device__ __forceinline__ bool flux_of(const AdjGrid &G, const double *const *vel, const double *const *mu, int i,
                                        int j, int k, Line &Ln, Flux &Fx) {
    constexpr int di = D == 0, dj = D == 1, dk = D == 2;
    constexpr int ci = C == 0, cj = C == 1, ck = C == 2;
    if (!line_of<C, D>(G, vel[C], i, j, k, Ln)) return false;
    const long id = fid<C>(G, i, j, k), s = fstride<C, D>(G);
    const double mL = Ln.oL ? mu[C][id] : 0.0, mU = Ln.oU ? mu[C][id + s] : 0.0;
    if (mL == mU) return false;  // both weights vanish
    Fx.wphi = G.dt * G.ih[D] * (mU - mL);
    Fx.wdel = G.dt * G.inv_re * G.ih2[D] * (mL - mU);
    if (C == D) Fx.a = 0.5 * (Ln.X[1] + Ln.X[2]);
    else
        Fx.a = 0.5 * (real_face<D>(G, vel[D], i - ci + di, j - cj + dj, k - ck + dk) +
                      real_face<D>(G, vel[D], i + di, j + dj, k + dk));
    Fx.S = 0.0;
    if (Fx.a > 0.0) Fx.S = smart_slopes(Ln.X[0], Ln.X[1], Ln.X[2], Fx.sU, Fx.sC, Fx.sD);
    else if (Fx.a < 0.0) Fx.S = smart_slopes(Ln.X[3], Ln.X[2], Ln.X[1], Fx.sU, Fx.sC, Fx.sD);
    return true;
}

// transposed contribution of interface (C, D, L) to the value of component
// C at L + (POS-1) e; with LID also its contribution to the lid beside L
template <int C, int D, int POS, bool LID>
__device__ __forceinline__ double line_adj(const AdjGrid &G, const double *const *vel, const double *const *mu, int i,
                                           int j, int k, double &glid) {
    Line Ln;
    Flux Fx;
    if (!flux_of<C, D>(G, vel, mu, i, j, k, Ln, Fx)) return 0.0;
    double cx[4], lx[4];
    coefs_of<C, D, POS>(Ln, cx, lx);
    double r = Fx.wdel * (cx[2] - cx[1]);
    if (LID) glid += Fx.wdel * (lx[2] - lx[1]);
    if (Fx.a != 0.0) {
        const double wa = Fx.wphi * Fx.a;
        if (Fx.a > 0.0) {
            r += wa * ((Fx.sU * cx[0] + Fx.sC * cx[1]) + Fx.sD * cx[2]);
            if (LID) glid += wa * ((Fx.sU * lx[0] + Fx.sC * lx[1]) + Fx.sD * lx[2]);
        } else {
            r += wa * ((Fx.sU * cx[3] + Fx.sC * cx[2]) + Fx.sD * cx[1]);
            if (LID) glid += wa * ((Fx.sU * lx[3] + Fx.sC * lx[2]) + Fx.sD * lx[1]);
        }
        if (C == D) r += Fx.wphi * 0.5 * Fx.S * (cx[1] + cx[2]);
    }
    return r;
}

// transposed contribution of interface (C, D, L), C != D, to one of the two
// faces of component D that carry its transport velocity
template <int C, int D>
__device__ __forceinline__ double transport_adj(const AdjGrid &G, const double *const *vel, const double *const *mu,
                                                int i, int j, int k) {
    Line Ln;
    Flux Fx;
    if (!flux_of<C, D>(G, vel, mu, i, j, k, Ln, Fx)) return 0.0;
    return Fx.a != 0.0 ? Fx.wphi * 0.5 * Fx.S : 0.0;
}

// the four interfaces along D whose lines hold the face t = (i,j,k) of
// component C: L = t - 2e .. t + e (t at position 3 .. 0 of their lines)
template <int C, int D, bool LID>
__device__ __forceinline__ double along(const AdjGrid &G, const double *const *vel, const double *const *mu, int i,
                                        int j, int k, double &glid) {
    constexpr int di = D == 0, dj = D == 1, dk = D == 2;
    double r = line_adj<C, D, 3, false>(G, vel, mu, i - 2 * di, j - 2 * dj, k - 2 * dk, glid);
    r += line_adj<C, D, 2, LID>(G, vel, mu, i - di, j - dj, k - dk, glid);
    r += line_adj<C, D, 1, LID>(G, vel, mu, i, j, k, glid);
    r += line_adj<C, D, 0, false>(G, vel, mu, i + di, j + dj, k + dk, glid);
    return r;
}

// the interfaces of component C along T whose transport velocity averages
// the face t = (i,j,k) of component T: L = t - e_T and t - e_T + e_C
template <int C, int T>
__device__ __forceinline__ double carried(const AdjGrid &G, const double *const *vel, const double *const *mu, int i,
                                          int j, int k) {
    constexpr int ti = T == 0, tj = T == 1, tk = T == 2;
    constexpr int ci = C == 0, cj = C == 1, ck = C == 2;
    return transport_adj<C, T>(G, vel, mu, i - ti, j - tj, k - tk) +
           transport_adj<C, T>(G, vel, mu, i - ti + ci, j - tj + cj, k - tk + ck);
}

// lam = mu + dt (dR/du)^T mu at face x of component T, gathered in a fixed
// order; for the top row of u also g_lid += dt (dR/dlid)^T mu beside it
template <int T>
__device__ __forceinline__ void gather_face(const AdjGrid &G, const double *const *vel, const double *const *mu,
                                            double *__restrict__ lam, double *__restrict__ glid, long x) {
    const int e0 = ext(G, T, 0), e1 = ext(G, T, 1);
    const int i = (int)(x % e0), j = (int)((x / e0) % e1), k = (int)(x / ((long)e0 * e1));
    if (!open_face(G, T, i, j, k)) {
        lam[x] = 0.0;
        return;
    }
    double gl = 0.0;
    double r = mu[T][x];
    if (T == 0 && j == G.ny - 1) {
        r += along<T, 0, false>(G, vel, mu, i, j, k, gl);
        r += along<T, 1, true>(G, vel, mu, i, j, k, gl);
    } else {
        r += along<T, 0, false>(G, vel, mu, i, j, k, gl);
        r += along<T, 1, false>(G, vel, mu, i, j, k, gl);
    }
    r += along<T, 2, false>(G, vel, mu, i, j, k, gl);
    if (T != 0) r += carried<0, T>(G, vel, mu, i, j, k);
    if (T != 1) r += carried<1, T>(G, vel, mu, i, j, k);
    if (T != 2) r += carried<2, T>(G, vel, mu, i, j, k);
    lam[x] = r;
    if (T == 0 && j == G.ny - 1 && glid) glid[(long)k * (G.nx + 1) + i] += gl;
}

struct AdjVecs {
    const double *vel[3];
    const double *mu[3];
    double *lam[3];
    long n[3];       // faces per component
    unsigned b[3];   // blocks per component
};

// one thread per face of the three components; the blocks of each component
// are contiguous, so a block never mixes components
__global__ __launch_bounds__(256) void k_mom_adjoint(AdjGrid G, AdjVecs V, double *__restrict__ glid) {
    unsigned b = blockIdx.x;
    int t = 0;
    if (b >= V.b[0]) { b -= V.b[0]; t = 1; if (b >= V.b[1]) { b -= V.b[1]; t = 2; } }
    const long x = (long)b * blockDim.x + threadIdx.x;
    if (x >= V.n[t]) return;
    if (t == 0) gather_face<0>(G, V.vel, V.mu, V.lam[0], glid, x);
    else if (t == 1) gather_face<1>(G, V.vel, V.mu, V.lam[1], glid, x);
    else gather_face<2>(G, V.vel, V.mu, V.lam[2], glid, x);
}

// out = scale * a on open faces of component c, 0 on closed faces
__global__ void k_scale_open(AdjGrid G, int c, const double *__restrict__ a, double scale, double *__restrict__ out,
                             long n) {
    for (long x = (long)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (long)gridDim.x * blockDim.x) {
        const int e0 = ext(G, c, 0), e1 = ext(G, c, 1);
        const int i = (int)(x % e0), j = (int)((x / e0) % e1), k = (int)(x / ((long)e0 * e1));
        out[x] = open_face(G, c, i, j, k) ? scale * a[x] : 0.0;
    }
}

// per-block sums of squares over open faces (fixed order: grid-stride
// per thread, wave butterfly, fixed four-wave combine)
__global__ void k_sumsq_open(AdjGrid G, int c, const double *__restrict__ a, long n, double *__restrict__ part) {
    __shared__ double s[4];
    double acc = 0.0;
    for (long x = (long)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (long)gridDim.x * blockDim.x) {
        const int e0 = ext(G, c, 0), e1 = ext(G, c, 1);
        const int i = (int)(x % e0), j = (int)((x / e0) % e1), k = (int)(x / ((long)e0 * e1));
        if (open_face(G, c, i, j, k)) acc += a[x] * a[x];
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
    AdjVecs V;
    V.n[0] = (long)(A.nx + 1) * A.ny * A.nz;
    V.n[1] = (long)A.nx * (A.ny + 1) * A.nz;
    V.n[2] = (long)A.nx * A.ny * (A.nz + 1);
    unsigned nb = 0;
    for (int c = 0; c < 3; ++c) {
        V.vel[c] = vel[c];
        V.mu[c] = mu[c];
        V.lam[c] = lam[c];
        V.b[c] = (unsigned)((V.n[c] + 255) / 256);
        nb += V.b[c];
    }
    hipLaunchKernelGGL(k_mom_adjoint, dim3(nb), dim3(256), 0, s, G, V, glid);
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
