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
// it (each interface evaluated once per tile, in LDS), so the result has no
// atomics and repeats bitwise.  SMART is piecewise
// linear in (U, C, D): the adjoint uses the slopes of the branch the forward
// step took; a zero transport velocity gives a zero flux and no
// contribution.
#include "nsp_internal.h"

namespace nsp {

namespace {

struct AdjGrid {
    int nx, ny, nz;
    int ex[3][3];  // faces of component c along direction d
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

// 32-bit index and neighbour distance along D in the array of component C
// (the launcher refuses arrays of 2^31 or more faces)
template <int C>
__device__ __forceinline__ int fid32(const AdjGrid &G, int i, int j, int k) {
    return (k * G.ex[C][1] + j) * G.ex[C][0] + i;
}
template <int C, int D>
__device__ __forceinline__ int fstride32(const AdjGrid &G) {
    return D == 0 ? 1 : (D == 1 ? G.ex[C][0] : G.ex[C][0] * G.ex[C][1]);
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
// are X0..X3; Delta = X2 - X1; Phi = a (a > 0: SMART(X0, X1, X2), else
// SMART(X3, X2, X1)), a the mean of the two faces of the transport component
// that straddle the interface (own axis: of X1 and X2).

// SMART (normalised variable, Gaskell & Lau) face value of the upwind
// triple (U, C, D) and its slopes on the branch taken, without branches
__device__ __forceinline__ double smart_lin(double U, double C, double D, double &sU, double &sC, double &sD) {
    const double delta = D - U;
    const bool z = delta == 0.0;
    const double ph = (C - U) / (z ? 1.0 : delta);
    const bool b1 = ph > 0.0 && ph < 1.0 / 6.0;
    const bool b2 = ph >= 1.0 / 6.0 && ph < 5.0 / 6.0;
    const bool b3 = ph >= 5.0 / 6.0 && ph < 1.0;
    const double pf = b1 ? 3.0 * ph : (b2 ? 0.75 * ph + 0.375 : (b3 ? 1.0 : ph));
    sU = z ? 0.0 : (b1 ? -2.0 : (b2 ? -0.125 : 0.0));
    sC = z ? 1.0 : (b1 ? 3.0 : (b2 ? 0.75 : (b3 ? 0.0 : 1.0)));
    sD = z ? 0.0 : (b2 ? 0.375 : (b3 ? 1.0 : 0.0));
    return z ? C : U + pf * delta;
}

// A block gathers lam for a tile of TX x TY x TZ faces of component T.
// The block evaluates, once each, the interfaces the tile's faces read into
// LDS: those of component T along x, y and z whose lines hold a face of the
// tile (lower faces from 2 before the tile to 1 past it), and those of the
// two other components along T whose transport velocity averages a face of
// the tile.  Each face sums its records in a fixed order, family by family.
// 16 x 8 x 4 faces: x rows of 16 doubles fill whole 128-byte lines
constexpr int TX = 16, TY = 8, TZ = 4, kTile = TX * TY * TZ;
constexpr int kAdjThreads = kTile;
constexpr int NFX = (TX + 3) * TY * TZ, NFY = TX * (TY + 3) * TZ, NFZ = TX * TY * (TZ + 3);
constexpr int cmax(int a, int b) { return a > b ? a : b; }
// the largest family of carried interfaces: the tile extended by one face
// along the carried component's axis
constexpr int NKMAX = cmax(cmax((TX + 1) * TY * TZ, TX * (TY + 1) * TZ), TX * TY * (TZ + 1));

// The cell flags of a tile and 3 cells around it, staged in LDS (cells
// outside the domain: 0, so their faces read as closed); every face an
// interface of the tile touches lies in this box.
constexpr int FBX = TX + 6, FBY = TY + 6, FBZ = TZ + 6;
struct FlagBox {
    const uint8_t *f;  // LDS, [FBZ][FBY][FBX]
    int ox, oy, oz;    // global cell of element 0
    __device__ __forceinline__ int index(int i, int j, int k) const {
        return ((k - oz) * FBY + (j - oy)) * FBX + (i - ox);
    }
    __device__ __forceinline__ bool open(int c, int i, int j, int k) const {
        const uint8_t bit = c == 0 ? FL_XM : (c == 1 ? FL_YM : FL_ZM);
        return (f[index(i, j, k)] & bit) != 0;
    }
};

// The transpose of interface (C, D, L = (i,j,k)) applied to its adjoint
// weights wphi = dt/h (mu(L+e) - mu(L)), wdel = dt nu/h^2 (mu(L) - mu(L+e))
// (closed faces: mu = 0): r[0..3] to the faces of component C at L - e, L,
// L + e, L + 2e; rl to the lid beside L; tw to each of the two faces of
// component D that carry the transport velocity (C != D).
template <int C, int D>
__device__ __forceinline__ void iface(const AdjGrid &G, const FlagBox &FB, const double *const *vel,
                                      const double *const *mu, int i, int j, int k, double r[4], double &rl,
                                      double &tw) {
    constexpr int di = D == 0, dj = D == 1, dk = D == 2;
    constexpr int fd = D == 0 ? 1 : (D == 1 ? FBX : FBX * FBY);  // flag-box strides along D and C
    constexpr int fc = C == 0 ? 1 : (C == 1 ? FBX : FBX * FBY);
    constexpr uint8_t bc = C == 0 ? FL_XM : (C == 1 ? FL_YM : FL_ZM), bd = D == 0 ? FL_XM : (D == 1 ? FL_YM : FL_ZM);
    // open bits from LDS first; the global loads then depend on them only
    const int b = FB.index(i, j, k);
    const bool oL = (FB.f[b] & bc) != 0, oU = (FB.f[b + fd] & bc) != 0;
    const bool om = (FB.f[b - fd] & bc) != 0, o2 = (FB.f[b + 2 * fd] & bc) != 0;
    const bool t0 = C != D && (FB.f[b - fc + fd] & bd) != 0, t1 = C != D && (FB.f[b + fd] & bd) != 0;
    r[0] = r[1] = r[2] = r[3] = 0.0;
    rl = tw = 0.0;
    if (!oL && !oU) return;
    const double *phi = vel[C];
    const int id = fid32<C>(G, i, j, k), s = fstride32<C, D>(G);
    double a0 = 0.0, a1 = 0.0;
    if (C != D) {
        // the two faces of component D at L + e_D - e_C and L + e_D
        const int jd = fid32<D>(G, i + di, j + dj, k + dk);
        a1 = t1 ? vel[D][jd] : 0.0;
        a0 = t0 ? vel[D][jd - fstride32<D, C>(G)] : 0.0;
    }
    const bool isL = C == 0 && D == 1 && j == G.ny - 1, isU = C == 0 && D == 1 && j + 1 == G.ny - 1;
    // interior: the four positions are open faces and no lid is near, so
    // the image rule is the identity
    const bool inner = oL && oU && om && o2 && !isL && !isU;
    double X0, X1, X2, X3, mL, mU;
    if (inner) {
        X0 = phi[id - s];
        X1 = phi[id];
        X2 = phi[id + s];
        X3 = phi[id + 2 * s];
        mL = mu[C][id];
        mU = mu[C][id + s];
    } else {
        const double Pm = om ? phi[id - s] : 0.0, P0 = oL ? phi[id] : 0.0;
        const double P1 = oU ? phi[id + s] : 0.0, P2 = o2 ? phi[id + 2 * s] : 0.0;
        mL = oL ? mu[C][id] : 0.0;
        mU = oU ? mu[C][id + s] : 0.0;
        const double lv = (isL || isU) ? G.lid[k * (G.nx + 1) + i] : 0.0;
        const double wL = isL ? lv : 0.0, wU = isU ? lv : 0.0;
        // image-resolved values
        if (C == D) {
            X1 = oL ? P0 : 0.0;
            X2 = P1;
            X0 = oL ? Pm : -P1;
            X3 = oL ? (!oU ? -P0 : P2) : P2;
        } else {
            if (oL) {
                X1 = P0;
                X0 = om ? Pm : 2.0 * 0.0 - P0;
                X2 = oU ? P1 : 2.0 * wL - P0;
                X3 = !oU ? 2.0 * wL - X0 : (o2 ? P2 : 2.0 * wU - X2);
            } else {
                X2 = P1;
                X1 = 2.0 * 0.0 - P1;
                X3 = o2 ? P2 : 2.0 * wU - P1;
                X0 = 2.0 * 0.0 - X3;
            }
        }
    }
    const double wphi = G.dt * G.ih[D] * (mU - mL);
    const double wdel = G.dt * G.inv_re * G.ih2[D] * (mL - mU);
    const double a = C == D ? 0.5 * (X1 + X2) : 0.5 * (a0 + a1);
    const bool pos = a > 0.0;
    double sU, sC, sD;
    const double S = smart_lin(pos ? X0 : X3, pos ? X1 : X2, pos ? X2 : X1, sU, sC, sD);
    // weights of X0..X3
    const double wa = a != 0.0 ? wphi * a : 0.0;
    const double ws = a != 0.0 ? wphi * 0.5 * S : 0.0;
    double w0 = pos ? wa * sU : 0.0;
    double w1 = (pos ? wa * sC : wa * sD) - wdel;
    double w2 = (pos ? wa * sD : wa * sC) + wdel;
    double w3 = pos ? 0.0 : wa * sU;
    if (C == D) {
        w1 += ws;
        w2 += ws;
    } else {
        tw = ws;
    }
    // through the transpose of the image rule onto the real values
    if (inner) {
        r[0] = w0;
        r[1] = w1;
        r[2] = w2;
        r[3] = w3;
    } else if (C == D) {
        if (oL) {
            r[0] = om ? w0 : 0.0;
            r[1] = w1 - (oU ? 0.0 : w3);
            r[2] = oU ? w2 : 0.0;
            r[3] = (oU && o2) ? w3 : 0.0;
        } else {
            r[2] = w2 - w0;
            r[3] = o2 ? w3 : 0.0;
        }
    } else {
        if (oL) {
            // X3
            if (!oU) {
                w0 -= w3;
                rl += isL ? 2.0 * w3 : 0.0;
            } else if (o2) {
                r[3] = w3;
            } else {
                r[2] = -w3;
                rl += isU ? 2.0 * w3 : 0.0;
            }
            // X2
            if (oU) r[2] += w2;
            else {
                r[1] -= w2;
                rl += isL ? 2.0 * w2 : 0.0;
            }
            r[1] += w1;
            // X0
            if (om) r[0] = w0;
            else r[1] -= w0;
        } else {
            const double w3x = w3 - w0;  // X0 = -X3
            if (o2) r[3] = w3x;
            else {
                r[2] = -w3x;
                rl = isU ? 2.0 * w3x : 0.0;
            }
            r[2] += w2 - w1;
        }
    }
}

// Records of one interface family at a time: r[pos][record], row 4 the lid
// part of the y interfaces of u.  The families are evaluated and gathered
// one after another (own interfaces along x, y, z, then the carried ones),
// so the block needs LDS for the largest family only (38.9 KB instead of
// the 89.6 KB all families would take) and several blocks share a compute
// unit.
constexpr int NREC = cmax(cmax(NFX, NFY), NFZ);
static_assert(NKMAX <= NREC, "each family of carried records fits one record row");
struct AdjLds {
    double rec[5][NREC];
    uint8_t flg[FBX * FBY * FBZ];  // cell flags of the tile and 3 cells around it
};

// local box of a record family: base offset from the tile origin, extents
struct Box {
    int bx, by, bz, ex, ey, ez;
    __device__ int size() const { return ex * ey * ez; }
    __device__ void at(int q, int &a, int &b, int &c) const {
        a = q % ex;
        b = (q / ex) % ey;
        c = q / (ex * ey);
    }
};

template <int T, int C>
__device__ __forceinline__ Box carried_box() {
    // L = t - e_T + {0, e_C}
    return Box{-(T == 0), -(T == 1), -(T == 2), TX + (C == 0), TY + (C == 1), TZ + (C == 2)};
}

// own interfaces of component T along D whose lines hold a face of the
// tile: lower faces from 2 before the tile to 1 past it
template <int D>
__device__ __forceinline__ Box own_box() {
    return Box{-2 * (D == 0), -2 * (D == 1), -2 * (D == 2), TX + 3 * (D == 0), TY + 3 * (D == 1), TZ + 3 * (D == 2)};
}

template <int T, int D>
__device__ __forceinline__ void own_records(const AdjGrid &G, const FlagBox &FB, const double *const *vel,
                                            const double *const *mu, int x0, int y0, int z0, AdjLds &S) {
    const Box B = own_box<D>();
    for (int q = threadIdx.x; q < B.size(); q += kAdjThreads) {
        double r[4], rl, tw;
        int a, b, c;
        B.at(q, a, b, c);
        iface<T, D>(G, FB, vel, mu, x0 + B.bx + a, y0 + B.by + b, z0 + B.bz + c, r, rl, tw);
        for (int m = 0; m < 4; ++m) S.rec[m][q] = r[m];
        if (T == 0 && D == 1) S.rec[4][q] = rl;
    }
}

// the four records of face t along D: lower faces t - 2e .. t + e hold t at
// positions 3 .. 0 of their lines
template <int D>
__device__ __forceinline__ double own_sum(const AdjLds &S, int tx, int ty, int tz) {
    const Box B = own_box<D>();
    const int q = (tz * B.ey + ty) * B.ex + tx;
    constexpr int st = D == 0 ? 1 : (D == 1 ? TX : TX * TY);
    return (S.rec[3][q] + S.rec[2][q + st]) + (S.rec[1][q + 2 * st] + S.rec[0][q + 3 * st]);
}

template <int T>
__device__ void adj_tile(const AdjGrid &G, const double *const *vel, const double *const *mu, double *__restrict__ lam,
                         double *__restrict__ glid, int x0, int y0, int z0, AdjLds &S) {
    constexpr int C1 = T == 0 ? 1 : 0, C2 = T == 2 ? 1 : 2;  // the other two components
    const Box K1 = carried_box<T, C1>(), K2 = carried_box<T, C2>();
    const FlagBox FB{S.flg, x0 - 3, y0 - 3, z0 - 3};
    for (int q = threadIdx.x; q < FBX * FBY * FBZ; q += kAdjThreads) {
        const int i = FB.ox + q % FBX, j = FB.oy + (q / FBX) % FBY, k = FB.oz + q / (FBX * FBY);
        const bool in = (unsigned)i < (unsigned)G.nx && (unsigned)j < (unsigned)G.ny && (unsigned)k < (unsigned)G.nz;
        S.flg[q] = in ? G.flags[((long)k * G.ny + j) * G.nx + i] : (uint8_t)0;
    }
    const int tx = threadIdx.x % TX, ty = (threadIdx.x / TX) % TY, tz = threadIdx.x / (TX * TY);
    const int i = x0 + tx, j = y0 + ty, k = z0 + tz;
    // every thread takes part in every phase's records and barriers; only
    // faces inside the array gather and store
    const bool in = i < ext(G, T, 0) && j < ext(G, T, 1) && k < ext(G, T, 2);
    const long x = in ? fid<T>(G, i, j, k) : 0;
    __syncthreads();
    const bool open = in && FB.open(T, i, j, k);
    double acc = open ? mu[T][x] : 0.0;
    own_records<T, 0>(G, FB, vel, mu, x0, y0, z0, S);
    __syncthreads();
    if (open) acc += own_sum<0>(S, tx, ty, tz);
    __syncthreads();
    own_records<T, 1>(G, FB, vel, mu, x0, y0, z0, S);
    __syncthreads();
    if (open) acc += own_sum<1>(S, tx, ty, tz);
    if (T == 0 && in && j == G.ny - 1) {
        // lid beside the top row of u: the y interfaces below and above it
        const int q0 = (tz * (TY + 3) + ty + 1) * TX + tx;
        glid[(long)k * (G.nx + 1) + i] += S.rec[4][q0] + S.rec[4][q0 + TX];
    }
    __syncthreads();
    own_records<T, 2>(G, FB, vel, mu, x0, y0, z0, S);
    __syncthreads();
    if (open) acc += own_sum<2>(S, tx, ty, tz);
    __syncthreads();
    // carried interfaces (the other components along T, whose transport
    // velocity averages a face of the tile): K1 in row 0, K2 in row 1
    const int n1 = K1.size(), n2 = n1 + K2.size();
    for (int q = threadIdx.x; q < n2; q += kAdjThreads) {
        double r[4], rl, tw;
        int a, b, c;
        if (q < n1) {
            K1.at(q, a, b, c);
            iface<C1, T>(G, FB, vel, mu, x0 + K1.bx + a, y0 + K1.by + b, z0 + K1.bz + c, r, rl, tw);
            S.rec[0][q] = tw;
        } else {
            K2.at(q - n1, a, b, c);
            iface<C2, T>(G, FB, vel, mu, x0 + K2.bx + a, y0 + K2.by + b, z0 + K2.bz + c, r, rl, tw);
            S.rec[1][q - n1] = tw;
        }
    }
    __syncthreads();
    if (!in) return;
    if (!open) {
        lam[x] = 0.0;
        return;
    }
    // carried interfaces: L = t - e_T and t - e_T + e_C
    {
        const int q = (tz * K1.ey + ty) * K1.ex + tx;
        const int st = C1 == 0 ? 1 : (C1 == 1 ? K1.ex : K1.ex * K1.ey);
        acc += S.rec[0][q] + S.rec[0][q + st];
    }
    {
        const int q = (tz * K2.ey + ty) * K2.ex + tx;
        const int st = C2 == 0 ? 1 : (C2 == 1 ? K2.ex : K2.ex * K2.ey);
        acc += S.rec[1][q] + S.rec[1][q + st];
    }
    lam[x] = acc;
}

struct AdjVecs {
    const double *vel[3];
    const double *mu[3];
    double *lam[3];
    int tiles[3][3];  // tiles of each component along x, y, z
    unsigned b[3];    // blocks of each component
};

// one block per tile; the blocks of each component are contiguous
__global__ __launch_bounds__(kAdjThreads) void k_mom_adjoint(AdjGrid G, AdjVecs V, double *__restrict__ glid) {
    __shared__ AdjLds S;
    unsigned b = blockIdx.x;
    int t = 0;
    if (b >= V.b[0]) { b -= V.b[0]; t = 1; if (b >= V.b[1]) { b -= V.b[1]; t = 2; } }
    const int bx = b % V.tiles[t][0], by = (b / V.tiles[t][0]) % V.tiles[t][1], bz = b / (V.tiles[t][0] * V.tiles[t][1]);
    if (t == 0) adj_tile<0>(G, V.vel, V.mu, V.lam[0], glid, bx * TX, by * TY, bz * TZ, S);
    else if (t == 1) adj_tile<1>(G, V.vel, V.mu, V.lam[1], glid, bx * TX, by * TY, bz * TZ, S);
    else adj_tile<2>(G, V.vel, V.mu, V.lam[2], glid, bx * TX, by * TY, bz * TZ, S);
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
    const int n[3] = {A.nx, A.ny, A.nz};
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) G.ex[c][d] = n[d] + (c == d);
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
    // 32-bit face indices
    if ((long long)(A.nx + 1) * (A.ny + 1) * (A.nz + 1) >= (1LL << 31)) return hipErrorInvalidValue;
    AdjVecs V;
    const int n[3] = {A.nx, A.ny, A.nz}, tile[3] = {TX, TY, TZ};
    unsigned nb = 0;
    for (int c = 0; c < 3; ++c) {
        V.vel[c] = vel[c];
        V.mu[c] = mu[c];
        V.lam[c] = lam[c];
        unsigned cnt = 1;
        for (int d = 0; d < 3; ++d) {
            V.tiles[c][d] = (n[d] + (c == d) + tile[d] - 1) / tile[d];
            cnt *= (unsigned)V.tiles[c][d];
        }
        V.b[c] = cnt;
        nb += cnt;
    }
    hipLaunchKernelGGL(k_mom_adjoint, dim3(nb), dim3(kAdjThreads), 0, s, G, V, glid);
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
