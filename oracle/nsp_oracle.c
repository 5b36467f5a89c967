/*
 * Plain FP64 CPU oracle for the projection Navier-Stokes step and its
 * Poisson solve.  TEST INFRASTRUCTURE ONLY: it is linked by the tests,
 * by the smoke check and by the CPU-baseline leg of the benchmark, never by
 * the product library.  It shares no code, header or table with the HIP
 * path.  Everything is written for readability: no blocking, no fast paths.
 *
 * What it computes (Croce, Ruprecht, Krause, "Parallel-in-space-and-time
 * simulation of the 3D unsteady Navier-Stokes equations", Sec. 2):
 *   - incompressible Navier-Stokes in dimensionless form, Eq. (1);
 *   - Chorin-Temam projection on a uniform staggered (MAC) grid with forward
 *     Euler in time, central differences for diffusion and the pressure
 *     gradient, SMART (bounded QUICK, normalised-variable form of Gaskell &
 *     Lau) upwinding for convection, first-order cell enumeration for solid
 *     cells with no-slip walls (Sec. 2, discretization paragraph);
 *   - the pressure Poisson equation of the projection, solved here with
 *     Jacobi-preconditioned CG (the paper uses BiCGStab; the operator is
 *     symmetric positive semi-definite so CG applies), plus an FP32-inner /
 *     FP64-outer defect-correction variant.
 *
 * Readings where the paper is silent (all shared, as written rules, with
 * the GPU path):
 *   - a face is open when it is interior and both adjacent cells are fluid;
 *     closed faces carry velocity 0;
 *   - stencil values beyond a closed face come from an image rule: along the
 *     component's own axis the closed face holds 0 and the next position is
 *     the odd reflection; across it a no-slip wall sits half a cell away and
 *     the image is 2*wall - mirror value, resolved nearest-first;
 *   - the lid velocity enters only as the wall value of u on the top face;
 *   - convection is in conservative flux form, with the transport velocity
 *     the average of the two straddling normal components;
 *   - the Poisson right-hand side b = -div(F)/dt is made mean-free over the
 *     fluid cells, and the pressure gauge is mean_fluid(p) = 0;
 *   - PCG stops when ||r||_2 <= rtol ||b||_2 on the recursive residual; the
 *     true residual is then recomputed and, if above 2 rtol ||b||, CG is
 *     restarted from it;
 *   - a warm start with ||b - A x0|| > ||b|| is replaced by x0 = 0 (every
 *     solver, before its first iteration).
 *
 * OpenMP is used only on loops whose iterations write disjoint outputs, so
 * results do not depend on the thread count.  Every reduction is a serial
 * sum in natural (i fastest, then j, then k) order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* threads of the OpenMP loops (for timing the oracle on a given core count) */
int og_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void og_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

typedef struct {
    int nx, ny, nz;
    double hx, hy, hz;
    double re;
    const uint8_t *solid; /* nz*ny*nx, nonzero = solid; NULL = all fluid */
    const double *lid;    /* nz*(nx+1): wall value of u on the top face (y = Ly) */
    int periodic_z;       /* 1: periodic in z (the paper's runs), 0: walls at z = 0, Lz */
    int slip_obstacles;   /* 1: free-slip on obstacle surfaces, 0: no-slip (the paper's) */
    int upwind;           /* 1: first-order upwind (donor-cell) convective face values instead
                             of SMART: a coarse-propagator variant */
} og_grid;

typedef struct {
    int iters;    /* CG iterations (inner iterations for the mixed solver) */
    int outer;    /* defect-correction sweeps (mixed) / restarts (fp64) */
    int status;   /* 0 ok, 2 not converged, 3 non-finite */
    double rel_res_true;
} og_info;

/* ---------------------------------------------------------------- indexing */

static double hdir(const og_grid *g, int d) { return d == 0 ? g->hx : (d == 1 ? g->hy : g->hz); }
static int ndir(const og_grid *g, int d) { return d == 0 ? g->nx : (d == 1 ? g->ny : g->nz); }

/* z index of a cell or face position: wrapped into [0, nz) when the domain
 * is periodic in z (the w face at z = Lz is then the face at z = 0) */
static int wrapz(const og_grid *g, int k) {
    if (!g->periodic_z) return k;
    k %= g->nz;
    return k < 0 ? k + g->nz : k;
}

static size_t cidx(const og_grid *g, int i, int j, int k) {
    k = wrapz(g, k);
    return ((size_t)k * g->ny + j) * g->nx + i;
}

static int fluid(const og_grid *g, int i, int j, int k) {
    k = wrapz(g, k);
    if (i < 0 || i >= g->nx || j < 0 || j >= g->ny || k < 0 || k >= g->nz) return 0;
    if (g->solid && g->solid[cidx(g, i, j, k)]) return 0;
    return 1;
}

/* extent of the face array of component c along direction d */
static int fext(const og_grid *g, int c, int d) { return ndir(g, d) + (c == d ? 1 : 0); }

static int face_exists(const og_grid *g, int c, const int f[3]) {
    const int k = wrapz(g, f[2]);
    for (int d = 0; d < 2; ++d)
        if (f[d] < 0 || f[d] >= fext(g, c, d)) return 0;
    return k >= 0 && k < fext(g, c, 2);
}

/* storage index of a face value; with periodic z the position is wrapped,
 * so reads of the w plane at z = Lz see the plane at z = 0 */
static size_t fidx(const og_grid *g, int c, const int f[3]) {
    return ((size_t)wrapz(g, f[2]) * fext(g, c, 1) + f[1]) * fext(g, c, 0) + f[0];
}

/* storage index without wrapping: where a sweep over every stored face
 * writes (the duplicate w plane at z = Lz gets the value of z = 0) */
static size_t fidx_raw(const og_grid *g, int c, const int f[3]) {
    return ((size_t)f[2] * fext(g, c, 1) + f[1]) * fext(g, c, 0) + f[0];
}

/* the face of component c at f separates cell f - e_c from cell f */
static int face_open(const og_grid *g, int c, const int f[3]) {
    if (!face_exists(g, c, f)) return 0;
    int lo[3] = {f[0], f[1], f[2]};
    lo[c] -= 1;
    return fluid(g, lo[0], lo[1], lo[2]) && fluid(g, f[0], f[1], f[2]);
}

size_t og_face_count(const og_grid *g, int c) {
    return (size_t)fext(g, c, 0) * fext(g, c, 1) * fext(g, c, 2);
}

/* real face value: closed faces are walls with zero normal velocity */
static double real_val(const og_grid *g, int c, const double *phi, const int f[3]) {
    return face_open(g, c, f) ? phi[fidx(g, c, f)] : 0.0;
}

/* ----------------------------------------------------------- image values */

/* Value of the no-slip wall seen by component c when the wall lies half a
 * cell beyond the open face f in direction d, sense s.  Only u sees the lid,
 * and only across the top boundary of the domain. */
static double wall_value(const og_grid *g, int c, const int f[3], int d, int s) {
    if (c == 0 && d == 1 && s > 0 && f[1] == g->ny - 1)
        return g->lid[(size_t)f[2] * (g->nx + 1) + f[0]];
    return 0.0;
}

/* The closed position f of a component across whose axis d the stencil
 * looks lies in the grid along d when a solid cell closes it (an obstacle
 * wall), outside when the domain boundary does.  With free-slip obstacles
 * the image across an obstacle wall is the mirror value itself (zero
 * tangential stress) instead of 2*wall - mirror. */
static int slip_wall(const og_grid *g, const int f[3], int d) {
    if (!g->slip_obstacles) return 0;
    if (d == 2 && g->periodic_z) return 1;
    return f[d] >= 0 && f[d] < ndir(g, d);
}

/* Value used by the stencil of the open face f of component c at offset m
 * (|m| = 1 or 2) along direction d: the real value where the position is an
 * open face, the image value otherwise. */
static double stencil_val(const og_grid *g, int c, const double *phi, const int f[3], int d, int m) {
    int s = m > 0 ? 1 : -1;
    int two = (m == 2 || m == -2);
    int f1[3] = {f[0], f[1], f[2]};
    int f2[3] = {f[0], f[1], f[2]};
    f1[d] += s;
    f2[d] += 2 * s;
    double phi0 = phi[fidx(g, c, f)];
    if (d == c) {
        /* along the component's own axis: a closed face holds 0, the
         * position beyond it is the odd reflection of phi0 about it */
        if (!face_open(g, c, f1)) return two ? -phi0 : 0.0;
        if (!two) return phi[fidx(g, c, f1)];
        if (!face_open(g, c, f2)) return 0.0;
        return phi[fidx(g, c, f2)];
    }
    /* across the component's axis: a closed neighbour means a wall half a
     * cell away; images are 2*wall - mirror (no-slip) or the mirror value
     * (free-slip obstacle), mirror resolved nearest-first */
    if (!face_open(g, c, f1)) {
        double mirror = two ? stencil_val(g, c, phi, f, d, -s) : phi0;
        if (slip_wall(g, f1, d)) return mirror;
        return 2.0 * wall_value(g, c, f, d, s) - mirror;
    }
    if (!two) return phi[fidx(g, c, f1)];
    if (!face_open(g, c, f2)) {
        if (slip_wall(g, f2, d)) return phi[fidx(g, c, f1)];
        return 2.0 * wall_value(g, c, f1, d, s) - phi[fidx(g, c, f1)];
    }
    return phi[fidx(g, c, f2)];
}

/* ------------------------------------------------------------------ SMART */

/* SMART face value in normalised-variable form (Gaskell & Lau 1988): the
 * upwind, central and downwind values U, C, D give phi_hat = (C-U)/(D-U);
 * the face value is 3 phi_hat on (0,1/6), 3/4 phi_hat + 3/8 on [1/6,5/6),
 * 1 on [5/6,1) and phi_hat (first-order upwind) elsewhere. */
/* seg (if not NULL) receives the segment taken: 0 upwind (D = U, or phi_hat
 * outside [0,1)), 1 slope 3, 2 QUICK, 3 the cap at 1. */
static double smart_seg(double U, double C, double D, int *seg) {
    double delta = D - U;
    if (delta == 0.0) {
        if (seg) *seg = 0;
        return C;
    }
    double ph = (C - U) / delta;
    double pf;
    int k;
    if (ph > 0.0 && ph < 1.0 / 6.0) {
        pf = 3.0 * ph;
        k = 1;
    } else if (ph >= 1.0 / 6.0 && ph < 5.0 / 6.0) {
        pf = 0.75 * ph + 0.375;
        k = 2;
    } else if (ph >= 5.0 / 6.0 && ph < 1.0) {
        pf = 1.0;
        k = 3;
    } else {
        pf = ph;
        k = 0;
    }
    if (seg) *seg = k;
    return U + pf * delta;
}

double og_smart(double U, double C, double D) { return smart_seg(U, C, D, NULL); }

/* --------------------------------------------------------- momentum (a1) */

/* Convective flux of component c through the control-volume face at
 * f + s/2 e_d: transport velocity times the SMART upwind face value.  code
 * (if not NULL) receives the branch taken: 0 for a zero transport velocity,
 * else 1 + (transport velocity < 0) + 2 * (SMART segment). */
static double conv_flux(const og_grid *g, int c, const double *vel[3], const int f[3], int d, int s,
                        signed char *code) {
    const double *phi = vel[c];
    double abar;
    if (d == c) {
        int f1[3] = {f[0], f[1], f[2]};
        f1[d] += s;
        abar = 0.5 * (real_val(g, c, phi, f) + real_val(g, c, phi, f1));
    } else {
        /* the two d-faces straddling position f along c */
        int q1[3] = {f[0], f[1], f[2]}, q2[3] = {f[0], f[1], f[2]};
        if (s > 0) { q1[d] += 1; q2[d] += 1; }
        q1[c] -= 1;
        abar = 0.5 * (real_val(g, d, vel[d], q1) + real_val(g, d, vel[d], q2));
    }
    if (code) *code = 0;
    if (abar == 0.0) return 0.0;
    double phi0 = phi[fidx(g, c, f)];
    double U, C, D;
    /* donor cell: the face carries the value of the node on its upwind side,
     * the C of the SMART triple below */
    if (s > 0) {
        if (abar > 0.0) { U = stencil_val(g, c, phi, f, d, -1); C = phi0; D = stencil_val(g, c, phi, f, d, 1); }
        else { U = stencil_val(g, c, phi, f, d, 2); C = stencil_val(g, c, phi, f, d, 1); D = phi0; }
    } else {
        if (abar > 0.0) { U = stencil_val(g, c, phi, f, d, -2); C = stencil_val(g, c, phi, f, d, -1); D = phi0; }
        else { U = stencil_val(g, c, phi, f, d, 1); C = phi0; D = stencil_val(g, c, phi, f, d, -1); }
    }
    if (g->upwind) {
        if (code) *code = (signed char)(1 + (abar < 0.0));
        return abar * C;
    }
    int seg = 0;
    const double v = smart_seg(U, C, D, &seg);
    if (code) *code = (signed char)(1 + (abar < 0.0) + 2 * seg);
    return abar * v;
}

/* Predictor F = phi + dt (Lap(phi)/Re - Conv(phi)) for every open face of
 * every component; closed faces get 0.  out[c] has the layout of vel[c]. */
void og_momentum(const og_grid *g, const double *u, const double *v, const double *w, double dt,
                 double *Fu, double *Fv, double *Fw) {
    const double *vel[3] = {u, v, w};
    double *out[3] = {Fu, Fv, Fw};
    for (int c = 0; c < 3; ++c) {
        int ex = fext(g, c, 0), ey = fext(g, c, 1), ez = fext(g, c, 2);
#pragma omp parallel for schedule(static)
        for (int k = 0; k < ez; ++k)
            for (int j = 0; j < ey; ++j)
                for (int i = 0; i < ex; ++i) {
                    int f[3] = {i, j, k};
                    size_t id = fidx(g, c, f), od = fidx_raw(g, c, f);
                    if (!face_open(g, c, f)) { out[c][od] = 0.0; continue; }
                    double phi0 = vel[c][id];
                    double conv = 0.0, lap = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        double h = hdir(g, d);
                        double fp = conv_flux(g, c, vel, f, d, 1, NULL);
                        double fm = conv_flux(g, c, vel, f, d, -1, NULL);
                        conv += (fp - fm) / h;
                        double vp = stencil_val(g, c, vel[c], f, d, 1);
                        double vm = stencil_val(g, c, vel[c], f, d, -1);
                        lap += (vp - 2.0 * phi0 + vm) / (h * h);
                    }
                    out[c][od] = phi0 + dt * (lap / g->re - conv);
                }
    }
}

/* The branch each convective flux of the predictor takes (conv_flux's
 * code) at the state (u, v, w): codes[c] has 6 entries per face of
 * component c (direction d, side s = -1, +1 at 2 d + (s > 0)); closed faces
 * get -1.  Test infrastructure for finite-difference checks: the flux is
 * piecewise smooth, and two nearby states whose codes agree lie on the same
 * smooth piece. */
void og_momentum_branches(const og_grid *g, const double *u, const double *v, const double *w, signed char *cu,
                          signed char *cv, signed char *cw) {
    const double *vel[3] = {u, v, w};
    signed char *out[3] = {cu, cv, cw};
    for (int c = 0; c < 3; ++c) {
        int ex = fext(g, c, 0), ey = fext(g, c, 1), ez = fext(g, c, 2);
#pragma omp parallel for schedule(static)
        for (int k = 0; k < ez; ++k)
            for (int j = 0; j < ey; ++j)
                for (int i = 0; i < ex; ++i) {
                    int f[3] = {i, j, k};
                    signed char *o = out[c] + 6 * fidx_raw(g, c, f);
                    if (!face_open(g, c, f)) {
                        for (int q = 0; q < 6; ++q) o[q] = -1;
                        continue;
                    }
                    for (int d = 0; d < 3; ++d) {
                        (void)conv_flux(g, c, vel, f, d, -1, &o[2 * d]);
                        (void)conv_flux(g, c, vel, f, d, 1, &o[2 * d + 1]);
                    }
                }
    }
}

/* ------------------------------------------------- divergence and gradient */

/* (D.F)_c = sum_d (F(c + e_d/2) - F(c - e_d/2)) / h_d on fluid cells, 0 on
 * solid cells; closed faces count as 0. */
void og_divergence(const og_grid *g, const double *Fu, const double *Fv, const double *Fw, double *div) {
    const double *F[3] = {Fu, Fv, Fw};
#pragma omp parallel for schedule(static)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t id = cidx(g, i, j, k);
                if (!fluid(g, i, j, k)) { div[id] = 0.0; continue; }
                double s = 0.0;
                for (int d = 0; d < 3; ++d) {
                    int lo[3] = {i, j, k}, hi[3] = {i, j, k};
                    hi[d] += 1;
                    s += (real_val(g, d, F[d], hi) - real_val(g, d, F[d], lo)) / hdir(g, d);
                }
                div[id] = s;
            }
}

/* (G p)_f = (p(f) - p(f - e_c)) / h_c on open faces, 0 on closed faces. */
void og_gradient(const og_grid *g, const double *p, double *Gu, double *Gv, double *Gw) {
    double *out[3] = {Gu, Gv, Gw};
    for (int c = 0; c < 3; ++c) {
        int ex = fext(g, c, 0), ey = fext(g, c, 1), ez = fext(g, c, 2);
#pragma omp parallel for schedule(static)
        for (int k = 0; k < ez; ++k)
            for (int j = 0; j < ey; ++j)
                for (int i = 0; i < ex; ++i) {
                    int f[3] = {i, j, k};
                    size_t od = fidx_raw(g, c, f);
                    if (!face_open(g, c, f)) { out[c][od] = 0.0; continue; }
                    int lo[3] = {i, j, k};
                    lo[c] -= 1;
                    out[c][od] = (p[cidx(g, i, j, k)] - p[cidx(g, lo[0], lo[1], lo[2])]) / hdir(g, c);
                }
    }
}

/* ------------------------------------------------------- Poisson operator */

/* (A p)_c = sum over the open faces of c of (p_c - p_neighbour) / h_d^2;
 * this is -D G, symmetric positive semi-definite. */
void og_apply_A(const og_grid *g, const double *p, double *q) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t id = cidx(g, i, j, k);
                if (!fluid(g, i, j, k)) { q[id] = 0.0; continue; }
                double s = 0.0;
                for (int d = 0; d < 3; ++d) {
                    double h = hdir(g, d);
                    for (int sg = -1; sg <= 1; sg += 2) {
                        int nb[3] = {i, j, k};
                        nb[d] += sg;
                        if (!fluid(g, nb[0], nb[1], nb[2])) continue; /* face closed */
                        s += (p[id] - p[cidx(g, nb[0], nb[1], nb[2])]) / (h * h);
                    }
                }
                q[id] = s;
            }
}

/* Jacobi preconditioner: the diagonal of A. */
static void diag_A(const og_grid *g, double *dg) {
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t id = cidx(g, i, j, k);
                double s = 0.0;
                if (fluid(g, i, j, k))
                    for (int d = 0; d < 3; ++d) {
                        double h = hdir(g, d);
                        for (int sg = -1; sg <= 1; sg += 2) {
                            int nb[3] = {i, j, k};
                            nb[d] += sg;
                            if (fluid(g, nb[0], nb[1], nb[2])) s += 1.0 / (h * h);
                        }
                    }
                dg[id] = s;
            }
}

static size_t ncells(const og_grid *g) { return (size_t)g->nx * g->ny * g->nz; }

static int is_fluid_id(const og_grid *g, size_t id) { return !(g->solid && g->solid[id]); }

static double dot(const og_grid *g, const double *a, const double *b) {
    size_t n = ncells(g);
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* mean over fluid cells */
static double mean_fluid(const og_grid *g, const double *a) {
    size_t n = ncells(g), nf = 0;
    double s = 0.0;
    for (size_t i = 0; i < n; ++i)
        if (is_fluid_id(g, i)) { s += a[i]; ++nf; }
    return nf ? s / (double)nf : 0.0;
}

static void subtract_mean(const og_grid *g, double *a) {
    double m = mean_fluid(g, a);
    size_t n = ncells(g);
    for (size_t i = 0; i < n; ++i)
        if (is_fluid_id(g, i)) a[i] -= m;
}

/* ------------------------------------------------------ Jacobi-PCG (a3) */

/* Cold start: a warm start worse than none is dropped.  When the squared
 * norm of the starting residual b - A x exceeds that of b, x is set to 0
 * (then r = b).  The relative stopping test ||r|| <= rtol ||b|| cannot be
 * met from a starting residual far above ||b||: with b at the rounding
 * level (a flow uniform to rounding along periodic z) Krylov iterations on
 * rounding noise drift into A's null space and break down.  From x = 0
 * the same systems converge in a few iterations.  Squared sums are
 * compared, so x = 0 on entry (r = b exactly) is never a cold start.
 * Returns 1 if x was reset. */
static int cold_start_if_worse(const og_grid *g, const double *b, double *x, double *tmp) {
    size_t n = ncells(g);
    og_apply_A(g, x, tmp);
    double rr = 0.0, bb = 0.0;
    for (size_t i = 0; i < n; ++i) {
        double d = b[i] - tmp[i];
        rr += d * d;
        bb += b[i] * b[i];
    }
    if (!(rr > bb)) return 0;
    for (size_t i = 0; i < n; ++i) x[i] = 0.0;
    return 1;
}

/* Solves A x = b for a mean-free b, x holding the initial guess on entry.
 * On exit x is gauge-fixed (mean_fluid(x) = 0). */
int og_pcg(const og_grid *g, const double *b, double *x, double rtol, int maxit, og_info *info) {
    size_t n = ncells(g);
    double *r = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double));
    double *d = malloc(n * sizeof(double)), *q = malloc(n * sizeof(double));
    double *dg = malloc(n * sizeof(double));
    diag_A(g, dg);
    memset(info, 0, sizeof(*info));
    double bnorm = sqrt(dot(g, b, b));
    if (bnorm == 0.0) {
        for (size_t i = 0; i < n; ++i) x[i] = 0.0;
        free(r); free(z); free(d); free(q); free(dg);
        return 0;
    }
    int it = 0, status = 0, restarts = 0;
    double rel_true = 0.0;
    cold_start_if_worse(g, b, x, q);
    for (;;) {
        /* (re)start from the true residual */
        og_apply_A(g, x, q);
        for (size_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
        for (size_t i = 0; i < n; ++i) z[i] = dg[i] > 0.0 ? r[i] / dg[i] : 0.0;
        for (size_t i = 0; i < n; ++i) d[i] = z[i];
        double rz = dot(g, r, z);
        double rnorm = sqrt(dot(g, r, r));
        for (;;) {
            if (!isfinite(rnorm)) { status = 3; break; }
            if (rnorm <= rtol * bnorm) break;
            if (it >= maxit) { status = 2; break; }
            og_apply_A(g, d, q);
            double alpha = rz / dot(g, d, q);
            for (size_t i = 0; i < n; ++i) x[i] += alpha * d[i];
            for (size_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
            for (size_t i = 0; i < n; ++i) z[i] = dg[i] > 0.0 ? r[i] / dg[i] : 0.0;
            double rz_new = dot(g, r, z);
            double beta = rz_new / rz;
            rz = rz_new;
            for (size_t i = 0; i < n; ++i) d[i] = z[i] + beta * d[i];
            rnorm = sqrt(dot(g, r, r));
            ++it;
        }
        /* true residual */
        og_apply_A(g, x, q);
        for (size_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
        rel_true = sqrt(dot(g, r, r)) / bnorm;
        if (status != 0 || !isfinite(rel_true) || rel_true <= 2.0 * rtol || it >= maxit) break;
        ++restarts;
    }
    if (status == 0 && !isfinite(rel_true)) status = 3;
    subtract_mean(g, x);
    info->iters = it;
    info->outer = restarts;
    info->status = status;
    info->rel_res_true = rel_true;
    free(r); free(z); free(d); free(q); free(dg);
    return status;
}

/* ------------------------------- single-reduction Jacobi-PCG (a3) */

/* The same Krylov method as og_pcg with its two inner-product stages merged
 * into one (Chronopoulos & Gear 1989).  Besides x and r it carries
 * u = M^-1 r, w = A u, the search direction p and s = A p:
 *   start:  u = M^-1 r,  w = A u,  gamma = <r,u>,  delta = <w,u>
 *   step:   beta  = gamma / gamma_prev            (0 on the first step)
 *           alpha = gamma / (delta - beta gamma / alpha_prev)
 *                                                  (gamma / delta first)
 *           p = u + beta p,   s = w + beta s
 *           x = x + alpha p,  r = r - alpha s
 *           u = M^-1 r,  w = A u,  then gamma, delta and ||r||^2 together
 * The denominator is <p, A p>: expand p = u + beta p_prev, use that p_prev
 * is A-conjugate to p, and that s_prev = (r_prev - r)/alpha_prev with
 * <u, r_prev> = 0.  Stopping, true residual, restart and cold start as in
 * og_pcg. */
int og_pcg_sr(const og_grid *g, const double *b, double *x, double rtol, int maxit, og_info *info) {
    size_t n = ncells(g);
    double *r = malloc(n * sizeof(double)), *u = malloc(n * sizeof(double));
    double *w = malloc(n * sizeof(double)), *p = malloc(n * sizeof(double));
    double *sv = malloc(n * sizeof(double)), *dg = malloc(n * sizeof(double));
    diag_A(g, dg);
    memset(info, 0, sizeof(*info));
    double bnorm = sqrt(dot(g, b, b));
    if (bnorm == 0.0) {
        for (size_t i = 0; i < n; ++i) x[i] = 0.0;
        free(r); free(u); free(w); free(p); free(sv); free(dg);
        return 0;
    }
    int it = 0, status = 0, restarts = 0;
    double rel_true = 0.0;
    cold_start_if_worse(g, b, x, w);
    for (;;) {
        og_apply_A(g, x, w);
        for (size_t i = 0; i < n; ++i) r[i] = b[i] - w[i];
        for (size_t i = 0; i < n; ++i) u[i] = dg[i] > 0.0 ? r[i] / dg[i] : 0.0;
        og_apply_A(g, u, w);
        double gamma = dot(g, r, u), delta = dot(g, w, u);
        double rnorm = sqrt(dot(g, r, r));
        double gamma_prev = 0.0, alpha = 0.0;
        int first = 1;
        for (;;) {
            if (!isfinite(rnorm)) { status = 3; break; }
            if (rnorm <= rtol * bnorm) break;
            if (it >= maxit) { status = 2; break; }
            double beta = first ? 0.0 : gamma / gamma_prev;
            alpha = first ? gamma / delta : gamma / (delta - beta * gamma / alpha);
            for (size_t i = 0; i < n; ++i) {
                p[i] = first ? u[i] : u[i] + beta * p[i];
                sv[i] = first ? w[i] : w[i] + beta * sv[i];
            }
            for (size_t i = 0; i < n; ++i) x[i] += alpha * p[i];
            for (size_t i = 0; i < n; ++i) r[i] -= alpha * sv[i];
            for (size_t i = 0; i < n; ++i) u[i] = dg[i] > 0.0 ? r[i] / dg[i] : 0.0;
            og_apply_A(g, u, w);
            gamma_prev = gamma;
            gamma = dot(g, r, u);
            delta = dot(g, w, u);
            rnorm = sqrt(dot(g, r, r));
            first = 0;
            ++it;
        }
        og_apply_A(g, x, w);
        for (size_t i = 0; i < n; ++i) r[i] = b[i] - w[i];
        rel_true = sqrt(dot(g, r, r)) / bnorm;
        if (status != 0 || !isfinite(rel_true) || rel_true <= 2.0 * rtol || it >= maxit) break;
        ++restarts;
    }
    if (status == 0 && !isfinite(rel_true)) status = 3;
    subtract_mean(g, x);
    info->iters = it;
    info->outer = restarts;
    info->status = status;
    info->rel_res_true = rel_true;
    free(r); free(u); free(w); free(p); free(sv); free(dg);
    return status;
}

/* ---------------------------------------------- BiCGStab (Sec. 2) */

/* The paper solves the pressure equation with BiCGStab (van der Vorst 1992).
 * Right-preconditioned by the Jacobi diagonal M = diag(A), from the warm
 * start x, shadow residual r^ = r0; per iteration two products with A and
 * four inner products:
 *   rho' = <r^, r>;  beta = (rho'/rho)(alpha/omega);  p = r + beta (p - omega v)
 *   y = M^-1 p;  v = A y;  alpha = rho' / <r^, v>;  s = r - alpha v
 *   z = M^-1 s;  t = A z;  omega = <t, s> / <t, t>
 *   x = x + alpha y + omega z;  r = s - omega t
 * Stops like og_pcg (recursive ||r|| <= rtol ||b||, then the true residual,
 * restarting from it if above 2 rtol); a breakdown (rho' = 0 or <r^, v> = 0)
 * also restarts from the true residual, at most 16 restarts. */
int og_bicgstab(const og_grid *g, const double *b, double *x, double rtol, int maxit, og_info *info) {
    size_t n = ncells(g);
    double *r = malloc(n * sizeof(double)), *rh = malloc(n * sizeof(double));
    double *p = malloc(n * sizeof(double)), *v = malloc(n * sizeof(double));
    double *y = malloc(n * sizeof(double)), *sv = malloc(n * sizeof(double));
    double *z = malloc(n * sizeof(double)), *t = malloc(n * sizeof(double));
    double *dg = malloc(n * sizeof(double));
    diag_A(g, dg);
    memset(info, 0, sizeof(*info));
    double bnorm = sqrt(dot(g, b, b));
    int it = 0, status = 0, restarts = 0;
    double rel_true = 0.0;
    if (bnorm == 0.0) {
        for (size_t i = 0; i < n; ++i) x[i] = 0.0;
        goto done;
    }
    cold_start_if_worse(g, b, x, t);
    for (;;) {
        og_apply_A(g, x, t);
        for (size_t i = 0; i < n; ++i) { r[i] = b[i] - t[i]; rh[i] = r[i]; p[i] = 0.0; v[i] = 0.0; }
        double rho = 1.0, alpha = 1.0, omega = 1.0;
        double rnorm = sqrt(dot(g, r, r));
        for (;;) {
            if (!isfinite(rnorm)) { status = 3; break; }
            if (rnorm <= rtol * bnorm) break;
            if (it >= maxit) { status = 2; break; }
            double rho1 = dot(g, rh, r);
            if (rho1 == 0.0) break;
            double beta = (rho1 / rho) * (alpha / omega);
            for (size_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
            for (size_t i = 0; i < n; ++i) y[i] = dg[i] > 0.0 ? p[i] / dg[i] : 0.0;
            og_apply_A(g, y, v);
            double rv = dot(g, rh, v);
            if (rv == 0.0) break;
            alpha = rho1 / rv;
            for (size_t i = 0; i < n; ++i) sv[i] = r[i] - alpha * v[i];
            for (size_t i = 0; i < n; ++i) z[i] = dg[i] > 0.0 ? sv[i] / dg[i] : 0.0;
            og_apply_A(g, z, t);
            double tt = dot(g, t, t);
            omega = tt > 0.0 ? dot(g, t, sv) / tt : 0.0;
            for (size_t i = 0; i < n; ++i) x[i] = x[i] + alpha * y[i] + omega * z[i];
            for (size_t i = 0; i < n; ++i) r[i] = sv[i] - omega * t[i];
            rho = rho1;
            rnorm = sqrt(dot(g, r, r));
            ++it;
            if (omega == 0.0) break;
        }
        og_apply_A(g, x, t);
        for (size_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
        rel_true = sqrt(dot(g, r, r)) / bnorm;
        if (status != 0 || !isfinite(rel_true) || rel_true <= 2.0 * rtol || it >= maxit) break;
        if (++restarts > 16) { status = 2; break; }
    }
    if (status == 0 && !isfinite(rel_true)) status = 3;
    if (status == 0 && it >= maxit && rel_true > 2.0 * rtol) status = 2;
    subtract_mean(g, x);
done:
    info->iters = it;
    info->outer = restarts;
    info->status = status;
    info->rel_res_true = rel_true;
    free(r); free(rh); free(p); free(v); free(y); free(sv); free(z); free(t); free(dg);
    return status;
}

/* ------------------------------------- mixed precision: FP32 inner PCG */

/* (A p)_c in single precision: same open faces, FP32 values and 1/h^2. */
static void apply_A32(const og_grid *g, const float *p, float *q) {
    float ih2[3];
    for (int d = 0; d < 3; ++d) ih2[d] = (float)(1.0 / (hdir(g, d) * hdir(g, d)));
#pragma omp parallel for schedule(static)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t id = cidx(g, i, j, k);
                if (!fluid(g, i, j, k)) { q[id] = 0.0f; continue; }
                float s = 0.0f;
                for (int d = 0; d < 3; ++d)
                    for (int sg = -1; sg <= 1; sg += 2) {
                        int nb[3] = {i, j, k};
                        nb[d] += sg;
                        if (!fluid(g, nb[0], nb[1], nb[2])) continue;
                        s += (p[id] - p[cidx(g, nb[0], nb[1], nb[2])]) * ih2[d];
                    }
                q[id] = s;
            }
}

/* dot product of FP32 vectors accumulated in FP64 (products are exact) */
static double dot32(const og_grid *g, const float *a, const float *b) {
    size_t n = ncells(g);
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += (double)a[i] * (double)b[i];
    return s;
}

/* Jacobi-PCG in FP32 for A e = r from e = 0, until ||r_k|| <= eta ||r_0||
 * or maxit iterations.  Returns the iteration count. */
static int pcg32(const og_grid *g, const float *dg, const float *rhs, float *e, double eta, int maxit) {
    size_t n = ncells(g);
    float *r = malloc(n * sizeof(float)), *z = malloc(n * sizeof(float));
    float *d = malloc(n * sizeof(float)), *q = malloc(n * sizeof(float));
    for (size_t i = 0; i < n; ++i) {
        e[i] = 0.0f;
        r[i] = rhs[i];
        z[i] = dg[i] > 0.0f ? r[i] / dg[i] : 0.0f;
        d[i] = z[i];
    }
    double rz = dot32(g, r, z);
    double r0 = sqrt(dot32(g, r, r));
    double rnorm = r0;
    int it = 0;
    while (rnorm > eta * r0 && it < maxit && isfinite(rnorm)) {
        apply_A32(g, d, q);
        float alpha = (float)(rz / dot32(g, d, q));
        for (size_t i = 0; i < n; ++i) e[i] += alpha * d[i];
        for (size_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
        for (size_t i = 0; i < n; ++i) z[i] = dg[i] > 0.0f ? r[i] / dg[i] : 0.0f;
        double rz_new = dot32(g, r, z);
        float beta = (float)(rz_new / rz);
        rz = rz_new;
        for (size_t i = 0; i < n; ++i) d[i] = z[i] + beta * d[i];
        rnorm = sqrt(dot32(g, r, r));
        ++it;
    }
    free(r); free(z); free(d); free(q);
    return it;
}

/* Defect correction: the FP64 residual r = b - A x is recomputed each
 * sweep; its mean-free FP32 copy is solved to eta by FP32 Jacobi-PCG and the
 * correction is added in FP64, until ||r||_2 <= rtol ||b||_2. */
int og_pcg_mixed(const og_grid *g, const double *b, double *x, double rtol, double eta, int maxit,
                 int max_outer, og_info *info) {
    size_t n = ncells(g);
    double *r = malloc(n * sizeof(double)), *dg = malloc(n * sizeof(double));
    float *dg32 = malloc(n * sizeof(float)), *r32 = malloc(n * sizeof(float)), *e = malloc(n * sizeof(float));
    diag_A(g, dg);
    for (size_t i = 0; i < n; ++i) dg32[i] = (float)dg[i];
    memset(info, 0, sizeof(*info));
    double bnorm = sqrt(dot(g, b, b));
    int status = 0, inner = 0, outer = 0;
    double rel = 0.0;
    if (bnorm == 0.0) {
        for (size_t i = 0; i < n; ++i) x[i] = 0.0;
    } else {
        cold_start_if_worse(g, b, x, r);
        for (;;) {
            og_apply_A(g, x, r);
            for (size_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
            double rnorm = sqrt(dot(g, r, r));
            rel = rnorm / bnorm;
            if (!isfinite(rnorm)) { status = 3; break; }
            if (rnorm <= rtol * bnorm) break;
            if (outer >= max_outer) { status = 2; break; }
            double m = mean_fluid(g, r);
            for (size_t i = 0; i < n; ++i) r32[i] = is_fluid_id(g, i) ? (float)(r[i] - m) : 0.0f;
            inner += pcg32(g, dg32, r32, e, eta, maxit);
            for (size_t i = 0; i < n; ++i) x[i] += (double)e[i];
            ++outer;
        }
        subtract_mean(g, x);
    }
    info->iters = inner;
    info->outer = outer;
    info->status = status;
    info->rel_res_true = rel;
    free(r); free(dg); free(dg32); free(r32); free(e);
    return status;
}

/* Mixed precision that keeps its Krylov space: FP32 Jacobi-PCG on the
 * correction e of the FP64 iterate x, with reliable updates (Sleijpen & van
 * der Vorst 1996).  The FP32 recursive residual drifts from b - A(x + e) by
 * FP32 rounding; whenever it has fallen by the factor delta below its norm
 * at the last update (or below rtol ||b||, or the iteration limit is hit),
 * e is added to x in FP64, the FP64 residual b - A x is recomputed, tested
 * against rtol ||b||, and its mean-free FP32 copy replaces the recursive
 * residual.  The search direction d is kept across the update, so CG goes
 * on in the same Krylov space instead of restarting:
 *   start:   r = b - A x, rt = fp32(r - mean r), e = 0, z = M^-1 rt, d = z
 *   step:    q = A d, alpha = <rt,z>/<d,q>, e += alpha d, rt -= alpha q,
 *            z = M^-1 rt;  [update: x += e, e = 0, r = b - A x, stop if
 *            ||r|| <= rtol ||b||, rt = fp32(r - mean r), z = M^-1 rt]
 *            beta = <rt,z>_new / <rt,z>_old, d = z + beta d
 * Inner products in FP64 from FP32 values (products exact), alpha and beta
 * rounded to FP32 as in pcg32.  outer counts the updates (at most
 * max_updates), iters the FP32 iterations. */
int og_pcg_mixed_ru(const og_grid *g, const double *b, double *x, double rtol, double delta, int maxit,
                    int max_updates, og_info *info) {
    size_t n = ncells(g);
    double *r = malloc(n * sizeof(double)), *dg = malloc(n * sizeof(double));
    float *dg32 = malloc(n * sizeof(float)), *rt = malloc(n * sizeof(float)), *e = malloc(n * sizeof(float));
    float *z = malloc(n * sizeof(float)), *d = malloc(n * sizeof(float)), *q = malloc(n * sizeof(float));
    diag_A(g, dg);
    for (size_t i = 0; i < n; ++i) dg32[i] = (float)dg[i];
    memset(info, 0, sizeof(*info));
    double bnorm = sqrt(dot(g, b, b));
    int status = 0, it = 0, updates = 0;
    double rel = 0.0;
    if (bnorm == 0.0) {
        for (size_t i = 0; i < n; ++i) x[i] = 0.0;
        goto done;
    }
    cold_start_if_worse(g, b, x, r);
    /* FP64 residual of x; 1 when it meets the tolerance */
    og_apply_A(g, x, r);
    for (size_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double rnorm = sqrt(dot(g, r, r));
    rel = rnorm / bnorm;
    if (!isfinite(rnorm)) { status = 3; goto fold; }
    if (rnorm <= rtol * bnorm) goto fold;
    for (size_t i = 0; i < n; ++i) e[i] = 0.0f;
    double m = mean_fluid(g, r);
    for (size_t i = 0; i < n; ++i) rt[i] = is_fluid_id(g, i) ? (float)(r[i] - m) : 0.0f;
    for (size_t i = 0; i < n; ++i) { z[i] = dg32[i] > 0.0f ? rt[i] / dg32[i] : 0.0f; d[i] = z[i]; }
    double rho = dot32(g, rt, z);
    double rlast = sqrt(dot32(g, rt, rt));
    for (;;) {
        apply_A32(g, d, q);
        float alpha = (float)(rho / dot32(g, d, q));
        for (size_t i = 0; i < n; ++i) e[i] += alpha * d[i];
        for (size_t i = 0; i < n; ++i) rt[i] -= alpha * q[i];
        for (size_t i = 0; i < n; ++i) z[i] = dg32[i] > 0.0f ? rt[i] / dg32[i] : 0.0f;
        double rho_new = dot32(g, rt, z);
        double rn = sqrt(dot32(g, rt, rt));
        ++it;
        if (rn <= delta * rlast || rn <= rtol * bnorm || it >= maxit || !isfinite(rn)) {
            /* reliable update */
            for (size_t i = 0; i < n; ++i) x[i] += (double)e[i];
            for (size_t i = 0; i < n; ++i) e[i] = 0.0f;
            ++updates;
            og_apply_A(g, x, r);
            for (size_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
            rnorm = sqrt(dot(g, r, r));
            rel = rnorm / bnorm;
            if (!isfinite(rnorm)) { status = 3; break; }
            if (rnorm <= rtol * bnorm) break;
            if (updates >= max_updates || it >= maxit) { status = 2; break; }
            m = mean_fluid(g, r);
            for (size_t i = 0; i < n; ++i) rt[i] = is_fluid_id(g, i) ? (float)(r[i] - m) : 0.0f;
            for (size_t i = 0; i < n; ++i) z[i] = dg32[i] > 0.0f ? rt[i] / dg32[i] : 0.0f;
            rho_new = dot32(g, rt, z);
            rlast = sqrt(dot32(g, rt, rt));
        }
        float beta = (float)(rho_new / rho);
        rho = rho_new;
        for (size_t i = 0; i < n; ++i) d[i] = z[i] + beta * d[i];
    }
fold:
    subtract_mean(g, x);
done:
    info->iters = it;
    info->outer = updates;
    info->status = status;
    info->rel_res_true = rel;
    free(r); free(dg); free(dg32); free(rt); free(e); free(z); free(d); free(q);
    return status;
}

/* ------------------------------------------------- correction and step */

/* u = F - dt G p on open faces, 0 on closed faces. */
void og_correct(const og_grid *g, const double *Fu, const double *Fv, const double *Fw, const double *p,
                double dt, double *u, double *v, double *w) {
    const double *F[3] = {Fu, Fv, Fw};
    double *out[3] = {u, v, w};
    for (int c = 0; c < 3; ++c) {
        int ex = fext(g, c, 0), ey = fext(g, c, 1), ez = fext(g, c, 2);
#pragma omp parallel for schedule(static)
        for (int k = 0; k < ez; ++k)
            for (int j = 0; j < ey; ++j)
                for (int i = 0; i < ex; ++i) {
                    int f[3] = {i, j, k};
                    size_t id = fidx(g, c, f), od = fidx_raw(g, c, f);
                    if (!face_open(g, c, f)) { out[c][od] = 0.0; continue; }
                    int lo[3] = {i, j, k};
                    lo[c] -= 1;
                    double gp = (p[cidx(g, i, j, k)] - p[cidx(g, lo[0], lo[1], lo[2])]) / hdir(g, c);
                    out[c][od] = F[c][id] - dt * gp;
                }
    }
}

/* Poisson right-hand side of the projection: b = -div(F)/dt, made mean-free
 * over the fluid cells. */
void og_rhs(const og_grid *g, const double *Fu, const double *Fv, const double *Fw, double dt, double *b) {
    og_divergence(g, Fu, Fv, Fw, b);
    size_t n = ncells(g);
    for (size_t i = 0; i < n; ++i) b[i] = -b[i] / dt;
    subtract_mean(g, b);
}

/* nsteps forward-Euler projection steps of size dt, in place on (u,v,w,p).
 * prec 0: FP64 PCG; prec 1: FP32 inner PCG with FP64 defect correction;
 * prec 2: FP32 PCG with reliable updates (eta is delta, max_outer the
 * update limit).
 * iters (optional, nsteps entries) receives the CG iterations per step.
 * Returns the worst status over the steps. */
int og_fine_steps_solver(const og_grid *g, double *u, double *v, double *w, double *p, int nsteps, double dt,
                         int prec, int solver, double rtol, int maxit, double eta, int max_outer, int *iters,
                         double *rel_true);

int og_fine_steps(const og_grid *g, double *u, double *v, double *w, double *p, int nsteps, double dt,
                  int prec, double rtol, int maxit, double eta, int max_outer, int *iters, double *rel_true) {
    return og_fine_steps_solver(g, u, v, w, p, nsteps, dt, prec, 0, rtol, maxit, eta, max_outer, iters, rel_true);
}

int og_fine_steps_ex(const og_grid *g, double *u, double *v, double *w, double *p, int nsteps, double dt,
                     int prec, int solver, double rtol, int maxit, double eta, int max_outer, int extrap,
                     int *iters, double *rel_true);

/* as og_fine_steps; solver 0: Jacobi-PCG (prec 0 FP64, 1 mixed), 1: FP64
 * Jacobi-BiCGStab (prec ignored), 2: single-reduction Jacobi-PCG (FP64) */
int og_fine_steps_solver(const og_grid *g, double *u, double *v, double *w, double *p, int nsteps, double dt,
                         int prec, int solver, double rtol, int maxit, double eta, int max_outer, int *iters,
                         double *rel_true) {
    return og_fine_steps_ex(g, u, v, w, p, nsteps, dt, prec, solver, rtol, maxit, eta, max_outer, 0, iters,
                            rel_true);
}

/* as og_fine_steps_solver.  extrap = 1: the Poisson solve of step s >= 1
 * starts from the linear extrapolation 2 p^s - p^(s-1) of the last two
 * pressures of this call instead of p^s (step 0 starts from the caller's
 * p, as always).  The equation solved and its stopping test are the same,
 * so a step's result is unchanged up to the solver tolerance; only the
 * initial guess, and so the iteration count, differs. */
int og_fine_steps_ex(const og_grid *g, double *u, double *v, double *w, double *p, int nsteps, double dt,
                     int prec, int solver, double rtol, int maxit, double eta, int max_outer, int extrap,
                     int *iters, double *rel_true) {
    size_t nu = og_face_count(g, 0), nv = og_face_count(g, 1), nw = og_face_count(g, 2);
    size_t n = ncells(g);
    double *Fu = malloc(nu * sizeof(double)), *Fv = malloc(nv * sizeof(double));
    double *Fw = malloc(nw * sizeof(double)), *b = malloc(n * sizeof(double));
    double *pprev = extrap ? malloc(n * sizeof(double)) : NULL;
    int worst = 0;
    for (int s = 0; s < nsteps; ++s) {
        og_momentum(g, u, v, w, dt, Fu, Fv, Fw);
        og_rhs(g, Fu, Fv, Fw, dt, b);
        if (extrap) {
            for (size_t c = 0; c < n; ++c) {
                const double ps = p[c];
                if (s > 0) p[c] = 2.0 * ps - pprev[c];
                pprev[c] = ps;
            }
        }
        og_info info;
        int st = solver == 1               ? og_bicgstab(g, b, p, rtol, maxit, &info)
                 : solver == 2 && prec == 0 ? og_pcg_sr(g, b, p, rtol, maxit, &info)
                 : prec == 0                ? og_pcg(g, b, p, rtol, maxit, &info)
                 : prec == 2                ? og_pcg_mixed_ru(g, b, p, rtol, eta, maxit, max_outer, &info)
                                            : og_pcg_mixed(g, b, p, rtol, eta, maxit, max_outer, &info);
        if (st > worst) worst = st;
        if (iters) iters[s] = info.iters;
        if (rel_true) rel_true[s] = info.rel_res_true;
        og_correct(g, Fu, Fv, Fw, p, dt, u, v, w);
    }
    free(Fu); free(Fv); free(Fw); free(b); free(pprev);
    return worst;
}

/* ================================================================ adjoint
 *
 * One forward step is u' = P(M(u; lid)), M(u) = u + dt R(u) on open faces
 * (R = Lap/Re - Conv), P the orthogonal projector onto discretely
 * divergence-free face fields (P = I - G (G^T G)^+ G^T, since D = -G^T).
 * The adjoint of a step, given lam' = dJ/du', is
 *     mu = P lam'                       (P is symmetric: the same projection)
 *     lam = mu + dt (dR/du)^T mu        (this function)
 *     g_lid += dt (dR/dlid)^T mu        (this function)
 * R is piecewise linear in the stencil values: inside each segment of the
 * SMART diagram the face value is a fixed linear combination of U, C, D
 * (slopes (0,1,0) upwind, (-2,3,0) steep, (-1/8,3/4,3/8) QUICK, (0,0,1)
 * capped), and every image value is a linear form in face values and the
 * lid.  The adjoint differentiates the branch the forward step took; where
 * the transport velocity is exactly 0 the flux is identically 0 and
 * contributes nothing.
 */

typedef struct {
    int n;
    size_t idx[4];
    double coef[4];
    double lcoef; /* coefficient of the lid value lid[lidx] */
    size_t lidx;
} og_form;

static void form_face(og_form *F, size_t idx, double coef) {
    F->idx[F->n] = idx;
    F->coef[F->n] = coef;
    F->n++;
}

static int wall_is_lid(const og_grid *g, int c, const int f[3], int d, int s) {
    return c == 0 && d == 1 && s > 0 && f[1] == g->ny - 1;
}

/* the stencil value of stencil_val() as a linear form */
static void stencil_form(const og_grid *g, int c, const int f[3], int d, int m, og_form *F) {
    int s = m > 0 ? 1 : -1;
    int two = (m == 2 || m == -2);
    int f1[3] = {f[0], f[1], f[2]};
    int f2[3] = {f[0], f[1], f[2]};
    f1[d] += s;
    f2[d] += 2 * s;
    size_t i0 = fidx(g, c, f);
    F->n = 0;
    F->lcoef = 0.0;
    F->lidx = (size_t)f[2] * (g->nx + 1) + f[0];
    if (d == c) {
        if (!face_open(g, c, f1)) { if (two) form_face(F, i0, -1.0); return; }
        if (!two) { form_face(F, fidx(g, c, f1), 1.0); return; }
        if (face_open(g, c, f2)) form_face(F, fidx(g, c, f2), 1.0);
        return;
    }
    if (!face_open(g, c, f1)) {
        if (wall_is_lid(g, c, f, d, s)) F->lcoef += 2.0;
        if (!two) { form_face(F, i0, -1.0); return; }
        og_form inner;
        stencil_form(g, c, f, d, -s, &inner);
        for (int k = 0; k < inner.n; ++k) form_face(F, inner.idx[k], -inner.coef[k]);
        F->lcoef -= inner.lcoef;
        return;
    }
    if (!two) { form_face(F, fidx(g, c, f1), 1.0); return; }
    if (!face_open(g, c, f2)) {
        if (wall_is_lid(g, c, f1, d, s)) F->lcoef += 2.0;
        form_face(F, fidx(g, c, f1), -1.0);
        return;
    }
    form_face(F, fidx(g, c, f2), 1.0);
}

/* value of a form (used by the tests to check it against stencil_val) */
double og_stencil_form_value(const og_grid *g, int c, const double *phi, int i, int j, int k, int d, int m) {
    int f[3] = {i, j, k};
    og_form F;
    stencil_form(g, c, f, d, m, &F);
    double v = 0.0;
    for (int q = 0; q < F.n; ++q) v += F.coef[q] * phi[F.idx[q]];
    return v + F.lcoef * g->lid[F.lidx];
}

double og_stencil_value(const og_grid *g, int c, const double *phi, int i, int j, int k, int d, int m) {
    int f[3] = {i, j, k};
    return stencil_val(g, c, phi, f, d, m);
}

/* slopes of the SMART face value with respect to U, C, D on the branch
 * og_smart takes */
static void smart_slopes(double U, double C, double D, double s[3]) {
    double delta = D - U;
    s[0] = 0.0; s[1] = 1.0; s[2] = 0.0;
    if (delta == 0.0) return;
    double ph = (C - U) / delta;
    if (ph > 0.0 && ph < 1.0 / 6.0) { s[0] = -2.0; s[1] = 3.0; s[2] = 0.0; }
    else if (ph >= 1.0 / 6.0 && ph < 5.0 / 6.0) { s[0] = -0.125; s[1] = 0.75; s[2] = 0.375; }
    else if (ph >= 5.0 / 6.0 && ph < 1.0) { s[0] = 0.0; s[1] = 0.0; s[2] = 1.0; }
}

static void scatter_form(const og_form *F, double wgt, double *lam, double *glid) {
    for (int q = 0; q < F->n; ++q) lam[F->idx[q]] += wgt * F->coef[q];
    if (F->lcoef != 0.0 && glid) glid[F->lidx] += wgt * F->lcoef;
}

static double form_value(const og_form *F, const double *phi, const double *lid) {
    double v = 0.0;
    for (int q = 0; q < F->n; ++q) v += F->coef[q] * phi[F->idx[q]];
    return v + F->lcoef * lid[F->lidx];
}

/* lam = mu + dt (dR/du)^T mu, g_lid += dt (dR/dlid)^T mu, with R evaluated at
 * (u, v, w).  mu is read on open faces only; lam is written on every face
 * (0 on closed faces).  Serial loops: the scatter order is fixed. */
void og_momentum_adjoint(const og_grid *g, const double *u, const double *v, const double *w, double dt,
                         const double *mu_u, const double *mu_v, const double *mu_w, double *lam_u, double *lam_v,
                         double *lam_w, double *g_lid) {
    const double *vel[3] = {u, v, w};
    const double *mu[3] = {mu_u, mu_v, mu_w};
    double *lam[3] = {lam_u, lam_v, lam_w};
    for (int c = 0; c < 3; ++c) {
        size_t nf = og_face_count(g, c);
        for (size_t id = 0; id < nf; ++id) lam[c][id] = 0.0;
    }
    for (int c = 0; c < 3; ++c) {
        int ex = fext(g, c, 0), ey = fext(g, c, 1), ez = fext(g, c, 2);
        for (int k = 0; k < ez; ++k)
            for (int j = 0; j < ey; ++j)
                for (int i = 0; i < ex; ++i) {
                    int f[3] = {i, j, k};
                    if (!face_open(g, c, f)) continue;
                    size_t i0 = fidx(g, c, f);
                    double m0 = mu[c][i0];
                    lam[c][i0] += m0;
                    if (m0 == 0.0) continue;
                    og_form self;
                    self.n = 0;
                    self.lcoef = 0.0;
                    self.lidx = 0;
                    form_face(&self, i0, 1.0);
                    for (int d = 0; d < 3; ++d) {
                        double h = hdir(g, d);
                        og_form Vm2, Vm1, Vp1, Vp2;
                        stencil_form(g, c, f, d, -2, &Vm2);
                        stencil_form(g, c, f, d, -1, &Vm1);
                        stencil_form(g, c, f, d, 1, &Vp1);
                        stencil_form(g, c, f, d, 2, &Vp2);
                        /* diffusion (v+1 - 2 phi0 + v-1)/h^2 / Re */
                        double wd = dt * m0 / (g->re * h * h);
                        scatter_form(&Vp1, wd, lam[c], g_lid);
                        scatter_form(&Vm1, wd, lam[c], g_lid);
                        lam[c][i0] += -2.0 * wd;
                        /* convection: -(flux(+) - flux(-))/h */
                        for (int s = -1; s <= 1; s += 2) {
                            /* transport velocity: two real face values */
                            size_t a_idx[2];
                            int a_comp, a_open[2];
                            if (d == c) {
                                int f1[3] = {f[0], f[1], f[2]};
                                f1[d] += s;
                                a_comp = c;
                                a_idx[0] = i0; a_open[0] = 1;
                                a_open[1] = face_open(g, c, f1);
                                a_idx[1] = a_open[1] ? fidx(g, c, f1) : 0;
                            } else {
                                int q1[3] = {f[0], f[1], f[2]}, q2[3] = {f[0], f[1], f[2]};
                                if (s > 0) { q1[d] += 1; q2[d] += 1; }
                                q1[c] -= 1;
                                a_comp = d;
                                a_open[0] = face_open(g, d, q1);
                                a_open[1] = face_open(g, d, q2);
                                a_idx[0] = a_open[0] ? fidx(g, d, q1) : 0;
                                a_idx[1] = a_open[1] ? fidx(g, d, q2) : 0;
                            }
                            double a1 = a_open[0] ? vel[a_comp][a_idx[0]] : 0.0;
                            double a2 = a_open[1] ? vel[a_comp][a_idx[1]] : 0.0;
                            double abar = 0.5 * (a1 + a2);
                            if (abar == 0.0) continue;
                            const og_form *U, *C, *D;
                            if (s > 0) {
                                if (abar > 0.0) { U = &Vm1; C = &self; D = &Vp1; }
                                else { U = &Vp2; C = &Vp1; D = &self; }
                            } else {
                                if (abar > 0.0) { U = &Vm2; C = &Vm1; D = &self; }
                                else { U = &Vp1; C = &self; D = &Vm1; }
                            }
                            double Uv = form_value(U, vel[c], g->lid), Cv = form_value(C, vel[c], g->lid),
                                   Dv = form_value(D, vel[c], g->lid);
                            double phis = og_smart(Uv, Cv, Dv);
                            double sl[3];
                            smart_slopes(Uv, Cv, Dv, sl);
                            /* d(-s flux/h) */
                            double wc = -(double)s * dt * m0 / h;
                            if (a_open[0]) lam[a_comp][a_idx[0]] += wc * 0.5 * phis;
                            if (a_open[1]) lam[a_comp][a_idx[1]] += wc * 0.5 * phis;
                            scatter_form(U, wc * abar * sl[0], lam[c], g_lid);
                            scatter_form(C, wc * abar * sl[1], lam[c], g_lid);
                            scatter_form(D, wc * abar * sl[2], lam[c], g_lid);
                        }
                    }
                }
    }
    /* closed faces carry no adjoint */
    for (int c = 0; c < 3; ++c) {
        int ex = fext(g, c, 0), ey = fext(g, c, 1), ez = fext(g, c, 2);
        for (int k = 0; k < ez; ++k)
            for (int j = 0; j < ey; ++j)
                for (int i = 0; i < ex; ++i) {
                    int f[3] = {i, j, k};
                    if (!face_open(g, c, f)) lam[c][fidx(g, c, f)] = 0.0;
                }
    }
}
