/*
 * nsp.h - C ABI of the MI355X (gfx950) projection Navier-Stokes / Parareal
 * library (libnsp.so).
 *
 * The library implements the hot path of the space-time Parareal scheme of
 * Croce, Ruprecht & Krause for the 3D incompressible Navier-Stokes equations
 * (Eq. (1)): the fine propagator F and the coarse propagator G, each a
 * sequence of forward-Euler Chorin-Temam projection steps on a uniform
 * staggered grid (Sec. 2, discretization paragraph), the pressure Poisson
 * solve of that projection, and the Parareal update of Eq. (6).
 *
 * Conventions shared by every entry point
 *  - Array arguments are DEVICE pointers owned by the caller, FP64, densely
 *    packed, x fastest.  For a grid of nx*ny*nz cells one slice holds
 *        u [nz][ny][nx+1]   (x-faces)      v [nz][ny+1][nx]   (y-faces)
 *        w [nz+1][ny][nx]   (z-faces)      p [nz][ny][nx]     (cell centres)
 *    and a batch of B slices is B such arrays back to back (batch-major).
 *  - y is the vertical direction; the lid (top face y = ly) moves in +x.
 *  - A face is open when it is interior and both adjacent cells are fluid.
 *    Values stored at closed faces are never read; every call that writes
 *    velocities writes 0 there.
 *  - Every call is enqueued on `stream` (a hipStream_t; NULL = the null
 *    stream) and returns after the stream has finished it, so host outputs
 *    (info, jump) are valid on return.  Calls on one handle must not overlap.
 *  - No C++ exception crosses this boundary.  Every call returns an
 *    nsp_status; nsp_last_error() gives a message for the last failure on a
 *    handle.  On NSP_ERR_NOT_CONVERGED and NSP_ERR_NONFINITE the outputs are
 *    still written (best iterate).
 */
#ifndef NSP_H
#define NSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NSP_OK = 0,
    NSP_ERR_ARG = 1,           /* null pointer, bad size, non-integer step count */
    NSP_ERR_NOT_CONVERGED = 2, /* a Poisson solve hit maxit / max_outer */
    NSP_ERR_NONFINITE = 3,     /* a residual norm became NaN or Inf */
    NSP_ERR_HIP = 4,           /* a HIP runtime call failed */
    NSP_ERR_UNSUPPORTED = 5    /* valid request the library does not implement */
} nsp_status;

typedef enum {
    NSP_FP64 = 0,     /* Jacobi-PCG in FP64 */
    NSP_MIXED = 1,    /* FP32 Jacobi-PCG inner solves, FP64 defect correction (each inner solve
                         restarts CG from the new residual) */
    NSP_MIXED_RU = 2  /* one FP32 Jacobi-PCG run with reliable updates: the FP64 residual replaces
                         the FP32 one whenever it has fallen by inner_rtol, keeping the search
                         direction, so the Krylov space survives the corrections */
} nsp_precision;

typedef enum {
    NSP_PCG = 0,      /* Jacobi-preconditioned CG (A is symmetric positive semi-definite) */
    NSP_BICGSTAB = 1, /* Jacobi-preconditioned BiCGStab, the paper's solver (Sec. 2); FP64 only */
    NSP_PCG_SR = 2    /* the same CG with its inner products merged into one stage per iteration
                         (Chronopoulos & Gear): one grid-wide reduction per iteration instead of
                         two, at 81 instead of 66 bytes per cell; FP64 only */
} nsp_solver;

typedef struct nsp_handle nsp_handle;

/* Grid of one handle.  The domain is [0,lx]x[0,ly]x[0,lz] with nx*ny*nz
 * uniform cells (Sec. 2: uniform Cartesian staggered mesh).  `solid_host`
 * (HOST pointer, nz*ny*nx bytes, nonzero = solid cell, or NULL) is copied at
 * creation: solid cells approximate obstacles by cell enumeration with
 * no-slip walls.  The fluid cells must form one face-connected region.
 * `max_batch` bounds the batch of every later call; workspace for that many
 * slices is allocated at creation.  periodic_z = 0: no-slip walls on all
 * six faces; periodic_z = 1: periodic in z (the boundary condition of the
 * paper's runs, Sec. 3), walls in x and y.  With periodic z the w array keeps
 * its nz+1 planes and the plane at z = lz repeats the plane at z = 0: every
 * call writes both equal, reads use the plane at z = 0.  slip_obstacles = 1
 * makes obstacle surfaces free-slip (an extension: the paper's obstacles are
 * no-slip, Sec. 3): zero normal velocity and zero tangential stress, i.e. the
 * stencil image of a tangential component across an obstacle face is its
 * mirror value instead of minus it; the domain walls and the lid are not
 * obstacles and stay no-slip.  The adjoint refuses such grids
 * (NSP_ERR_UNSUPPORTED); any other value is NSP_ERR_ARG. */
typedef struct {
    int nx, ny, nz;
    double lx, ly, lz;
    double re;               /* Reynolds number of Eq. (1) */
    int periodic_z;          /* 0: walls in z, 1: periodic in z */
    const uint8_t *solid_host;
    int max_batch;
    int slip_obstacles;      /* 0: no-slip obstacle walls (the paper's), 1: free-slip */
} nsp_grid;

/* Poisson solve options.  The solve of A p = b, A = -D G the compatible
 * Neumann Laplacian, stops when ||b - A p||_2 <= rtol ||b||_2 (recursive
 * residual for FP64, recomputed FP64 residual for mixed).  Mixed: each inner
 * FP32 solve stops at relative residual inner_rtol or maxit iterations; at
 * most max_outer inner solves.  Mixed with reliable updates: an update
 * (e folded into p in FP64, FP64 residual recomputed and tested, its FP32
 * copy replacing the recursive residual) whenever the FP32 residual has
 * fallen by inner_rtol since the last one (0.01 is a good value), below
 * rtol ||b||, or at maxit; at most max_outer updates (count them in the
 * dozens: about one per factor inner_rtol of residual reduction); `outer`
 * reports the updates, `iters` the FP32 iterations.  solver NSP_BICGSTAB (FP64 only, else
 * NSP_ERR_UNSUPPORTED): right-preconditioned BiCGStab from the same warm
 * start, restarted from the true residual after a breakdown (at most 16
 * times); its workspace (three vectors per slice) is allocated on first use.
 * `iters` then counts BiCGStab iterations (two products with A each).
 * solver NSP_PCG_SR (FP64 only, else NSP_ERR_UNSUPPORTED): the iterates of
 * NSP_PCG in exact arithmetic, computed with one grid barrier per iteration
 * (the faster choice when a launch is latency-bound, e.g. one slice of up to
 * 128^3 cells); the same workspace as BiCGStab.  Results differ from
 * NSP_PCG's at the solver tolerance, never bit for bit.
 * extrapolate (0 or 1, else NSP_ERR_ARG): in the projection steps of one
 * call (nsp_fine_step, nsp_coarse_step and the sweeps of the Parareal
 * calls), the Poisson solve of every step after the first starts from
 * 2 p^s - p^(s-1), the linear extrapolation of the call's last two
 * pressures, instead of p^s (the warm start of Sec. 2's projection).  The
 * equation and the stopping test are unchanged, so the results agree with
 * extrapolate = 0 to the solver tolerance, not bit for bit; a smoothly
 * developing flow needs about a fifth fewer iterations.  The previous
 * pressure of every slice is kept in a workspace array allocated on first
 * use.  Ignored by nsp_poisson_solve(_noalloc) and by the adjoint entry
 * points (their recomputed steps must repeat the recorded ones). */
typedef struct {
    double rtol;
    int maxit;
    nsp_precision prec;
    double inner_rtol;
    int max_outer;
    nsp_solver solver;
    int extrapolate;
} nsp_poisson_opts;

/* Per-slice report of the last call. */
typedef struct {
    int iters;          /* CG iterations summed over the steps of the call (inner ones for mixed) */
    int max_iters;      /* largest per-step CG iteration count */
    int outer;          /* FP64 restarts, or mixed defect-correction sweeps, summed */
    int status;         /* worst nsp_status over the steps of this slice */
    double rel_res_true;/* ||b - A p|| / ||b|| of the last solve, recomputed in FP64 */
    double div_l2;      /* ||D u||_2 after the last step (= dt * ||b - A p||_2) */
} nsp_solve_info;

/* A batch of states (u, v, w, p); layout above.  Every call taking a batch
 * accepts batch 0 as a no-op (NSP_OK, nothing read or written; the pointers
 * may then be NULL); a batch below 0 or above max_batch is NSP_ERR_ARG. */
typedef struct {
    double *u, *v, *w, *p;
} nsp_state;

/* Create a handle: copies the grid and the solid mask to the device, sets
 * the lid to u = 1 (Sec. 3, both simulations), allocates workspace for
 * max_batch slices.  Returns NSP_ERR_ARG for non-positive sizes, a
 * max_batch outside 1..64 or fluid cells that are not face-connected
 * (across the z seam too when periodic). */
nsp_status nsp_create(const nsp_grid *grid, nsp_handle **out);
/* nsp_destroy waits for the device and frees the handle and all its
 * workspace (records of nsp_fine_solve_record included); destroy the
 * handle's graphs first.  NSP_ERR_ARG for a NULL handle.
 * nsp_last_error: the message of the handle's last failed call ("null
 * handle" for NULL), owned by the handle and valid until its next call. */
nsp_status nsp_destroy(nsp_handle *h);
const char *nsp_last_error(const nsp_handle *h);

/* Lid: the wall value of u on the top face, one value per top u-face
 * position, DEVICE array [nz][nx+1] (entries at i = 0 and i = nx are
 * unused).  Copied on `stream` (so a lid written by earlier work on that
 * stream is seen); returns after the copy. */
nsp_status nsp_set_lid(nsp_handle *h, const double *lid_dev, void *stream);

/* Pressure Poisson solve of the projection step (Sec. 2): A p = b for a
 * batch of right-hand sides.  b: [batch] cell arrays, first made mean-free
 * over the fluid cells (the Neumann problem needs it); not modified.
 * p: [batch] cell arrays, initial guess on entry, solution on exit with
 * mean_fluid(p) = 0.  info: HOST array of `batch` entries, or NULL. */
nsp_status nsp_poisson_solve(nsp_handle *h, const double *b, double *p, int batch,
                             const nsp_poisson_opts *opts, void *stream, nsp_solve_info *info);

/* nsp_poisson_solve for callers that cannot allocate device memory: tight
 * serving loops and harnesses that forbid allocation (like every call it
 * synchronises `stream` to read the solve's status, so it cannot itself be
 * recorded into a graph).  Same
 * arguments, kernels and results (bitwise) as nsp_poisson_solve, but every
 * scratch buffer of the solve (launch parameters, barrier words, per-slice
 * control blocks, partial sums, the right-hand-side copy and the CG vectors)
 * lives in one fixed device array of 96 MiB inside the library, which each
 * GPU it runs on holds until the process ends; the call allocates nothing.
 * Needed: 44 bytes per cell and slice (PCG, FP64 or mixed) or 68 (BiCGStab,
 * single-reduction PCG), plus a few hundred KiB: one 128^3 slice or two
 * 96^3 slices in PCG.  A solve
 * that needs more returns NSP_ERR_ARG with the size in nsp_last_error; the
 * current device must be the handle's.  Every call on one GPU shares that
 * GPU's array (it keeps the last call's contents; the call clears what must
 * start at zero), so calls that overlap on one GPU, on any handles or
 * streams, race: serialise them. */
nsp_status nsp_poisson_solve_noalloc(nsp_handle *h, const double *b, double *p, int batch,
                                     const nsp_poisson_opts *opts, void *stream, nsp_solve_info *info);

/* Fine propagator F(y, t1, t0) of Sec. 2.1.2: (t1 - t0)/dt forward-Euler
 * projection steps, in place on the batch y.  (t1 - t0)/dt must be a
 * non-negative integer to 1e-9 relative (NSP_ERR_ARG otherwise).  Each step:
 * predictor with SMART convection and central diffusion, Poisson solve
 * (warm-started from y.p), velocity correction. */
nsp_status nsp_fine_step(nsp_handle *h, nsp_state y, int batch, double t0, double t1, double dt,
                         const nsp_poisson_opts *opts, void *stream, nsp_solve_info *info);

/* The fine propagator as a replayable HIP graph: the batched fine sweep of
 * Sec. 2.1.2 (all slices of y in one persistent launch) recorded once and
 * replayed without host synchronisation.  nsp_fine_step_graph_create
 * records what nsp_fine_step(h, y, batch, t0, t1, dt, opts) would launch:
 * the graph holds the kernels that clear its control blocks and barrier
 * words, the persistent kernel (a cooperative node) and a kernel that folds
 * each replay's per-slice results into words the graph keeps.  The state
 * pointers y, the batch, the step count (t1 - t0)/dt (a positive integer,
 * else NSP_ERR_ARG), dt and *opts are fixed at creation; the launch shape
 * is the one nsp_fine_step would pick (nsp_autotune results included).  The
 * graph owns its parameter block, control blocks, partial sums and barrier
 * words, and shares the handle's workspace vectors, so eager calls on the
 * handle may run between replays on the same stream.  Creation is
 * synchronous and allocates; *out receives the graph.
 * nsp_graph_launch enqueues one replay on `stream` (asynchronous: y advances
 * by (t1 - t0)/dt steps when it runs; nothing is read back).
 * nsp_graph_finish synchronises `stream` and reports every replay since the
 * previous finish (with none it returns NSP_OK and leaves info as it is):
 * info (HOST, `batch` entries, or NULL) gets per slice the
 * summed CG iterations and sweeps, the most iterations of one step, the
 * worst status and the last replay's true residual; the return value is the
 * worst status (NSP_ERR_NOT_CONVERGED, NSP_ERR_NONFINITE, or NSP_ERR_HIP if
 * a replay abandoned a barrier wait).  Replays run the same kernels on the
 * same inputs as nsp_fine_step and give bitwise its results.
 * nsp_graph_destroy waits for the device and frees the graph; destroy a
 * graph before its handle. */
typedef struct nsp_graph nsp_graph;
nsp_status nsp_fine_step_graph_create(nsp_handle *h, nsp_state y, int batch, double t0, double t1, double dt,
                                      const nsp_poisson_opts *opts, nsp_graph **out);
nsp_status nsp_graph_launch(nsp_graph *g, void *stream);
nsp_status nsp_graph_finish(nsp_graph *g, void *stream, nsp_solve_info *info);
nsp_status nsp_graph_destroy(nsp_graph *g);

/* Coarse propagator G(y, t1, t0): the same scheme with the coarse step DT
 * (Sec. 2.1.2: forward Euler for both, larger step for G), with the
 * convection chosen by nsp_set_coarse_convection. */
nsp_status nsp_coarse_step(nsp_handle *h, nsp_state y, int batch, double t0, double t1, double DT,
                           const nsp_poisson_opts *opts, void *stream, nsp_solve_info *info);

/* Convection of the coarse propagator: the fine scheme's SMART (default) or
 * first-order upwind (donor cell: a convective face carries the value at the
 * node on its upwind side).  The paper runs G with the fine scheme and
 * leaves other coarse propagators to future work (Sec. 2.1.2); a
 * first-order G damps where SMART's forward-Euler steps amplify.  Applies to
 * nsp_coarse_step and to the coarse sweeps of the Parareal calls made with
 * this handle (for nsp_parareal_*_cgrid: the coarse handle's setting);
 * fine steps always use SMART.  NSP_ERR_ARG for another value. */
typedef enum { NSP_CONV_SMART = 0, NSP_CONV_UPWIND = 1 } nsp_convection;
nsp_status nsp_set_coarse_convection(nsp_handle *h, nsp_convection scheme);

/* Uneven batch: F over several grids in ONE launch.  hs[g] is the handle of
 * grid g, ys[g] its batch of batches[g] slices (groups with batches[g] = 0
 * take no part).  The launch uses hs[0]'s synchronisation words; all handles
 * must live on the same device. */
nsp_status nsp_group_fine_step(nsp_handle *const *hs, const nsp_state *ys, const int *batches, int ngroups,
                               double t0, double t1, double dt, const nsp_poisson_opts *opts, void *stream,
                               nsp_solve_info *info);

/* Parareal, Eq. (6), on nslices slices of [t0, T] (slice length
 * (T - t0)/nslices; fine steps dt and coarse steps DT per slice must be
 * integers).
 *   Y  : nslices+1 slice-end states; Y[0] is the initial value.
 *   Gk : nslices states, Gk[n] = G(Y[n]) of the previous sweep.
 *   Fk : nslices states of workspace receiving F(Y[n]).
 * nsp_parareal_start runs the initial coarse sweep Y[n+1] = G(Y[n]) and
 * fills Gk.  nsp_parareal_iterate performs iteration k (k = 0, 1, ...):
 * F(Y[n]) for all slices n >= k in one batched launch (slices n < k are
 * already exact), then the serial sweep n = k .. nslices-1:
 *   g = G(Ynew[n]);  Ynew[n+1] = F(Y[n]) + (g - Gk[n]);  Gk[n] = g.
 * jump (HOST, 2 doubles): max over slices and grid points of
 * |Ynew - Y| for (u,v,w) and for p.  The handle needs max_batch >=
 * nslices.  When a fine or coarse Poisson solve hits maxit / max_outer the
 * iteration still completes with that solve's best iterate (Y, Gk and jump
 * are written) and the call returns NSP_ERR_NOT_CONVERGED; any other error
 * stops it at once.  nsp_parareal_start reports coarse solves the same way.
 * Poisson solves of every verb start from the state's p unless that warm
 * start is worse than none (||b - A p|| > ||b||), then from p = 0. */
nsp_status nsp_parareal_start(nsp_handle *h, nsp_state Y, nsp_state Gk, int nslices, double t0, double T,
                              double DT, const nsp_poisson_opts *coarse, void *stream);
nsp_status nsp_parareal_iterate(nsp_handle *h, nsp_state Y, nsp_state Fk, nsp_state Gk, int nslices, int k,
                                double t0, double T, double dt, double DT, const nsp_poisson_opts *fine,
                                const nsp_poisson_opts *coarse, void *stream, double *jump);

/* Uneven-batch Parareal: iteration k over ngroups grids, F of all grids'
 * slices in one launch, the coarse sweep batched across grids slice by
 * slice.  Array arguments are indexed by group; jump receives 2 doubles per
 * group. */
nsp_status nsp_group_parareal_start(nsp_handle *const *hs, const nsp_state *Y, const nsp_state *Gk, int ngroups,
                                    int nslices, double t0, double T, double DT, const nsp_poisson_opts *coarse,
                                    void *stream);
nsp_status nsp_group_parareal_iterate(nsp_handle *const *hs, const nsp_state *Y, const nsp_state *Fk,
                                      const nsp_state *Gk, int ngroups, int nslices, int k, double t0, double T,
                                      double dt, double DT, const nsp_poisson_opts *fine,
                                      const nsp_poisson_opts *coarse, void *stream, double *jump);

/* Coarser-grid coarse propagator.  The paper runs G on the fine grid with a
 * larger step and leaves other coarse propagators to future work (Sec.
 * 2.1.2).  Here G~(y) = P(G_c(R(y))): G_c is the projection step of
 * Sec. 2 on the grid of the coarse handle hc, which must have half the
 * cells of h in every direction (nx, ny, nz of h even), the same box and the
 * same z boundary, and neither grid may hold obstacles (else
 * NSP_ERR_UNSUPPORTED; a size or box mismatch is NSP_ERR_ARG).  Fine cell
 * (k, j, i) lies in coarse cell (k/2, j/2, i/2).
 *   R (nsp_restrict): a coarse face value is the mean of the four fine faces
 *     tiling it (so the flux through it, and the discrete divergence, are
 *     kept); a coarse pressure is the mean of its eight fine cells.
 *   P (nsp_prolong): a fine face inside a coarse face takes its value; a
 *     fine face halfway between two coarse faces takes their mean; a fine
 *     cell takes its coarse cell's pressure.  R(P(y)) = y, and P keeps a
 *     divergence-free field (zero normal velocity on the walls)
 *     divergence-free.
 * yf / yc: DEVICE states of `batch` slices on the fine / coarse grid
 * (caller-owned, layout as nsp_state); the output is overwritten, nothing is
 * allocated.  nsp_parareal_start_cgrid / nsp_parareal_iterate_cgrid are
 * nsp_parareal_start / nsp_parareal_iterate with G~ in place of G: Y, Fk and
 * Gk stay fine-grid states (Gk[n] = G~(Y[n]) of the previous sweep), coarse
 * steps of size DT run on hc (its Reynolds number and lid), and the update
 * of Eq. (6) and its exactness after nslices iterations are unchanged. */
nsp_status nsp_restrict(nsp_handle *h, nsp_handle *hc, nsp_state yf, nsp_state yc, int batch, void *stream);
nsp_status nsp_prolong(nsp_handle *h, nsp_handle *hc, nsp_state yc, nsp_state yf, int batch, void *stream);
nsp_status nsp_parareal_start_cgrid(nsp_handle *h, nsp_handle *hc, nsp_state Y, nsp_state Gk, int nslices,
                                    double t0, double T, double DT, const nsp_poisson_opts *coarse, void *stream);
nsp_status nsp_parareal_iterate_cgrid(nsp_handle *h, nsp_handle *hc, nsp_state Y, nsp_state Fk, nsp_state Gk,
                                      int nslices, int k, double t0, double T, double dt, double DT,
                                      const nsp_poisson_opts *fine, const nsp_poisson_opts *coarse, void *stream,
                                      double *jump);

/* Adjoint of the fine propagator F (Sec. 2.1.2) for the objective
 *     J = 1/2 hx hy hz sum over open faces of (u_T^2 + v_T^2 + w_T^2),
 * the kinetic energy after nsteps projection steps of size dt from y0
 * (HOST output *J).  With grad.u/v/w non-NULL also writes dJ/d(u0, v0, w0)
 * (DEVICE face arrays, 0 on closed faces) and, if g_lid is non-NULL, dJ/dlid
 * (DEVICE [nz][nx+1], per top u-face lid value).  Each step u' = P(M(u))
 * (M the predictor, P the orthogonal projection of Sec. 2) is reversed as
 * mu = P lam' (the same projection, solved in FP64 to opts->rtol), lam =
 * mu + dt (dR/du)^T mu with the SMART slopes of the branch the forward step
 * took.  Forward states are stored every ckpt_every steps (0: only the
 * initial state) and recomputed segment by segment.  y0 is not modified.
 * The momentum adjoint is a gather (each face sums the transposed
 * contributions of the flux interfaces that read it, in a fixed order), so
 * repeated calls give bitwise equal gradients.  Workspace (checkpoints, one
 * segment) is allocated on first use and kept by the handle.
 * NSP_ERR_UNSUPPORTED on a grid periodic in z or with free-slip obstacles.
 * Equivalent to nsp_fine_solve_record followed by nsp_fine_solve_reverse. */
nsp_status nsp_fine_solve_adjoint(nsp_handle *h, nsp_state y0, int nsteps, double dt, int ckpt_every,
                                  const nsp_poisson_opts *opts, nsp_state grad, double *g_lid, double *J,
                                  void *stream);

/* One reverse momentum step of the adjoint above, on its own:
 *     lam = mu + dt (dR/du)^T mu   on open faces (0 on closed faces),
 *     g_lid += dt (dR/dlid)^T mu   (if g_lid is non-NULL),
 * R the momentum right-hand side of the fine step (Sec. 2: central
 * diffusion, SMART convection with the slopes of the branch taken at vel,
 * image rule at walls and obstacles, the lid above the top row of u) at the
 * velocity vel, with the handle's Reynolds number, obstacles and lid.  vel,
 * mu, lam: DEVICE face arrays of one slice (the p pointers are ignored);
 * g_lid: DEVICE [nz][nx+1], accumulated.  lam must not alias vel or mu
 * (NSP_ERR_ARG).  Asynchronous on `stream`; nothing is allocated.  Each face
 * gathers its contributions in a fixed order (no atomics), so results repeat
 * bitwise.  NSP_ERR_UNSUPPORTED on a grid periodic in z or with free-slip
 * obstacles. */
nsp_status nsp_momentum_adjoint(nsp_handle *h, nsp_state vel, nsp_state mu, nsp_state lam, double *g_lid, double dt,
                                void *stream);

/* The two halves of nsp_fine_solve_adjoint, for callers (an autograd
 * function) whose forward pass runs before they know whether a gradient is
 * wanted.  nsp_fine_solve_record runs the forward sweep from y0 and writes
 * *J (HOST).  With tape non-NULL it also keeps on the handle the checkpoints,
 * dJ/du at the end, nsteps, dt, ckpt_every and a copy of *opts, and writes
 * a nonzero id of this record to *tape (HOST); with tape NULL nothing is
 * kept and only J is computed.  A record replaces the previous one.
 * nsp_fine_solve_reverse runs the reverse sweep of the record `tape` and
 * writes grad (DEVICE face arrays, required) and, if non-NULL, g_lid
 * (DEVICE [nz][nx+1]); the record stays valid, so it may be reversed again.
 * It returns NSP_ERR_ARG without touching the outputs when the record is
 * stale: another record was made on the handle, or nsp_set_lid was called
 * after it.  nsp_fine_solve_tape_valid returns 1 when `tape` may be
 * reversed, else 0 (also for a NULL handle). */
nsp_status nsp_fine_solve_record(nsp_handle *h, nsp_state y0, int nsteps, double dt, int ckpt_every,
                                 const nsp_poisson_opts *opts, double *J, unsigned long long *tape, void *stream);
nsp_status nsp_fine_solve_reverse(nsp_handle *h, unsigned long long tape, nsp_state grad, double *g_lid,
                                  void *stream);
int nsp_fine_solve_tape_valid(const nsp_handle *h, unsigned long long tape);

/* Lid profile from sine modes: lid(x, z) = 1 + sum_{m,n=1..M} c[m-1][n-1]
 * sin(m pi x/lx) sin(n pi z/lz) at the top u-face positions x = i hx,
 * z = (k+1/2) hz.  coef: DEVICE M*M row-major, lid_dev: DEVICE [nz][nx+1].
 * nsp_lid_modes_grad is its transpose: g_coef[m][n] = sum g_lid * basis. */
nsp_status nsp_lid_from_modes(nsp_handle *h, const double *coef, int nmodes, double *lid_dev, void *stream);
nsp_status nsp_lid_modes_grad(nsp_handle *h, const double *g_lid, int nmodes, double *g_coef, void *stream);

/* Launch statistics of the persistent kernel, per launch kind: [0] fine /
 * coarse steps (also the Parareal sweeps), [1] Poisson solves, [2] the
 * projection of the adjoint's reverse step.  Counted since the last reset
 * over every launch this handle made (grouped launches count on the first
 * handle); nsp_autotune's trial launches are not counted.  For measurement:
 * launch durations come from HIP events recorded on the launch stream around
 * each launch.  out: HOST array of 3 entries, or NULL; reset != 0 clears the
 * counters after reading them. */
typedef struct {
    long long launches;
    double ms;             /* summed launch durations */
    double cell_steps;     /* sum over launches and slices of cells x steps (x 1 for solves) */
    double cg_cell_iters;  /* sum over slices of cells x Krylov iterations, all kinds */
    double cell_sweeps;    /* sum over slices of cells x defect-correction sweeps / restarts */
    double cg64_cell_iters;   /* the part in FP64 PCG iterations */
    double cg32_cell_iters;   /* the part in FP32 inner PCG iterations (mixed precision) */
    double bicg_cell_iters;   /* the part in BiCGStab iterations */
    double mixed_cell_sweeps; /* the part of cell_sweeps in mixed-precision launches */
    long long rr_launches;    /* launches whose CG vectors stayed in registers: every CG tile had its
                                 own workgroup (results equal the streaming kernel's bit for bit) */
} nsp_launch_stats;
nsp_status nsp_launch_stats_get(nsp_handle *h, nsp_launch_stats out[3], int reset);

/* Launch shape used for a batch: workgroups per launch.  0 = automatic.
 * nsp_autotune times candidate shapes on the handle's own workspace (a
 * 40-iteration Poisson solve on a synthetic right-hand side): workgroup
 * counts and, where the CG phases use column tiles, tile depths from the
 * grid's partial block (8 planes, or 4 where one slice has fewer 8-plane
 * tiles than the GPU has workgroups) up to 32 planes and (NSP_MIXED) one or
 * two rows per thread; it keeps the fastest for (batch, prec) and reports it
 * in *chosen_workgroups, *chosen_planes and *chosen_items (0 for flat tiles;
 * each may be NULL).  Results do not depend on the choice: partial sums are
 * kept per tile, or per block of rows and 4 or 8 planes fixed for the grid.
 * It allocates and frees two batch-sized device arrays and synchronises the
 * stream. */
nsp_status nsp_set_launch(nsp_handle *h, int workgroups);
nsp_status nsp_autotune(nsp_handle *h, int batch, nsp_precision prec, void *stream, int *chosen_workgroups,
                        int *chosen_planes, int *chosen_items);

/* Duration in milliseconds of the last persistent launch made through this
 * handle, measured with HIP events on the launch stream. */
nsp_status nsp_last_launch_ms(const nsp_handle *h, double *ms);

#ifdef __cplusplus
}
#endif
#endif /* NSP_H */
