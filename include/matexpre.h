/*
 * matexpre.h -- C ABI of the MatExPre hot path on one AMD MI355X (gfx950).
 *
 * The library solves the discrete Helmholtz problem
 *
 *     omega^2/c(x)^2 u + Lap_PML u = -f                      (paper Section 1, eq. helmholtz)
 *
 * on a structured 2D (five-point) or 3D (seven-point) node grid whose outer
 * cells form a perfectly matched layer with the quadratic stretch
 * s(x) = 1 + i C_pml/(delta omega) (dist/delta)^2 on every axis
 * (Section 3.3, eq. pml-1d-s; Section 4 introduction), zero Dirichlet values
 * beyond the grid.  It uses flexible GMRES preconditioned by MatExPre
 * (Section 3.4, Algorithm 1): for a residual r,
 *
 *     r_hat = psi_1(i t A_s) r,   then GMRES on (I - exp(i t A_s)) w = r_hat
 *     to relative tolerance fprtol, return w,
 *
 * with the complex-shifted operator A_s = A + i omega^2 s D, D = diag(1/c^2)
 * (Section 3.4).  The matrix-function actions are evaluated by substepped
 * Chebyshev expansions on HIP kernels.
 *
 * Conventions shared by every call
 * --------------------------------
 *  Layout    Grid vectors hold n0*n1*n2 complex values (n2 = 1 in 2D),
 *            interleaved (re, im), index i + n0*(j + n1*k), x fastest; the
 *            same layout as C99 _Complex and torch.complex64/complex128.
 *  Pointers  Vector arguments (f, u, x, y, r, w) are DEVICE pointers on the
 *            context's device, caller-owned, valid for the duration of the
 *            call, and must not overlap unless a call says otherwise.  The
 *            wave-speed array c may be a host or a device pointer.
 *  Streams   All device work is enqueued on the stream given to
 *            mxp_context_create (NULL = the null stream).  Every call returns
 *            only after its work has completed, so outputs and statistics are
 *            valid on return.
 *  Errors    Calls return mxp_status.  Arguments are validated before any
 *            device work; a negative status means nothing usable was written.
 *            MXP_NOT_CONVERGED (positive) means the iteration limit was hit:
 *            u holds the last iterate and the statistics are filled in.
 *            mxp_last_error() gives a message for the last failing call on the
 *            calling thread.  No C++ exception crosses this interface.
 *  Threads   A context (and its problems) is used by one host thread at a
 *            time.
 */
#ifndef MATEXPRE_H
#define MATEXPRE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MXP_OK = 0,
    MXP_NOT_CONVERGED = 1,
    MXP_ERR_INVALID_ARG = -1,
    MXP_ERR_OOM = -2,
    MXP_ERR_HIP = -3,
    MXP_ERR_BREAKDOWN = -4,
    MXP_ERR_NONFINITE = -5,
    MXP_ERR_UNSUPPORTED = -6
} mxp_status;

typedef enum {
    MXP_C64 = 0,   /* complex float  (8 bytes per value)  */
    MXP_C128 = 1,  /* complex double (16 bytes per value) */
    MXP_F32 = 2,   /* real float  (wave speed only)       */
    MXP_F64 = 3    /* real double (wave speed only)       */
} mxp_dtype;

typedef enum {
    MXP_PREC_FP64 = 0,  /* every step in complex double                              */
    MXP_PREC_MIXED = 1  /* matrix-function actions and the inner GMRES basis in       */
                        /* complex float; Gram-Schmidt sums, Hessenberg, the outer    */
                        /* FGMRES bases, true residual and outer iteration in double  */
} mxp_precision;

typedef struct mxp_context mxp_context;
typedef struct mxp_problem mxp_problem;

/* ---------------------------------------------------------------- context */

/* Device-memory hooks.  alloc returns `bytes` of device memory on the
 * context's device (NULL on failure, which the library reports as OOM);
 * release gives back a pointer alloc returned.  `user` is passed through.
 * The library calls them from the calling thread, or from the worker
 * threads of mxp_solve_batch, and only for memory whose device work has
 * completed when it is released (every call is synchronous on return), so a
 * stream-ordered caching allocator such as PyTorch's may recycle it at once. */
typedef void* (*mxp_alloc_fn)(size_t bytes, void* user);
typedef void (*mxp_free_fn)(void* ptr, void* user);

/* Binds `device` and borrows `hip_stream` (a hipStream_t, or NULL for the
 * null stream) for all later work.  Every device buffer the library keeps
 * (problem tables, solver workspaces, network state) is taken through
 * alloc / release, both NULL for hipMalloc / hipFree; the two must be given
 * together.  A call reserves what it needs when it starts (problem set-up at
 * mxp_problem_create, workspaces at the entry of a solve, an action or a
 * preconditioner apply), never in the middle of its device work; buffers are
 * kept with the problem for later calls and released by the destroy calls.
 * The hooks and `user` must stay valid until every problem and network made
 * on the context is destroyed.  *out receives the context.
 * Errors: INVALID_ARG (no such device, out == NULL, only one hook), HIP. */
mxp_status mxp_context_create(int device, void* hip_stream, mxp_alloc_fn alloc, mxp_free_fn release,
                              void* user, mxp_context** out);

/* Device allocations made through a context and the problems and networks
 * created on it: calls of alloc and release, bytes held now and at most, and
 * `late`, the allocations a call made after it had reserved its workspace
 * (zero unless a buffer was missed by the reservation). */
typedef struct {
    int64_t allocs, frees;
    int64_t bytes_live, bytes_peak;
    int64_t late;
} mxp_alloc_stats;
mxp_status mxp_context_alloc_stats(const mxp_context* ctx, mxp_alloc_stats* out);

/* Frees the context.  Problems created on it must be destroyed first. */
void mxp_context_destroy(mxp_context* ctx);

/* Message for the last failing call on this thread ("" if none).  The
 * pointer stays valid until the next call on this thread. */
const char* mxp_last_error(void);

/* Library version string.  It is part of the key of the autotuner cache
 * (MXP_AUTOTUNE_CACHE), so choices cached by another version are re-timed. */
const char* mxp_version(void);

/* ---------------------------------------------------------------- problem */

/* The problem statement (Section 1 eq. helmholtz; Section 3.3 eq. pml-1d-s;
 * Section 4 introduction).  Node x_i = i*h on every axis.  layer[d][0/1] is
 * the number of absorbing-layer cells on the low/high face of axis d; those
 * are the outermost nodes of the given grid, delta = layer*h, and the stretch
 * distance is measured from the inner edge (layer*h, (n-1-layer)*h).  0 gives
 * a bare Dirichlet face.
 *
 * absorber selects what the layer does.  MXP_ABSORB_PML (0, the default of a
 * zeroed struct) stretches the coordinates, s_d = 1 + i sigma_d(x_d) with
 * sigma_d = pml_C/(delta omega) (dist/delta)^pml_power.  MXP_ABSORB_CAP (1) is
 * the complex absorbing potential of Section 2.1 (eq. helmholtz-absorbing,
 * divided by c^2): the plain Laplacian plus i W/c^2 with
 * W/c^2 = 2 omega^2 sum_d sigma_d(x_d), the same profile, scaled so that a
 * plane wave at normal incidence decays at the PML's rate to first order.
 * Complex-float stepping (MXP_PREC_MIXED, MXP_C64 actions) needs the potential
 * to stay below about the Laplacian's range (pi pml_C / (ppw layer) <= 1.25,
 * ppw the points per wavelength); beyond it schedules fail with UNSUPPORTED.
 *
 * MXP_ABSORB_ABC (2) puts no layer on the grid (every layer width must be 0):
 * each face carries a boundary condition instead, imposed by ghost points as
 * in the paper's Marmousi-II experiment (Section 4.3.4).  hard[d][side] != 0
 * makes the face sound-hard (du/dn = 0); the other faces take the first-order
 * absorbing condition du/dn = i (omega/c) u (outgoing waves e^{i k r}, n the
 * outward normal).  The end nodes of every axis are unknowns: eliminating the
 * ghost node by the central difference of du/dn gives the end row
 * (2 u_inner - 2 u_end)/h^2 + (2 i omega/(c h)) u_end (the last term only on
 * absorbing faces, with c at that node). */
#define MXP_ABSORB_PML 0
#define MXP_ABSORB_CAP 1
#define MXP_ABSORB_ABC 2

typedef struct {
    int32_t dim;            /* 2 or 3                                           */
    int64_t n[3];           /* nodes per axis, x first; n[2] = 1 in 2D; each >= 3 */
    double h;               /* grid spacing, > 0                                */
    double omega;           /* angular frequency, > 0                           */
    int32_t layer[3][2];    /* absorbing cells per face, 0 <= layer < n/2       */
    double pml_C;           /* C_pml (the paper's experiments use 20), >= 0     */
    int32_t pml_power;      /* profile power (2 = quadratic), >= 1              */
    const void* c;          /* wave speed per node (host or device), or NULL    */
    mxp_dtype c_dtype;      /* MXP_F32 or MXP_F64 when c != NULL                */
    double c_const;         /* wave speed everywhere when c == NULL, > 0        */
    int32_t absorber;       /* MXP_ABSORB_PML (default), _CAP or _ABC            */
    int32_t hard[3][2];     /* MXP_ABSORB_ABC: nonzero = sound-hard face (low / high
                               side of each axis); the other faces absorb      */
} mxp_grid_desc;

/* Copies the description, validates it (c finite and > 0 everywhere), builds
 * the per-axis absorbing-layer coefficient tables and D = 1/c^2 on the
 * device.  The library owns everything it allocates; mxp_problem_destroy
 * frees it.  The caller's c may be freed after this call returns.
 * Errors: INVALID_ARG (any bound above violated), OOM, HIP. */
mxp_status mxp_problem_create(mxp_context* ctx, const mxp_grid_desc* desc, mxp_problem** out);
void mxp_problem_destroy(mxp_problem* prob);

/* Number of grid nodes n0*n1*n2 (0 for a NULL problem). */
int64_t mxp_problem_size(const mxp_problem* prob);

/* ---------------------------------------------------------------- options */

typedef struct {
    double t;               /* time length of the exponential (paper: t ~ 1/freq^2)  */
    double shift;           /* complex shift s >= 0 of A_s                            */
    double fprtol;          /* inner (fixed-point) relative tolerance, in (0, 1]     */
    double rtol;            /* outer relative residual tolerance ||b-Au||/||b||      */
    int32_t outer_restart;  /* FGMRES restart length, 1..200                         */
    int32_t inner_restart;  /* inner GMRES restart length, 1..200                    */
    int32_t max_outer;      /* outer iteration limit, >= 1                           */
    int32_t max_inner;      /* inner iteration limit per preconditioner apply, >= 1  */
    mxp_precision precision;
    int32_t cheb_S;         /* > 0 forces the number of Chebyshev substeps (0 = designed) */
    int32_t cheb_m;         /* > 0 forces the series degree per substep    (0 = designed) */
    int32_t use_learned;    /* 1: learned network tried first at outer iterations; 2: its output
                               warm-starts the inner GMRES of every preconditioner apply (the
                               exp form); see mxp_problem_set_learned.  0: off */
    double stall_ratio;     /* in [0, 1]: > 0 keeps a learned z_j if the residual estimate drops
                               below this factor times the previous one; 0 (default) sets the
                               factor from MatExPre's own iterations (see below) */
    int32_t use_graphs;     /* 1: each exp / psi_1 action is captured into a HIP graph on its
                               second use and replayed afterwards (single solves; the
                               results are identical); 0 (default): launched directly */
    int32_t inner_solver;   /* inner system and solver of Algorithm 1:
                               0 (default) GMRES(inner_restart) on
                                 (I - exp(i t A_s)) w = psi_1(i t A_s) r;
                               1 the plain fixed-point iteration w <- exp(i t A_s) w + psi_1 r
                                 from w = 0 (Section 2.1, Theorem 2.1), stopped by the same
                                 residual test;
                               2 GMRES(inner_restart) on (I - psi_1(i t A_s)) w = psi_2(i t A_s) r,
                                 the second inverse formula of Section 3.1;
                               3 its fixed-point iteration w <- psi_1(i t A_s) w + psi_2 r, the
                                 time-averaged map of Section 2.2, Theorem 2.2. */
    double fp64_below;      /* MXP_PREC_MIXED only, in [0, 1): outer iterations that start with
                               the residual estimate below fp64_below * ||f|| run the
                               preconditioner's matrix-function actions in complex double
                               (the inner basis stays complex float).  0 = never. */
    int32_t fp64_first;     /* MXP_PREC_MIXED only, >= 0: the first fp64_first outer iterations
                               of the solve run the preconditioner's actions in complex double.
                               Complex-float stepping noise in z_j enters the iterate with z_j's
                               FGMRES coefficient, which is largest for the first directions;
                               left in them it costs outer iterations once the residual nears
                               the noise (2048^2 random-field workload: 14 outer iterations
                               with 0, 12 = the complex-double count with 2).  Default 2;
                               0 = complex float throughout. */
} mxp_solve_opts;

/* Defaults for a problem: t = 40 h^2 (equal to 0.4/freq^2 at ten points per
 * wavelength, Section 4.1), shift = 1/freq (Section 4.1.2), fprtol = 0.08
 * (Section 4.2.1), rtol = 1e-6, restarts 30, max_outer 500, max_inner 300,
 * MXP_PREC_FP64, designed schedule, fp64_first = 2 (used by MXP_PREC_MIXED). */
mxp_status mxp_solve_opts_default(const mxp_grid_desc* desc, mxp_solve_opts* out);

typedef struct {
    int32_t outer_its;        /* outer FGMRES iterations                          */
    int32_t inner_its_total;  /* inner GMRES iterations summed over applies       */
    double inner_mean;        /* mean inner iterations per preconditioner apply   */
    double inner_std;         /* population standard deviation of the same        */
    int64_t stencil_steps;    /* stencil sweeps spent in matrix-function actions  */
    int64_t fn_actions;       /* matrix-function actions (exp, psi_1, psi_2)      */
    double true_relres;       /* ||b - A u|| / ||b|| of the returned u, in double */
    double seconds;           /* wall time of the call                            */
    int32_t restarts;         /* outer restart cycles after the first             */
    int32_t status;           /* this solve's outcome (mxp_status)                */
    int32_t learned_its;      /* network directions kept (use_learned 1) or warm starts kept (2) */
    int32_t fallbacks;        /* network outputs rejected (MatExPre alone used instead) */
    int32_t fp64_its;         /* mixed form: outer iterations with actions in double */
} mxp_solve_stats;

/* --------------------------------------------------------------- schedule */

/* The substepped Chebyshev schedule used for exp(i t A_s) and psi_1(i t A_s):
 * exp(i t A_s) = (p(A_s))^S with p the degree-m Chebyshev expansion of
 * exp(i tau z), tau = t/S, on the segment centre +- half_width (a horizontal
 * segment in the complex plane), and q the degree-m_psi expansion of
 * tau*psi_1(i tau z) on the same segment.  Designed from a rectangle that
 * contains the field of values of A_s so that the truncation error of the
 * whole action is below the stated tolerance. */
typedef struct {
    int32_t S;                    /* substeps                                       */
    int32_t m;                    /* degree of the exp series                       */
    int32_t m_psi;                /* degree of the psi_1 series                     */
    double centre_re, centre_im;  /* segment centre                                 */
    double half_width;            /* segment half-length                            */
    double box[4];                /* field-of-values box: re_min re_max im_min im_max */
    double trunc_bound;           /* bound on the truncation error of one action    */
    double similarity_cond;       /* condition number of the diagonal similarity that
                                     brings the field of values into the box (1, or
                                     sqrt 2 per axis with ghost-point end rows)     */
    double amplification;         /* max over the box of sum_k |c_k T_k|            */
    double coef[2 * 512];         /* exp series, (re, im) pairs, m+1 used           */
    double coef_psi[2 * 512];     /* psi_1 series, (re, im) pairs, m_psi+1 used     */
} mxp_schedule;

/* Host-only (no device work; usable without a GPU).  Designs the schedule for
 * a problem description, time length t, shift and precision.  c, if given,
 * must be a host pointer here.  Errors: INVALID_ARG, UNSUPPORTED (no schedule
 * within 512 terms). */
mxp_status mxp_design_schedule(const mxp_grid_desc* desc, double t, double shift,
                               mxp_precision precision, mxp_schedule* out);

/* ------------------------------------------------------- building blocks */
/* dtype selects complex float or complex double vectors; the arithmetic runs
 * in that precision.  x and y may not alias. */

/* y = A_s x, the shifted stencil operator (Section 3.4; shift = 0 gives A). */
mxp_status mxp_apply_A(mxp_problem* prob, double shift, mxp_dtype dtype, const void* x, void* y);

/* y = exp(i t A_s) x  (Section 3.1). */
mxp_status mxp_apply_exp(mxp_problem* prob, double t, double shift, mxp_dtype dtype,
                         const void* x, void* y);

/* y = exp(i t A_s) x as mxp_apply_exp, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the call allocates nothing.  Its Clenshaw buffers and
 * the schedule's diagonal tables live in a fixed 64 MiB device array that
 * every GPU the library runs on holds until the process ends; the schedule is
 * designed on the host at every call and 2D problems use the tiles
 * mxp_apply_exp tuned, else six Clenshaw levels per pass.  Calls on one GPU
 * share the array (each call finds it as the last one left it and overwrites
 * it): calls that overlap on one GPU, from several host threads, race.
 * Errors: as mxp_apply_exp; INVALID_ARG also when six vectors of the problem
 * plus its tables exceed 64 MiB (about 690k nodes in complex double, 1.39M in
 * complex float). */
mxp_status mxp_apply_exp_noalloc(mxp_problem* prob, double t, double shift, mxp_dtype dtype, const void* x,
                                 void* y);

/* y = psi_1(i t A_s) x  (Section 3.1, Def. psi; t psi_1(i t A) equals the time
 * integral of exp(i tau A) over [0, t]). */
mxp_status mxp_apply_psi1(mxp_problem* prob, double t, double shift, mxp_dtype dtype,
                          const void* x, void* y);

/* y = psi_2(i t A_s) x  (Section 3.1: t psi_2(i t A) is the time average over
 * [0, t] of the integral of exp(i tau A) from 0).  Evaluated on the exp
 * schedule's substeps: one psi_2 series and two psi_1 series at tau = t/S plus
 * S - 2 exp series.  Same arguments, layout and errors as mxp_apply_exp;
 * UNSUPPORTED if no psi_2 series within 512 terms meets the precision's bound. */
mxp_status mxp_apply_psi2(mxp_problem* prob, double t, double shift, mxp_dtype dtype,
                          const void* x, void* y);

/* y = exp(i t A_s) x (psi = 0) or psi_1(i t A_s) x (psi = 1) by the Arnoldi
 * method, the Krylov route the paper takes for its matrix functions (Section 4
 * introduction), as an alternative to the Chebyshev schedule.  A basis of A_s
 * (at most max_dim, 1..250, vectors of n complex doubles, allocated by the
 * library and kept with the problem) is orthogonalised by classical
 * Gram-Schmidt with a second pass, and y = ||x|| V f(i t H) e_1 with the small
 * exponential computed on the host.  A basis grows until
 * h_{m+1,m} |e_m^T f(i t H_m) e_1| <= tol (relative to its start vector;
 * tested at 8, 16, 24, 32 vectors and every 16 after).  If max_dim vectors do not suffice, the action is
 * restarted by time stepping: t is split into q = 2, 4, ..., 64 substeps with
 * a fresh basis each, to tolerance tol / q (psi_1 by variation of constants).
 * x, y: distinct complex double device vectors; *dim (may be NULL) receives
 * the number of basis vectors built in all.  Errors: INVALID_ARG;
 * NOT_CONVERGED (positive) if 64 substeps did not suffice, y then holds that
 * approximation. */
mxp_status mxp_apply_fn_krylov(mxp_problem* prob, int32_t psi, double t, double shift, double tol,
                               int32_t max_dim, const void* x, void* y, int32_t* dim);

/* w = M(r), Algorithm 1 (Section 3.4): psi_1 action, then GMRES from w = 0 on
 * (I - exp(i t A_s)) w = psi_1(i t A_s) r until the residual estimate is
 * <= fprtol * ||psi_1(i t A_s) r||.  r and w are vectors of dtype (MXP_C128 or
 * MXP_C64); the inner GMRES sums and Hessenberg matrix are complex double
 * either way (complex-float vectors are widened on entry and w is rounded on
 * return).  With MXP_PREC_MIXED the matrix-function actions and the inner
 * basis are complex float.  opts->inner_solver selects the inner system and
 * solver (the psi_2 form returns w ~ (I - psi_1(i t A_s))^{-1} psi_2(i t A_s) r).
 * *inner_its (may be NULL) receives the inner iteration count. */
mxp_status mxp_apply_precond(mxp_problem* prob, const mxp_solve_opts* opts, mxp_dtype dtype, const void* r,
                             void* w, int32_t* inner_its);

/* ------------------------------------------------------------ tiling */

/* 2D grids evaluate the Chebyshev series by temporally blocked passes: K
 * consecutive Clenshaw levels per pass over HBM (1..8), NX complex values per
 * work-item (1 or 2), Ly grid rows per wavefront segment (>= 1).  By default
 * the first action on a problem times a set of candidates on the problem's
 * own buffers and keeps the fastest (per precision).
 * mxp_set_tiles fixes the configuration (K = 0 restores autotuning at the
 * next action); mxp_get_tiles reports it (K = 0 if not tuned yet) with the
 * measured microseconds per Clenshaw level (0 if fixed by the caller).
 * precision selects the complex-double (MXP_PREC_FP64) or complex-float
 * (MXP_PREC_MIXED) kernels.  On 3D grids K = 2 and K = 3 select passes of
 * two (k_cheb3d) and three (k_cheb3d3) Clenshaw levels over z-chunks of Ly
 * planes (Ly = 0: 32), and K = 1 single-level z-marching sweeps whose z
 * segments are Ly planes (Ly = 0: chosen from the grid, as the autotuner
 * reports it); NX is unused there.  By default the first action times one
 * sweep against two-level (16-, 32- and 64-plane chunks) and three-level (16,
 * 32, 64, 128) passes on the problem's buffers and keeps the fastest per level, a
 * multi-level pass only when it wins by more than 3% (at 256^3 the
 * three-level pass in complex double, the sweep in complex float); grids with
 * per-node absorbing-face terms always take sweeps.  Errors: INVALID_ARG;
 * UNSUPPORTED for K = 2, 3 on such grids. */
mxp_status mxp_set_tiles(mxp_problem* prob, mxp_precision precision, int32_t K, int32_t NX, int32_t Ly);
mxp_status mxp_get_tiles(const mxp_problem* prob, mxp_precision precision, int32_t* K, int32_t* NX,
                         int32_t* Ly, double* us_per_level);

/* ------------------------------------------------------------------ solve */

/* Solves A u = -f by FGMRES(outer_restart) preconditioned by Algorithm 1
 * (Section 3.4).  f and u are device vectors of dtype (MXP_C128, or MXP_C64
 * for complex-float data); u is read as the initial guess (zero it for the
 * plain solve) and overwritten.  Stops when the true residual
 * ||-f - A u|| <= rtol ||f||.  The outer Krylov basis, Hessenberg matrix,
 * iterate and true residual are always complex double: complex-float f and
 * u are widened on entry and u is rounded once on return (stats then report
 * the residual of the double iterate).  stats may be NULL.
 * Returns OK, NOT_CONVERGED (max_outer reached), or an error. */
mxp_status mxp_solve(mxp_problem* prob, const mxp_solve_opts* opts, mxp_dtype dtype, const void* f, void* u,
                     mxp_solve_stats* stats);

/* Per-outer-iteration record of the last single solve on the problem
 * (mxp_solve or mxp_collect_pairs; batched solves leave it unchanged), as
 * the paper tabulates it (Section 4.1.2): inner_its[k] = inner GMRES
 * iterations of outer iteration k (-1 where a network direction was kept)
 * and relres[k] = the Arnoldi estimate of the relative residual after it.
 * *count receives the number of iterations recorded; min(cap, count) entries
 * are copied to the host arrays.  Errors: INVALID_ARG (count NULL, cap < 0,
 * or cap > 0 with a NULL array). */
mxp_status mxp_solve_history(const mxp_problem* prob, int32_t cap, int32_t* inner_its, double* relres,
                             int32_t* count);

/* Solves many right-hand sides of one or more problems together (Section 3.4
 * method, as mxp_solve, for each).  Problem q has nrhs[q] right-hand sides
 * stored back to back at f[q] (nrhs[q] * size(q) complex doubles, device) and
 * as many solutions at u[q] (read as initial guesses, overwritten); opts[q]
 * are its options.  Every right-hand side runs its own FGMRES; their
 * matrix-function actions advance in lockstep, and on 3D grids the stencil
 * sweeps of one step run as one launch over all grids, uneven sizes
 * included.  Right-hand sides are admitted while their estimated workspaces
 * fit in free device memory (at most max_resident at once when > 0; at least
 * one always runs).  stats (may be NULL) receives one entry per right-hand
 * side, in order, with its own status.  Results equal those of separate
 * mxp_solve calls bit for bit.  Returns OK, NOT_CONVERGED if any right-hand
 * side did not converge, or the first error (its message names the
 * right-hand side). */
mxp_status mxp_solve_batch(mxp_context* ctx, int32_t nprob, mxp_problem* const* problems,
                           const int32_t* nrhs, const void* const* f, void* const* u,
                           const mxp_solve_opts* opts, int32_t max_resident,
                           mxp_solve_stats* stats);

/* --------------------------------------------------------- learned stage */
/* Not in the paper: a small convolutional network trained on (residual,
 * MatExPre-preconditioned residual) pairs that the method generates, tried
 * as the flexible-GMRES preconditioner before MatExPre at every outer
 * iteration.  Network: six 3x3x3 convolutions with zero padding, channels
 * 3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 2, bias on every layer, ReLU after the
 * first five; bf16 weights and activations, float accumulation on the
 * matrix cores.  Parameters (float) are flattened layer by layer as
 * W[cout][cin][3][3][3] (taps dz, dy, dx with dx fastest) then b[cout].
 * Network tensors are channels-last: input bf16 [voxel][8] (channels Re r,
 * Im r, 1/c^2, then zeros), output float [voxel][2] (Re, Im); a shape is nb
 * volumes of nz x ny x nx voxels, x fastest, each zero-padded on its own.
 * Every pointer below is device memory unless marked host. */
typedef struct mxp_cnn mxp_cnn;

/* Number of network parameters. */
int64_t mxp_cnn_num_params(void);
/* New network on the context's device and stream, He-normal weights from
 * the seed, zero biases.  Errors: INVALID_ARG, OOM, HIP. */
mxp_status mxp_cnn_create(mxp_context* ctx, uint64_t seed, mxp_cnn** out);
void mxp_cnn_destroy(mxp_cnn* net);
/* Copy the parameters / the last computed gradients to host memory, or set
 * the parameters from host memory (resets the Adam state).  Errors:
 * INVALID_ARG, NONFINITE (set), HIP. */
mxp_status mxp_cnn_get_params(const mxp_cnn* net, float* host);
mxp_status mxp_cnn_set_params(mxp_cnn* net, const float* host);
mxp_status mxp_cnn_get_grads(const mxp_cnn* net, float* host);
/* Checkpoint: writes the parameters and the Adam state (step count and both
 * moments) to the host file path, or reads them back into a network, so that
 * training resumes exactly where it stopped.  The file starts with a tag and
 * the channel list; load rejects another architecture, a short or long file
 * (INVALID_ARG) and non-finite values (NONFINITE) before it touches the
 * network.  Errors: INVALID_ARG (also an unopenable path), NONFINITE, HIP. */
mxp_status mxp_cnn_save(const mxp_cnn* net, const char* path);
mxp_status mxp_cnn_load(mxp_cnn* net, const char* path);
/* out = network(in). */
mxp_status mxp_cnn_forward(mxp_cnn* net, int32_t nb, int32_t nz, int32_t ny, int32_t nx, const void* in,
                           float* out);
/* Parameter gradients of sum(gout * network(in)), gout float [voxel][2];
 * read them with mxp_cnn_get_grads. */
mxp_status mxp_cnn_backward(mxp_cnn* net, int32_t nb, int32_t nz, int32_t ny, int32_t nx, const void* in,
                            const float* gout);
/* Copies the stored activations of hidden layer `layer` (1..5, after its
 * ReLU) from the last mxp_cnn_backward or mxp_cnn_train_step to host memory:
 * bf16 bits [voxel][32], `voxels` = nb*nz*ny*nx of that call.  The data
 * gradient of that call masked layer `layer` by (activation > 0).
 * Errors: INVALID_ARG (layer out of range, voxels not those of the last
 * training-shape call), HIP. */
mxp_status mxp_cnn_get_activations(const mxp_cnn* net, int32_t layer, int64_t voxels, uint16_t* host);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the mean squared error
 * of network(in) against target (float [voxel][2]); *loss (host, may be NULL)
 * receives the loss before the step.  Errors: INVALID_ARG, NONFINITE, HIP. */
mxp_status mxp_cnn_train_step(mxp_cnn* net, int32_t nb, int32_t nz, int32_t ny, int32_t nx, const void* in,
                              const float* target, float lr, double* loss);
/* Training sample from a pair on the problem's grid: the crop of crop[0..2]
 * nodes (x, y, z) at offset[0..2]; in (bf16 [crop][8]) = (r * rscale, 1/c^2),
 * target (float [crop][2]) = z * zscale.  r, z: complex double [size].
 * Errors: INVALID_ARG (crop outside the grid). */
mxp_status mxp_cnn_make_sample(mxp_problem* prob, const void* r, const void* z, const int32_t offset[3],
                               const int32_t crop[3], double rscale, double zscale, void* in, float* target);
/* mxp_solve that also copies, for each outer iteration, the unit Krylov
 * vector v_j and its preconditioned vector z_j = M(v_j) (Algorithm 1) into
 * r_out / z_out (max_pairs complex double vectors each) with their norms in
 * rnorm / znorm (host); *npairs receives the count.  Returns as mxp_solve. */
mxp_status mxp_collect_pairs(mxp_problem* prob, const mxp_solve_opts* opts, const void* f, void* u,
                             int32_t max_pairs, void* r_out, void* z_out, double* rnorm, double* znorm,
                             int32_t* npairs, mxp_solve_stats* stats);
/* Attaches a network (not owned; NULL detaches) to a problem for solves with
 * opts.use_learned = 1 or 2.  The network sees its input scaled to unit
 * root-mean-square value, and its output, scaled back, is multiplied by
 * out_scale (the typical ||M(v)|| / ||v|| of the training pairs).
 *
 * use_learned = 2: each preconditioner apply M(r) starts its inner GMRES from
 * w_0 = network(r) (the network is trained on pairs (r, M(r))) when the
 * residual of w_0 on (I - exp(i t A_s)) w = r_hat, which costs one action, is
 * below ||r_hat||, else from zero.  Stats count kept starts in learned_its and
 * rejected ones in fallbacks.
 *
 * use_learned = 1: at an outer iteration z_j = network(v_j) is kept if the
 * Arnoldi residual estimate falls below a threshold times the previous one:
 * stall_ratio if > 0, else min(exp(g), exp(r * 48)) with g the mean log
 * reduction per MatExPre iteration so far and r the same per stencil step
 * those iterations took (a network try counts as 48 stencil steps: the
 * inference takes about as long as 40 sweeps, plus A z and a Gram-Schmidt
 * pass).  A kept direction takes a slot of the restart cycle, so it must
 * reduce the residual as much as the MatExPre iteration it displaces, and at
 * least as cost-effectively; the rule counts work, not time, so repeated
 * solves make the same choices.  A proposal whose new Hessenberg column is
 * zero or dependent on the earlier ones (rotated diagonal below 1e-8 of the
 * column's norm) is rejected whatever its residual estimate.  Otherwise z_j = M(v_j) from MatExPre (a
 * fallback); after two fallbacks in a row MatExPre alone is used until the
 * next restart cycle.  The first outer iteration always uses MatExPre.
 *
 * Convergence is judged by the complex-double true residual as always.
 * Single solves only (mxp_solve_batch rejects use_learned). */
mxp_status mxp_problem_set_learned(mxp_problem* prob, mxp_cnn* net, double out_scale);

#ifdef __cplusplus
}
#endif

#endif /* MATEXPRE_H */
