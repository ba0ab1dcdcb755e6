/*
 * mca.h -- C ABI of the MI355X (gfx950) steady-state memristor-crossbar solver.
 *
 * The method is the one of "A Fast Method for Steady-State Memristor Crossbar
 * Array Circuit Simulation" (Xie, Song, Zhou, Mei, Chen): Newton's method on
 * the nodal equations of a crossbar made of two uniform wire grids joined by
 * one nonlinear device per crosspoint, each Newton system solved by GMRES
 * preconditioned with the block matrix P of eq. (P), whose inverse is applied
 * through the block-inversion formula (eq. (block)) and the Kronecker
 * structure of the wire matrices (eqs. (Gt), (Gb), (M)).
 *
 * Conventions shared by every call
 *   - Crossbar: m rows x n columns.  Row i is one top-layer wire (nodes
 *     (i,0)..(i,n-1)); column j is one bottom-layer wire (nodes (0,j)..(m-1,j)).
 *     Both layers use the same row-major index k = i*n + j (the paper's
 *     perpendicular natural indexing, Section III-A), so every m x n array
 *     is a row-major block of m*n doubles.
 *   - Array arguments named *_t / *_b / d / g_dev are DEVICE pointers to m*n
 *     float64 values, v_in is a device pointer to m float64 values.  Memory is
 *     owned by the caller; the library allocates no device memory of its own.
 *     Input arrays may not overlap output arrays unless stated.
 *   - `stream` is a hipStream_t (NULL = the default stream).  mca_residual,
 *     mca_jacobian_apply and mca_precond_apply only enqueue work on it and
 *     return; mca_solve synchronises it (its Newton/GMRES control reads a few
 *     scalars back per iteration).
 *   - Every call returns an mca_status; no C++ exception crosses the ABI.
 *     After MCA_ERR_HIP, mca_last_error() names the failing HIP call.
 *   - Calls on one plan from several host threads are safe as long as they
 *     use distinct workspaces and output buffers.
 */
#ifndef MCA_H
#define MCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mca_status;
#define MCA_OK                 0
#define MCA_ERR_INVALID_ARG    1   /* a size, conductance, option or pointer is invalid   */
#define MCA_ERR_NONFINITE      2   /* NaN/Inf met in the inputs or during a solve         */
#define MCA_ERR_WORKSPACE      3   /* workspace too small, or plan not uploaded            */
#define MCA_ERR_NOT_CONVERGED  4   /* iteration limit reached; last iterate + stats kept  */
#define MCA_ERR_BREAKDOWN      5   /* GMRES breakdown before convergence                  */
#define MCA_ERR_HIP            6   /* a HIP runtime call failed                           */

/* Device models: the current I(u) that flows from the top node into the bottom
 * node through the device at a crosspoint, u = V_t - V_b.                      */
#define MCA_DEVICE_SINH    0   /* I = g v0 sinh(u / v0), dI/du = g cosh(u / v0) */
#define MCA_DEVICE_LINEAR  1   /* I = g u,               dI/du = g              */

/* Arithmetic of the preconditioner's eigenbasis transforms.  The Newton
 * residual, the Jacobian products, the Arnoldi orthogonalisation and the
 * Hessenberg least squares are FP64 in every mode; flexible GMRES absorbs the
 * rounding of a reduced-precision preconditioner.  Reduced precisions need
 * MCA_PRECOND_PERMODE (the literal order loses log10(lambda_max / a1) digits,
 * too many for them).                                                        */
#define MCA_PREC_FP64      0
#define MCA_PREC_FP32      1   /* FP32 operands, FP32 MFMA                                 */
#define MCA_PREC_BF16X3    2   /* split-BF16 (hi+lo) operands, 3 MFMA products, FP32 acc  */
#define MCA_PREC_BF16      3   /* BF16 operands (hi only), FP32 accumulation               */

/* How the preconditioner is applied.  LITERAL and PERMODE both give P^{-1} of
 * eq. (P) in exact arithmetic; APPROX is the paper's approximation (it inverts
 * P with its -a2 I block dropped, which is what M ~ Mhat amounts to); JACOBI
 * and NONE are baselines.                                                   */
#define MCA_PRECOND_LITERAL  0 /* the paper's order: w = r_b - D B^{-1} r_t, z_t = M^{-1} w,
                                  z_b = B^{-1}(r_t - A z_t)  (eqs. (block), (M))            */
#define MCA_PRECOND_PERMODE  1 /* the same 2x2 block formula applied per Kronecker eigenmode */
#define MCA_PRECOND_NONE     2 /* z = r (unpreconditioned GMRES, for comparison)            */
#define MCA_PRECOND_APPROX   3 /* the paper's approximation M ~ Mhat = G2hat (x) G1 (eq. (Mhat)),
                                  applied by tridiagonal solves; FP64 only, m, n <= 8192 */
#define MCA_PRECOND_JACOBI   4 /* point-Jacobi z = r ./ diag(J), a baseline (mca_solve only) */

#define MCA_FLAG_INITIAL_GUESS 1  /* mca_solve starts from v_t/v_b instead of V = 0       */
#define MCA_FLAG_TIMING        2  /* mca_solve times its kernel classes with HIP events     */
#define MCA_FLAG_GUESS_FALLBACK 4 /* with a guess: a guess whose residual is not below that
                                     of V = 0 (||F(0)|| = ||Y||) is dropped for V = 0       */
#define MCA_FLAG_SWEEP_START   8  /* start from one block Gauss-Seidel sweep on the
                                     linearisation at V = 0, J(0) V = Y:
                                     V_t = (G_t + D)^{-1} Y_t, V_b = (G_b + D)^{-1} D V_t,
                                     D = g_dev (tridiagonal solves along every wire);
                                     not with INITIAL_GUESS; m, n <= 2048                  */
#define MCA_FLAG_GRAPH        16  /* mca_solve_batched only: each Arnoldi step is captured
                                     once into a HIP graph kept in the batch and replayed
                                     by later cycles and solves with the same workspace,
                                     precision, restart length and Gram-Schmidt form    */
#define MCA_FLAG_MGS_PASSES   32  /* Arnoldi orthogonalisation in one pass over the
                                     vector per basis vector (modified Gram-Schmidt as
                                     written) instead of the default two passes per step
                                     (the same projections in compact WY form, restart
                                     <= 32); the two give the same h up to rounding     */
#define MCA_FLAG_TIMING_SAMPLED 64 /* mca_solve times only the preconditioner class
                                     (MCA_KCLASS_GEMM), on every 4th application: a timed
                                     event between dependent kernels leaves the GPU idle for
                                     a few microseconds, so timing every group slows the
                                     solve; kernel_ms / kernel_launches of the sampled
                                     groups is the average launch time (MCA_FLAG_TIMING,
                                     if also set, times every group)                  */

/* Kernel classes timed under MCA_FLAG_TIMING (mca_stats.kernel_ms / kernel_launches). */
#define MCA_KCLASS_GEMM      0    /* eigenbasis transforms of the preconditioner          */
#define MCA_KCLASS_JACOBIAN  1    /* Jacobian products                                    */
#define MCA_KCLASS_ORTHO     2    /* Arnoldi orthogonalisation and normalisation passes   */
#define MCA_KCLASS_RESIDUAL  3    /* residual evaluations                                 */
#define MCA_NUM_KCLASS       4

#define MCA_MAX_RESTART   64
#define MCA_MAX_NEWTON    64

/* One crossbar geometry (Section II): two uniform wire layers, one segment
 * conductance per layer, plus the boundary drive and terminations.
 *   Top wire i:    V_in[i] --g_src-- (i,0) --g_top-- ... --g_top-- (i,n-1) --g_top_end-- ground
 *   Bottom wire j: ground --g_bot_end0-- (0,j) --g_bot-- ... --g_bot-- (m-1,j) --g_bot_end1-- ground
 * Each wire's conductance matrix (eq. (G)) is tridiagonal with -g off the
 * diagonal, 2g inside the diagonal and g + (end conductance) at its two ends;
 * tying both ends through g gives the paper's eq. (G) exactly.
 * Valid geometry: m, n >= 1; every conductance finite and >= 0; g_top, g_bot
 * > 0; g_src + g_top_end > 0; g_bot_end0 + g_bot_end1 > 0 (so that neither
 * wire matrix is singular); v0 > 0 for the sinh device.                     */
typedef struct mca_geometry {
    int32_t m, n;
    int32_t device_model;          /* MCA_DEVICE_*                                  */
    int32_t reserved;              /* must be 0                                     */
    double  g_top, g_bot;          /* wire segment conductance per layer [S]       */
    double  g_src;                 /* drive source -> top node (i,0) [S]           */
    double  g_top_end;             /* top node (i,n-1) -> ground [S]               */
    double  g_bot_end0, g_bot_end1;/* bottom nodes (0,j), (m-1,j) -> ground [S]    */
    double  v0;                    /* device voltage scale [V]                      */
} mca_geometry;

/* Newton / flexible-GMRES controls.  mca_options_default fills:
 * newton_tol 1e-10, gmres_tol 1e-8, restart 30, max_newton 50, max_krylov 600,
 * precision MCA_PREC_FP64, precond MCA_PRECOND_LITERAL, flags 0.              */
typedef struct mca_options {
    double  newton_tol;   /* stop when ||F(V)||_2 <= newton_tol * ||Y||_2              */
    double  gmres_tol;    /* inner stop: ||J dV + F||_2 <= gmres_tol * ||F||_2          */
    int32_t restart;      /* flexible GMRES restart length, 1..MCA_MAX_RESTART          */
    int32_t max_newton;   /* Newton steps, 1..MCA_MAX_NEWTON                            */
    int32_t max_krylov;   /* GMRES iterations per Newton step (over all restarts)       */
    int32_t precision;    /* MCA_PREC_*                                                 */
    int32_t precond;      /* MCA_PRECOND_*                                              */
    int32_t flags;        /* MCA_FLAG_*                                                 */
} mca_options;

typedef struct mca_stats {
    int32_t newton_iters;                 /* Newton steps taken                          */
    int32_t krylov_iters;                 /* GMRES iterations over all Newton steps      */
    int32_t backtracks;                   /* step halvings of the line search            */
    int32_t restarts;                     /* GMRES restarts over all Newton steps        */
    double  rel_residual;                 /* final ||F||_2 / ||Y||_2                     */
    double  a_last;                       /* a1 = a2 = mean dI/du of the last Newton step */
    double  residual_history[MCA_MAX_NEWTON + 1]; /* ||F||/||Y|| before each step        */
    int32_t krylov_history[MCA_MAX_NEWTON];       /* GMRES iterations of each step       */
    /* MCA_FLAG_TIMING only (zero otherwise): GPU time of each kernel class between
     * HIP events recorded on the solve's stream around each group of launches, and
     * the number of kernel launches in those groups (MCA_FLAG_TIMING_SAMPLED: the
     * sampled preconditioner groups only).                                       */
    double  kernel_ms[MCA_NUM_KCLASS];
    int32_t kernel_launches[MCA_NUM_KCLASS];
    int32_t start;                        /* 1: started from the caller's guess, 0: V = 0 */
    double  err_bound;                    /* certified ||V - V*||_2 <= err_bound: F is the
                                             gradient of a strongly convex energy (J(V) >=
                                             blkdiag(G_t, G_b) since dI/du >= 0), so the error
                                             is at most ||F(V)||_2 / min(lambda_min(G_top),
                                             lambda_min(G_bot))                             */
} mca_stats;

typedef struct mca_plan mca_plan;

void        mca_options_default(mca_options *opts);
const char *mca_status_string(mca_status s);
const char *mca_last_error(void);     /* thread-local text of the last MCA_ERR_HIP */
/* sizeof of the ABI's structs, so that a binding can check its layout:
 * which 0 = mca_geometry, 1 = mca_options, 2 = mca_stats; 0 for other values. */
size_t      mca_abi_struct_size(int32_t which);

/* Validate `geom` and build the preconditioner's geometry data on the host:
 * the eigen-decompositions G_top = Q_n diag(lt) Q_n^T (n x n) and
 * G_bot = Q_m diag(lb) Q_m^T (m x m) of the two wire matrices.  The paper
 * writes P^{-1} through Kronecker products of these matrices (eqs. (M),
 * (M-1hat), (2matrix4)); their eigenbasis turns every Kronecker factor into a
 * diagonal, so a1, a2 only shift eigenvalues and nothing is refactorised per
 * Newton step.  *out receives a host object freed by mca_plan_destroy.  The
 * two wires are decomposed on the calling thread and one extra host thread
 * (joined before return; thread-safe for distinct plans).
 * Errors: MCA_ERR_INVALID_ARG (bad geometry or NULL out).                    */
mca_status mca_plan_create(const mca_geometry *geom, mca_plan **out);
void       mca_plan_destroy(mca_plan *plan);

/* Host copy of one wire's eigen-decomposition (the plan's set-up data):
 * layer 0 = top wire (G_top, n x n), layer 1 = bottom wire (G_bot, m x m).
 * lambda (may be NULL) receives the eigenvalues in ascending order, q (may be
 * NULL) the row-major eigenvector matrix, q[i*len + k] = entry i of vector k.
 * Host memory only; needs no GPU.  Errors: MCA_ERR_INVALID_ARG.             */
mca_status mca_plan_host_eigen(const mca_plan *plan, int32_t layer, double *lambda, double *q);

/* Device bytes the plan needs (Q_m, Q_m^T, Q_n, Q_n^T in FP64 and FP32, and
 * the eigenvalues).                                                          */
size_t     mca_plan_device_bytes(const mca_plan *plan);

/* Copy the plan's data into `dev_buf` (caller-owned device memory of at least
 * mca_plan_device_bytes bytes, 256-byte aligned) on `stream` and remember it.
 * The buffer must outlive every later call on this plan.  Synchronises stream.
 * Errors: MCA_ERR_INVALID_ARG, MCA_ERR_WORKSPACE (too small), MCA_ERR_HIP.  */
mca_status mca_plan_upload(mca_plan *plan, void *dev_buf, size_t bytes, void *stream);

/* Device workspace (bytes, 256-byte aligned) for mca_solve with `opts`
 * (NULL = defaults), and for mca_precond_apply with a form and precision.   */
size_t     mca_workspace_bytes(const mca_plan *plan, const mca_options *opts);
size_t     mca_precond_workspace_bytes(const mca_plan *plan, int32_t form, int32_t precision);

/* MNA residual, eqs. (MNA) and (F):
 *   f_t = G_t v_t + I(v_t - v_b) - Y_t,   f_b = G_b v_b - I(v_t - v_b)
 * with G_t = I_m (x) G_top, G_b = G_bot (x) I_n (eqs. (Gt), (Gb)),
 * Y_t[i,0] = g_src v_in[i] (zero elsewhere), Y_b = 0, and
 *   d = dI/du at every crosspoint (the diagonal of the device blocks of eq. (J)).
 * g_dev: device conductances.  f_t, f_b, d: outputs (d may be NULL).
 * Asynchronous on stream.  Errors: MCA_ERR_INVALID_ARG, MCA_ERR_WORKSPACE
 * (plan not uploaded), MCA_ERR_HIP.                                         */
mca_status mca_residual(const mca_plan *plan, const double *g_dev, const double *v_in,
                        const double *v_t, const double *v_b,
                        double *f_t, double *f_b, double *d, void *stream);

/* Jacobian product y = J x, eq. (J):
 *   y_t = G_t x_t + d (x_t - x_b),   y_b = G_b x_b - d (x_t - x_b)
 * (the four device blocks are diagonal, +-d, Section III-A).  d is the device
 * slope array of the linearisation point.  Asynchronous on stream.
 * Errors: MCA_ERR_INVALID_ARG, MCA_ERR_WORKSPACE (plan not uploaded), MCA_ERR_HIP. */
mca_status mca_jacobian_apply(const mca_plan *plan, const double *d,
                              const double *x_t, const double *x_b,
                              double *y_t, double *y_b, void *stream);

/* Preconditioner solve z = P^{-1} r for
 *   P = [[G_t + a1 I, -a1 I], [-a2 I, G_b + a2 I]]          (eq. (P))
 * with a1, a2 > 0 (in the solver both are the mean device slope).  `form`
 * picks the evaluation order (MCA_PRECOND_LITERAL or MCA_PRECOND_PERMODE; see
 * above), `precision` the arithmetic of the eigenbasis transforms.  The
 * Kronecker factor M^{-1} of eq. (M) is applied exactly through the wire
 * eigenbases: M^{-1} w <-> Q_m [(Q_m^T W Q_n) ./ mu] Q_n^T with
 *   mu_pq = lb_p lt_q / a1 + lb_p + (a2 / a1) lt_q.
 * ws: device workspace of mca_precond_workspace_bytes(plan, form, precision).
 * precision other than MCA_PREC_FP64 requires form MCA_PRECOND_PERMODE.
 * r_* and z_* must not overlap.  Asynchronous on stream.
 * Errors: MCA_ERR_INVALID_ARG, MCA_ERR_WORKSPACE, MCA_ERR_HIP.               */
mca_status mca_precond_apply(const mca_plan *plan, int32_t form, int32_t precision,
                             double a1, double a2,
                             const double *r_t, const double *r_b,
                             double *z_t, double *z_b,
                             void *ws, size_t ws_bytes, void *stream);

/* mca_precond_apply without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, forms, precisions,
 * arithmetic and kernels as mca_precond_apply; the workspace is a fixed
 * device array inside the library, MCA_NOALLOC_SCRATCH_BYTES (32 MiB) per
 * GPU, held from the library's load until the process ends.  The call
 * allocates nothing: no hipMalloc, hipFree or allocating library routine.
 * The array's address on the current GPU is looked up on the first call on
 * that GPU (hipGetSymbolAddress; better made outside graph capture).
 * Limit: mca_precond_workspace_bytes(plan, form, precision) <=
 * MCA_NOALLOC_SCRATCH_BYTES, which holds every form up to 1024 x 1024
 * crosspoints (the FP64 per-mode form needs 32 mn bytes, the others at most
 * 24 mn); larger calls return MCA_ERR_WORKSPACE before any launch.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap on one GPU (other streams or host threads) race
 * and must be serialised by the caller.  Asynchronous on stream.
 * Errors: those of mca_precond_apply, MCA_ERR_WORKSPACE for sizes beyond the
 * limit, MCA_ERR_HIP if the array's address cannot be found.               */
#define MCA_NOALLOC_SCRATCH_BYTES (32u << 20)
mca_status mca_precond_apply_noalloc(const mca_plan *plan, int32_t form, int32_t precision,
                                     double a1, double a2,
                                     const double *r_t, const double *r_b,
                                     double *z_t, double *z_b, void *stream);

/* Steady state: v_t, v_b with F(v_t, v_b) = 0 (eq. (F)), by Newton's method
 * (eq. (Newton3)); each step solves J dV = -F with flexible GMRES(restart),
 * modified Gram-Schmidt Arnoldi, right-preconditioned by P (eq. (P)) with
 * a1 = a2 = mean(dI/du) of the current iterate (Section III-A).  Each Newton
 * step is damped by halving while ||F(V + s dV)|| > (1 - 1e-4 s) ||F(V)||.
 * Starts from V = 0 (whose first step is the linear solve J(0)^{-1} Y), or
 * from v_t/v_b with MCA_FLAG_INITIAL_GUESS.  Writes the final iterate to
 * v_t, v_b in every outcome except MCA_ERR_INVALID_ARG / MCA_ERR_WORKSPACE.
 * stats (host, may be NULL) is filled in every outcome.  Synchronises stream.
 * Errors: MCA_ERR_INVALID_ARG, MCA_ERR_WORKSPACE, MCA_ERR_NONFINITE,
 * MCA_ERR_NOT_CONVERGED, MCA_ERR_BREAKDOWN, MCA_ERR_HIP.                     */
mca_status mca_solve(const mca_plan *plan, const double *g_dev, const double *v_in,
                     double *v_t, double *v_b, const mca_options *opts,
                     void *ws, size_t ws_bytes, mca_stats *stats, void *stream);

/* ------------------------------------------------------------------ batches
 * Many crossbars, each with its own geometry (sizes may differ), solved
 * together: every Newton / GMRES step of every crossbar runs in the same
 * kernel launches (the Monte-Carlo use of Section IV, where many crossbars
 * with varied devices and wires are simulated).  Each crossbar follows the
 * same method and stopping rules as mca_solve; one that has converged or
 * failed drops out of the launches while the others go on.
 *
 * Concatenated arrays: crossbar b's m_b x n_b arrays (g_dev, v_t, v_b) start
 * at element cross_offsets[b] = sum_{c<b} m_c n_c of one device array, its
 * drives v_in at element row_offsets[b] = sum_{c<b} m_c (see
 * mca_batch_offsets).  Batches support form MCA_PRECOND_PERMODE with
 * precision MCA_PREC_FP32, MCA_PREC_BF16X3 or MCA_PREC_BF16.               */
typedef struct mca_batch mca_batch;

/* Validate count geometries and build every crossbar's eigen-decompositions
 * (host threads).  *out receives a host object freed by mca_batch_destroy.
 * Errors: MCA_ERR_INVALID_ARG (count < 1, NULL pointer or a bad geometry). */
mca_status mca_batch_create(int32_t count, const mca_geometry *geoms, mca_batch **out);
void       mca_batch_destroy(mca_batch *batch);

/* Offsets of the concatenated arrays (host arrays of count + 1 entries each,
 * either may be NULL); the last entry is the total length.                */
mca_status mca_batch_offsets(const mca_batch *batch, int64_t *cross_offsets,
                             int64_t *row_offsets);

/* Device bytes of the batch's set-up data (eigenbases in FP32 and bfloat16
 * hi/lo planes, eigenvalues, launch tables), and their upload into
 * caller-owned device memory (256-byte aligned, kept until the last solve).
 * Synchronises stream.  Errors: MCA_ERR_INVALID_ARG, MCA_ERR_WORKSPACE,
 * MCA_ERR_HIP.                                                             */
size_t     mca_batch_device_bytes(const mca_batch *batch);
mca_status mca_batch_upload(mca_batch *batch, void *dev_buf, size_t bytes, void *stream);

/* Edge of the square output tiles (64 or 128) of the batch's grouped
 * eigenbasis products, fixed at creation from the crossbar sizes: 128 when
 * every crossbar's sides are at least 256 and the batch gives at least 256
 * such tiles per product, else 64.  0 for a NULL batch.  Host only.        */
int32_t    mca_batch_product_tile(const mca_batch *batch);

/* Device workspace of mca_solve_batched with opts (NULL = PERMODE, BF16X3,
 * other fields as mca_options_default); 0 when opts are not supported.    */
size_t     mca_batch_workspace_bytes(const mca_batch *batch, const mca_options *opts);

/* Steady state of every crossbar of the batch (as mca_solve, per crossbar).
 * g_dev, v_in, v_t, v_b: concatenated device arrays (see above); v_t/v_b
 * carry the initial guesses with MCA_FLAG_INITIAL_GUESS.  stats: host array
 * of count records (may be NULL).  With MCA_FLAG_TIMING (every
 * preconditioner application of the batch) or MCA_FLAG_TIMING_SAMPLED (every
 * fourth), and without MCA_FLAG_GRAPH, stats[0].kernel_ms[MCA_KCLASS_GEMM]
 * holds the GPU time between HIP events recorded on the stream just before
 * and just after the four grouped products of those applications (each
 * interval also holds the few microseconds an event leaves the GPU idle), and
 * stats[0].kernel_launches[MCA_KCLASS_GEMM] four per timed application; the
 * other classes and records stay zero.
 * The batch keeps pinned host counters and, with MCA_FLAG_GRAPH, the captured
 * Arnoldi steps (dropped when the workspace address, precision, restart
 * length, Gram-Schmidt form or uploaded block change): calls on one batch
 * must not overlap.
 * Returns MCA_OK when every crossbar converged, else the status of the first
 * crossbar that did not (the per-crossbar outcome is in the residual
 * history of stats).  Synchronises stream.
 * Errors: MCA_ERR_INVALID_ARG, MCA_ERR_WORKSPACE (too small, or batch not
 * uploaded), MCA_ERR_NONFINITE, MCA_ERR_NOT_CONVERGED, MCA_ERR_HIP.       */
mca_status mca_solve_batched(const mca_batch *batch, const double *g_dev, const double *v_in,
                             double *v_t, double *v_b, const mca_options *opts,
                             void *ws, size_t ws_bytes, mca_stats *stats, void *stream);

/* ------------------------------------------------------- warm-start network
 * A 6-layer 3x3 CNN predicts a crossbar's steady state from its inputs, to
 * start mca_solve (MCA_FLAG_INITIAL_GUESS) nearer to the solution than V = 0
 * (Newton's method, eq. (Newton3), converges from the guess; the guess only
 * changes the iteration count).  It corrects a mean-field guess: the paper's
 * approximate preconditioner (eq. (block) with M ~ Mhat) applied to the drive
 * vector Y at a1 = a2 = a = mean(g_dev); as Y_b = 0 that guess is
 * V0_t[i][j] = v_in[i] phi[j], V0_b = 0 with phi = g_src (G_top + a I)^{-1} e_0.
 * Per crosspoint (i, j) the input channels are log10(g_dev) + 5,
 * v_in[i]/0.15 - 1, (g_top - 0.5)/0.3 and v_in[i] (1 - phi[j]) / 0.1; five 3x3
 * convolutions with 32 channels and ReLU, then a linear 3x3 convolution to
 * (y_t, y_b); V_t = V0_t - 0.01 y_t, V_b = 0.01 y_b.  Zero "same" padding.
 * Arithmetic: bfloat16 weights and activations on MFMA, FP32 accumulation,
 * FP32 master parameters and Adam state.
 *
 * params: device FP32 vector of mca_cnn_param_count() values: per layer
 * w[dy][dx][ci][co] (row-major; ci = 4, 32, 32, 32, 32, 32; co = 32, 32, 32,
 * 32, 32, 2) followed by b[co].  A batch is `batch` crossbars of one size
 * m x n, described by a host array geoms[batch] (equal m, n; only g_top,
 * g_src and g_top_end are used); g_dev, v_t, v_b hold batch*m*n doubles
 * (crossbar after crossbar), v_in batch*m.  Arrays are device pointers; the
 * calls synchronise stream once (to upload the small wire table) and then
 * enqueue the rest asynchronously.                                          */
int64_t    mca_cnn_param_count(void);
/* device workspace (bytes) for a batch of m x n crossbars; 0 for bad sizes */
size_t     mca_cnn_workspace_bytes(int32_t batch, int32_t m, int32_t n);
/* predicted v_t, v_b.  Errors: MCA_ERR_INVALID_ARG, MCA_ERR_WORKSPACE, MCA_ERR_HIP. */
mca_status mca_cnn_predict(const float *params, int32_t batch, const mca_geometry *geoms,
                           const double *g_dev, const double *v_in, double *v_t, double *v_b,
                           void *ws, size_t ws_bytes, void *stream);
/* Training loss against solved voltages v_t, v_b: the mean over the batch of
 * (y - y_target)^2 over every crosspoint and both outputs, y_target from the
 * voltage map above; grad (device, param_count floats) receives its
 * gradient, loss (device, 1 float) its value.  Same errors as predict.      */
mca_status mca_cnn_gradient(const float *params, int32_t batch, const mca_geometry *geoms,
                            const double *g_dev, const double *v_in, const double *v_t,
                            const double *v_b, float *grad, float *loss, void *ws,
                            size_t ws_bytes, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; step >= 1)
 * on params with moment vectors adam_m, adam_v (device, param_count floats,
 * zero before step 1).  Errors: MCA_ERR_INVALID_ARG, MCA_ERR_HIP.          */
mca_status mca_cnn_adam(float *params, const float *grad, float *adam_m, float *adam_v,
                        int32_t step, float lr, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MCA_H */
