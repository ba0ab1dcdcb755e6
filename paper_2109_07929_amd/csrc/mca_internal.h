// mca_internal.h -- shared declarations of the HIP solver library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/mca.h"

namespace mca {

// Coefficients of one uniform wire (Section II, eq. (G)): segment conductance g
// between neighbours, end0 from the first node and end1 from the last node to
// their far sides.  Node k of a wire of `len` nodes carries on the diagonal
// g * (number of neighbouring segments) + end0 [k == 0] + end1 [k == len-1].
struct Wire {
    double g, end0, end1;
    int len;
};

// Device data of an uploaded plan.
struct DevPlan {
    const double *Qm, *QmT;   // m x m: Qm[i*m + p] = entry i of eigenvector p of G_bot
    const double *Qn, *QnT;   // n x n: Qn[j*n + q] = entry j of eigenvector q of G_top
    const double *lb, *lt;    // eigenvalues of G_bot (m) and G_top (n), ascending
    // reduced-precision copies: FP32, and bfloat16 hi / lo planes (v = hi + lo)
    const float *Qm32, *QmT32, *Qn32, *QnT32;
    const void *QmH, *QmL, *QmTH, *QmTL, *QnH, *QnL, *QnTH, *QnTL;
    // persymmetric G_bot (equal end terminations, m even): its eigenvectors are
    // [u; J u]/sqrt2 (symmetric) or [u; -J u]/sqrt2 (antisymmetric), u of length
    // h = m/2.  Us, Ua (h x h) hold u/sqrt2 column-wise, UsT, UaT their
    // transposes; lbp = (lambda_sym, lambda_anti), the mode order of the folded
    // transforms.  Null when G_bot is not persymmetric.
    const double *Us, *UsT, *Ua, *UaT, *lbp;
    // reduced-precision [U_s^T; U_a^T] and [U_s; U_a] (m x h) for the folded chain
    const float *QmTf32, *Qmf32;
    const void *QmTfH, *QmTfL, *QmfH, *QmfL;
};

}  // namespace mca

struct mca_plan {
    mca_geometry geom;
    mca::Wire top, bot;
    std::vector<double> lb, lt;      // host eigenvalues
    std::vector<double> Qm, Qn;      // host eigenvectors (row-major, columns are vectors)
    bool persym = false;             // G_bot persymmetric with m even: folded transforms
    std::vector<double> Us, Ua, ls, la;   // halves (h x h, u / sqrt2) and their eigenvalues
    size_t dev_bytes = 0;
    void *dev_buf = nullptr;         // caller-owned, set by mca_plan_upload
    mca::DevPlan dev{};
};

namespace mca {

// Host: eigenpairs of a symmetric tridiagonal matrix (diag a, off b).
// lam ascending; Q row-major n x n with Q[i*n + k] = entry i of eigenvector k.
void tridiag_eigen(int n, const double *a, const double *b, double *lam, double *Q);

// Error text of the last failed HIP call on this thread.
void set_hip_error(const char *what, hipError_t e);

// ---------------------------------------------------------------- kernels
// All launchers enqueue on `s` and return the launch status.

// Number of per-block partial sums the Krylov reductions of a vector of
// length len use (fixed per length, so every reduction order is fixed).
int reduce_blocks(size_t len);

hipError_t launch_residual(const mca_plan *P, const double *g_dev, const double *v_in,
                           const double *vt, const double *vb, double *ft, double *fb,
                           double *d, double *partials, hipStream_t s);
// Host wait for a 64-bit flag slot in pinned host memory that a kernel sets to
// (1 << 32) | value with a release store at system scope (the host clears the
// slot to 0 before enqueueing that kernel); *value receives the low word.
mca_status wait_flag64(const long long *slot, hipStream_t s, int *value);

// final sums of partials: out[c] = sum_b partials[b*ncomp + c], c < ncomp;
// with mark set, *mark = epoch afterwards (release store at system scope: a
// host polling a pinned marker then sees out)
hipError_t launch_reduce(const double *partials, int nblocks, int ncomp, double *out,
                         hipStream_t s, int *mark = nullptr, int epoch = 0);

// y = J x (eq. (J)); with v0 also per-block partials of <y, v0> (grid of
// reduce_blocks(2mn) blocks).  Kernels given a skip flag return at once when
// it is set (a converged GMRES cycle).
hipError_t launch_jacobian(const mca_plan *P, const double *d, const double *xt,
                           const double *xb, double *yt, double *yb, hipStream_t s,
                           const double *v0 = nullptr, double *partials = nullptr,
                           const int *skip = nullptr);

// w = r_b + ((G_b + a2 I) r_t) / a1            (first step of the literal form)
hipError_t launch_precond_pre(const mca_plan *P, double a1, double a2, const double *rt,
                              const double *rb, double *w, hipStream_t s,
                              const int *skip = nullptr);
// Folded first step for a persymmetric G_bot (m = 2h): with w as above,
// P[i] = w[i] + w[m-1-i] into f[0, h*n), Q[i] = w[i] - w[m-1-i] into f[h*n, m*n).
hipError_t launch_precond_pre_fold(const mca_plan *P, double a1, double a2, const double *rt,
                                   const double *rb, double *f, hipStream_t s,
                                   const int *skip = nullptr);
// Unfold the inverse Q_m transform of a persymmetric G_bot: from the symmetric and
// antisymmetric halves Ys, Ya (n x h each), X^T[j][i] = Ys + Ya and
// X^T[j][m-1-i] = Ys - Ya (X^T n x m, m = 2h).
hipError_t launch_unfold(const double *ys, const double *ya, int n, int h, double *xt,
                         hipStream_t s, const int *skip = nullptr);
// z_b = ((G_t + a1 I) z_t - r_t) / a1          (last step of the literal form)
hipError_t launch_precond_post(const mca_plan *P, double a1, const double *zt,
                               const double *rt, double *zb, hipStream_t s,
                               const int *skip = nullptr);

// GEMM epilogues
enum GemmEpi { EPI_STORE = 0, EPI_DIV_MU = 1, EPI_PERMODE = 2, EPI_UNFOLD = 3, EPI_UNFOLD16 = 4 };

// O = L^T R (one or two batches sharing R), FP64 MFMA.
//   L: K x M row-major (ld = M), R: K x N row-major (ld = N), O: M x N row-major.
//   EPI_DIV_MU : O[p][q] = acc / (lb[p] lt[q] / a1 + lb[p] + (a2/a1) lt[q])
//   EPI_PERMODE: (O0, O1) = 2x2 per-mode solve of (acc0, acc1)      (needs 2 batches)
//   EPI_UNFOLD : L0 = Y_s, L1 = Y_a (K x M/2 each, ld = M/2) stand for
//                L = [Y_s + Y_a | column-mirrored (Y_s - Y_a)], so that O rows p and
//                M-1-p are A_p + B_p and A_p - B_p with A = Y_s^T R, B = Y_a^T R
//                (the persymmetric unfold fused into the product); only when
//                gemm_unfold_fits(M, N, K)
// O's row stride is ldo (0: N).  pair: two independent single-batch products in
// one launch, the second with L1, R1, O1 (the same sizes and epilogue).
struct GemmArgs {
    int M, N, K;
    const double *L0, *L1;     // L1 may be null (single batch)
    const double *R;
    double *O0, *O1;
    const double *lb, *lt;     // for the epilogues (length M and N)
    double a1, a2;
    const double *shift;       // optional: a1 = a2 = shift[0], 1 / a1 = shift[1] (device)
    int vec;                   // set by the launcher: rows are 16-byte aligned
    const int *skip;           // optional: return at once when *skip != 0
    int ldo;                   // output row stride (0: N)
    int pair;                  // second independent product (L1, R1, O1) in the same launch
    const double *R1;
};
hipError_t launch_gemm_f64(const GemmArgs &a, int epi, hipStream_t s);
bool gemm_unfold_fits(int M, int N, int K);

// Per-mode preconditioner in reduced precision (gemm_lp.hip): four NT products
// on FP32 / BF16 MFMA with the per-mode 2x2 solve in the second one.
// An operand in its MFMA format: FP32 values in p[0], or bfloat16 hi (p[0]) and
// lo (p[1]) planes.
struct LpPlanes {
    void *p[2];
};
struct LowPrecChain {
    int m, n;
    double a1, a2;
    const int *skip;
    LpPlanes QnT, QmT, Qm, Qn;          // eigenbases
    const double *lt, *lb;              // eigenvalues of G_top, G_bot
    const double *rt, *rb;              // input r (FP64)
    int r_split;                        // x already holds r in operand format (folded, with fold)
    LpPlanes x[2], u[2], w[2];          // workspace: split r and two intermediates, m*n each
    double *zt, *zb;                    // output z (FP64)
    // persymmetric G_bot with m / 2 a multiple of 128: the folded chain, with
    // QmTf = [U_s^T; U_a^T] and Qmf = [U_s; U_a] (m x m/2 each) and the
    // eigenvalues of G_bot in the folded mode order (symmetric first)
    int fold;
    LpPlanes QmTf, Qmf;
    const double *lbp;
};
hipError_t launch_precond_lowprec(int precision, const LowPrecChain &c, hipStream_t s);

// Grouped form over a batch of crossbars (batch.hip): one crossbar's product
// in a grouped launch.  Data operands and outputs of every crossbar sit at an
// element offset from the launch's base planes (layer 1 at + mn).
struct LpDesc {
    int M, N, K, inst;
    const void *Q[2];                   // the crossbar's eigenbasis operand (planes)
    size_t off_data, off_out, mn;
    const double *lam_row, *lam_col;    // eigenvalues along output rows / columns
    int vec;                            // 16-byte aligned rows, K % 8 == 0
    // persymmetric fold of the crossbar's Q_m-side products (see the
    // single-crossbar chain): row strides, split, interleave, unfold, and alt:
    // the data operand comes from the launch's alternative planes
    int lda, ldb, split, ileave, unfold, alt;
};
struct GroupedLp {
    const LpDesc *descs;
    const int4 *tiles;                  // (descriptor, m0, n0, unused)
    const void *data[2];
    const void *data_alt[2];            // the data planes of descriptors with alt set
    void *out[2];
    size_t data_elem_bytes, out_elem_bytes;
    const double *a_inst;               // per-crossbar a1 = a2, stride a_stride doubles
    int a_stride;
    const int *ctl;                     // per-crossbar control blocks (4 ints), stop flag first
};
// The four products of the per-mode chain over a batch, after splitting the
// whole Krylov vector r (len doubles) into operand planes x.
struct GroupedChain {
    const LpDesc *descs[4];
    const int4 *tiles[4];
    int ntiles[4];
    int tile;                           // tile edge of the tables: 64 or 128
    const double *r;
    size_t len;
    int r_split;                        // x already holds r in operand format
    int r_folded;                       // and w the folded chains' input (with r_split)
    LpPlanes x, u, w;
    float *z;                           // output z in FP32 (the products accumulate in FP32)
    const double *a_inst;
    int a_stride;
    const int *ctl;
    // crossbars with a folded chain (their product-1 descriptors have alt set):
    // x is folded into w first, block b of that pass taking chunk fold_tab[b].y
    // (kFoldChunk elements of the m/2 x n half) of crossbar fold_tab[b].x
    const int2 *fold_tab;
    int fold_blocks;
    // optional: recorded on the stream just before the first product and just
    // after the fourth (timing of the products alone)
    hipEvent_t ev[2];
};
constexpr int kFoldChunk = 2048;
hipError_t launch_precond_lowprec_grouped(int precision, const GroupedChain &c, hipStream_t s);
// host: FP64 -> FP32 (p0) or bfloat16 hi (p0) + lo (p1)
void split_host(const double *src, size_t count, int precision, void *p0, void *p1);

// The paper's approximate preconditioner (tridiag.hip): batched tridiagonal
// solves with (wire + shift I), every line of a launch with the same matrix.
// TridiagTables holds one shifted wire's factorisation: chunked Thomas tables
// (P > 0, lines of up to kChunkMaxLen elements) or parallel cyclic reduction
// multipliers (longer lines, up to kTridiagMaxLen).
constexpr int kTridiagMaxLen = 8192;
constexpr int kChunkMaxLen = 2048;
struct TridiagTables {
    int len, levels, K, P;          // chunked: K elements per chunk, P chunks
    double g;                       // the wire's coupling
    double *q;                      // chunked: inverse pivots, K x P
    double *alpha, *gamma, *invb;   // PCR: levels x len, levels x len, len
    double *work;                   // PCR: 6 x len set-up scratch
};
size_t tridiag_table_doubles(int len);
TridiagTables tridiag_carve(double *base, int len, double g);
hipError_t launch_tridiag_setup(const Wire &w, double shift, const TridiagTables &t, hipStream_t s);
// both wires' set-ups (one launch when both are chunked)
hipError_t launch_tridiag_setup2(const Wire &w1, double shift1, const TridiagTables &t1,
                                 const Wire &w2, double shift2, const TridiagTables &t2,
                                 hipStream_t s);
// out = T^{-1} (in + in2_scale * in2) along `lines` lines; rows: lines are
// contiguous (elem_stride 1), else consecutive lines are adjacent (line_stride 1)
hipError_t launch_tridiag_solve(const TridiagTables &t, int lines, bool rows, size_t line_stride,
                                size_t elem_stride, const double *in, const double *in2,
                                double in2_scale, double *out, const int *skip, hipStream_t s);
// One block Gauss-Seidel sweep on the linearisation at V = 0 (a start for
// Newton's method): V_t = (G_t + D)^{-1} Y_t, V_b = (G_b + D)^{-1} D V_t with
// D = g_dev, by per-wire tridiagonal solves (lines of up to kSweepMaxLen).
constexpr int kSweepMaxLen = 2048;
hipError_t launch_sweep_guess(const Wire &top, const Wire &bot, int m, int n, double g_src,
                              const double *g_dev, const double *v_in, double *vt, double *vb,
                              hipStream_t s);
// z = r ./ diag(J(D))
hipError_t launch_jacobi(const mca_plan *P, const double *D, const double *rt, const double *rb,
                         double *zt, double *zb, const int *skip, hipStream_t s);

// Krylov kernels over vectors of even length len (= 2mn), 16-byte aligned.
// partial dot products x.y -> partials[reduce_blocks(len)] (any length)
hipError_t launch_dot_partials(const double *x, const double *y, size_t len,
                               double *partials, hipStream_t s);
// h = sum(partials_in); h_out[0] = h; w -= h * v_prev; partials_out = partial dots (w, v_next),
// or partial ||w||^2 when v_next == nullptr.
hipError_t launch_mgs_step(double *w, const double *v_prev, const double *v_next, size_t len,
                           const double *partials_in, double *partials_out, double *h_out,
                           hipStream_t s, const int *skip = nullptr);
// nrm = sqrt(sum(partials_in)); h_out[0] = nrm; w *= 1/nrm (when nrm > 0)
hipError_t launch_normalize(double *w, size_t len, const double *partials_in, double *h_out,
                            hipStream_t s, const int *skip = nullptr);

// One Arnoldi step j in two passes (modified Gram-Schmidt in compact WY form,
// see kernels.hip) over an unnormalised basis V (slot q holds u_q, v_q =
// sig_q u_q).  Pass 0: w = sig_j J z~_j with the projections on the basis.
// Pass 1: MGS's coefficients and w -= V h with the products of the new
// vector with the basis, then ||w||, the next row of L and the Givens update
// of column j (one block).  j + 1 <= kGsMaxV.
constexpr int kGsMaxV = 32;
constexpr int kGsBlocks = 1024;     // blocks of the update pass (and of longer first passes)
constexpr int kProjBlocks = 256;    // blocks of short first passes (every update block sums them)
constexpr int kGsFusedMaxV = 8;     // basis sizes whose coefficients the update blocks form
struct GsStep {
    int m, n, j;
    Wire top, bot;
    const double *d;              // device slopes D (m x n)
    const double *zt, *zb;        // preconditioned u_j (top, bottom layer)
    double *w;                    // slot j + 1 of V: the new vector (length 2mn)
    const double *V;              // slot 0 of V
    size_t ldv;                   // slot stride (2mn)
    double *sig;                  // sig_q (R + 1)
    double *L;                    // strictly lower V^T V, row-major, ld ldl
    int ldl;
    double *H;                    // Hessenberg, column-major, ld ldh
    int ldh;
    double *hcol;                 // H column j
    double *p1, *p2;              // partials: kGsMaxV and kGsMaxV + 1 values x kGsBlocks
    double *g, *cs, *sn, *resid;  // Givens state of the cycle
    double abs_tol;
    int *ctl;                     // cycle control block (stop flag first)
    int *snap;                    // device address of the host's snapshot slot of step j
                                  // (5 ints: the control block, then the marker)
    int epoch;                    // marker value written after the snapshot
    // with xp[0][0] set, the update pass also writes the new vector in the
    // reduced-precision preconditioner's operand format (per layer: FP32, or
    // bfloat16 hi [+ lo]), the conversion the next step's chain would make
    void *xp[2][2];
    int prec;
    // with fold_h (= m / 2) set as well, the planes take the persymmetric fold
    // of the new vector (rows i < m/2: x_i + x_{m-1-i}, rows m/2 + i:
    // x_i - x_{m-1-i}), the input of the folded chain
    int fold_h;
    // with post_rt set (literal form), pass 0 also forms the preconditioner's
    // last step z_b = ((G_t + a1 I) z_t - r_t) / a1 from z_t, stores it at
    // zb_store and uses it in place of zb
    const double *post_rt;
    double *zb_store;
    double post_a1, post_inv_a1;
    // optional device copies (Newton scalars, see launch_newton_next): with
    // shift set, post_a1 = shift[0] and post_inv_a1 = shift[1]; with tol set,
    // abs_tol = tol[0]
    const double *shift, *tol;
};
// pass 0: the Jacobian product with the projections; pass 1: the update;
// pass 2: ||w||, sig_{j+1}, row j + 1 of L, the Givens update and the snapshot
hipError_t launch_gs_step(const GsStep &g, int pass, hipStream_t s);
// pass 2 of step g.j together with the persymmetric literal form's first
// stencil and fold of the next step's preconditioner input (as
// launch_precond_pre_fold), in one launch
hipError_t launch_finish_fold(const GsStep &g, const mca_plan *P, double a1, double a2,
                              const double *rt, const double *rb, double *f, hipStream_t s,
                              const int *skip, const double *shift = nullptr);

// Newton scalars on the device (8 doubles): [0] a = sum D / mn (the shift
// a1 = a2 of eq. (P)), [1] 1 / a, [2] beta = ||F||, [3] -1 / beta, [4] the
// GMRES stop gmres_tol * beta.  launch_newton_next derives them from the
// residual's reduced sums (sums[0] = ||F||^2, sums[1] = sum D; may be pinned
// host memory) and starts the first GMRES cycle: g = (beta, 0, ...), sig[0] = 1
// (if sig), ctl = (stop, 0, running, 0) with stop set unless
// ||F||^2 <= accept2 and ||F||^2 > conv2 (both finite): a cycle enqueued
// ahead of the host's decision on the trial point then does nothing when
// the host is going to reject it or stop.
hipError_t launch_newton_next(const double *sums, double mn, double gmres_tol, double accept2,
                              double conv2, double *nsc, int *ctl, double *g, int R, double *sig,
                              hipStream_t s);
// y = x * alpha[0] (alpha on the device)
hipError_t launch_scale_dev(const double *x, const double *alpha, double *y, size_t len,
                            hipStream_t s);
// the persymmetric fold with the shift from the device (shift[0] = a, shift[1] = 1 / a)
hipError_t launch_precond_pre_fold_dev(const mca_plan *P, const double *shift, const double *rt,
                                       const double *rb, double *f, hipStream_t s,
                                       const int *skip);

// Device-side least squares of one GMRES cycle (see k_givens).
enum CycleReason { CYCLE_RUNNING = 0, CYCLE_CONVERGED = 1, CYCLE_BREAKDOWN = 2,
                   CYCLE_NONFINITE = 3 };
// sig (may be null): sig[0] = 1 (v_0 is stored normalised)
hipError_t launch_cycle_init(int *ctl, double *g, int R, double beta, hipStream_t s,
                             double *sig = nullptr);
// ... then ctl[0..3] written to snap (pinned host memory, device address)
// and snap[4] = epoch
hipError_t launch_givens(double *H, int ldh, int j, double *g, double *cs, double *sn,
                         double abs_tol, int *ctl, double *resid, int *snap, int epoch,
                         hipStream_t s);
hipError_t launch_backsolve(const double *H, int ldh, const double *g, const int *ctl,
                            double *y, hipStream_t s, const double *sig = nullptr);

// y = alpha * x
hipError_t launch_scale(const double *x, double alpha, double *y, size_t len, hipStream_t s);
// x (+)= sum_i coef[i] * Z[i], i < (kptr ? *kptr : k)   (coef on device)
hipError_t launch_update(const double *Z, size_t zstride, const double *coef, int k,
                         const int *kptr, size_t len, double *x, int accumulate, hipStream_t s);
// out = a + s * b
hipError_t launch_axpby(const double *a, double sc, const double *b, double *out, size_t len,
                        hipStream_t s);
// out = -(a + b)
hipError_t launch_neg_sum(const double *a, const double *b, double *out, size_t len,
                          hipStream_t s);
// fill with a value
hipError_t launch_fill(double *x, double v, size_t len, hipStream_t s);

}  // namespace mca
