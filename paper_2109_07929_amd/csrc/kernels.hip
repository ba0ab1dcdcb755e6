// kernels.hip -- HBM-bound kernels of the Newton-GMRES hot path (gfx950, FP64).
//
// Data layout: every crosspoint array is m x n row-major (index k = i*n + j,
// the paper's perpendicular natural indexing, Section III-A), and a Krylov
// vector of the coupled system is the top array followed by the bottom array
// (length 2mn, the paper's stacking [V_t; V_b] of eq. (F)).
//
// Wire stencils are written in branch-current form (dev::wire_apply), which
// equals the tridiagonal product exactly in real arithmetic and keeps the
// residual's rounding proportional to the branch currents.
#include "device_common.h"

namespace mca {
namespace {

using dev::block_sum;
using dev::sum_partials;
using dev::sinh_cosh;
using dev::TPB;
using dev::wire_apply;
using dev::xcd_run_chunk;

constexpr int kMaxReduceBlocks = 1024;

// --------------------------------------------------------------- residual
// F_t = G_t V_t + I - Y_t, F_b = G_b V_b - I (eqs. (MNA)/(F)); D = dI/du.
// partials[2*block + 0] = sum F^2, partials[2*block + 1] = sum D (skipped when null).
__global__ __launch_bounds__(TPB) void k_residual(
    int m, int n, Wire top, Wire bot, double v0, int linear,
    const double *__restrict__ gdev, const double *__restrict__ vin,
    const double *__restrict__ vt, const double *__restrict__ vb,
    double *__restrict__ ft, double *__restrict__ fb, double *__restrict__ d,
    double *__restrict__ partials)
{
    const size_t mn = (size_t)m * n;
    double acc[2] = {0.0, 0.0};
    const size_t k0 = (size_t)xcd_run_chunk(blockIdx.x, 0, gridDim.x) * TPB + threadIdx.x;
    for (size_t k = k0; k < mn; k += (size_t)gridDim.x * TPB) {
        const int i = (int)(k / n), j = (int)(k - (size_t)i * n);
        const double t = vt[k], b = vb[k];
        // top wire i along j; its first node is fed by the drive through g_src (= top.end0)
        double st = (j > 0) ? top.g * (t - vt[k - 1]) : top.end0 * (t - vin[i]);
        st += (j + 1 < n) ? top.g * (t - vt[k + 1]) : top.end1 * t;
        const double sb = wire_apply(bot, i, b, (i > 0) ? vb[k - n] : 0.0,
                                     (i + 1 < m) ? vb[k + n] : 0.0);
        const double u = t - b, g = gdev[k];
        double cur, slope;
        if (linear) {
            cur = g * u;
            slope = g;
        } else {
            double sh, ch;
            sinh_cosh(u / v0, sh, ch);
            cur = g * v0 * sh;
            slope = g * ch;
        }
        const double f1 = st + cur, f2 = sb - cur;
        ft[k] = f1;
        fb[k] = f2;
        if (d) d[k] = slope;
        acc[0] += f1 * f1 + f2 * f2;
        acc[1] += slope;
    }
    if (partials) {   // uniform across the grid
        block_sum<2>(acc);
        if (threadIdx.x == 0) {
            partials[2 * blockIdx.x + 0] = acc[0];
            partials[2 * blockIdx.x + 1] = acc[1];
        }
    }
}

__global__ __launch_bounds__(TPB) void k_reduce(const double *__restrict__ p, int nb, int nc,
                                                double *__restrict__ out, int *mark, int epoch)
{
    // one block; component c summed in a fixed order
    for (int c = 0; c < nc; ++c) {
        double v[1] = {0.0};
        for (int b = threadIdx.x; b < nb; b += TPB) v[0] += p[(size_t)b * nc + c];
        block_sum<1>(v);
        if (threadIdx.x == 0) out[c] = v[0];
    }
    // the sums are out (thread 0 stored them): publish them to a waiting host
    if (mark && threadIdx.x == 0)
        __hip_atomic_store(mark, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ---------------------------------------------------------------- Jacobian
// y_t = G_t x_t + d (x_t - x_b),  y_b = G_b x_b - d (x_t - x_b)     (eq. (J))
// With v0 (a Krylov vector of length 2mn, top half then bottom half) the
// kernel also leaves per-block partial sums of <y, v0> in partials: the first
// projection of the Arnoldi step, fused so that y is not read back.
__global__ __launch_bounds__(TPB) void k_jacobian(
    int m, int n, Wire top, Wire bot, const double *__restrict__ d,
    const double *__restrict__ xt, const double *__restrict__ xb,
    double *__restrict__ yt, double *__restrict__ yb, const double *__restrict__ v0,
    double *__restrict__ partials, const int *__restrict__ skip)
{
    if (skip && *skip) return;
    const size_t mn = (size_t)m * n;
    double acc[1] = {0.0};
    for (size_t k = (size_t)blockIdx.x * TPB + threadIdx.x; k < mn; k += (size_t)gridDim.x * TPB) {
        const int i = (int)(k / n), j = (int)(k - (size_t)i * n);
        const double t = xt[k], b = xb[k];
        const double st = wire_apply(top, j, t, (j > 0) ? xt[k - 1] : 0.0,
                                     (j + 1 < n) ? xt[k + 1] : 0.0);
        const double sb = wire_apply(bot, i, b, (i > 0) ? xb[k - n] : 0.0,
                                     (i + 1 < m) ? xb[k + n] : 0.0);
        const double c = d[k] * (t - b);
        const double y1 = st + c, y2 = sb - c;
        yt[k] = y1;
        yb[k] = y2;
        if (v0) acc[0] += y1 * v0[k] + y2 * v0[mn + k];
    }
    if (partials) {   // uniform across the grid
        block_sum<1>(acc);
        if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
    }
}

// ------------------------------------------------- literal-form stencils
// With A = G_t + a1 I, B = -a1 I, C = -a2 I, D = G_b + a2 I (eq. (P)),
// eq. (block) gives z_t = M^{-1} (r_b - D B^{-1} r_t) and z_b = B^{-1} (r_t - A z_t).
__global__ __launch_bounds__(TPB) void k_precond_pre(
    int m, int n, Wire bot, double inv_a1, double a2,
    const double *__restrict__ rt, const double *__restrict__ rb, double *__restrict__ w,
    const int *__restrict__ skip)
{
    if (skip && *skip) return;
    const size_t mn = (size_t)m * n;
    for (size_t k = (size_t)blockIdx.x * TPB + threadIdx.x; k < mn; k += (size_t)gridDim.x * TPB) {
        const int i = (int)(k / n);
        const double r = rt[k];
        const double s = wire_apply(bot, i, r, (i > 0) ? rt[k - n] : 0.0,
                                    (i + 1 < m) ? rt[k + n] : 0.0);
        w[k] = rb[k] + (s + a2 * r) * inv_a1;
    }
}

// w = r_b + ((G_b + a2 I) r_t) / a1 at rows i and m-1-i, folded: P = sum, Q = difference
// (with shift set: a2 = shift[0], 1 / a1 = shift[1] from the device)
__global__ __launch_bounds__(TPB) void k_precond_pre_fold(
    int m, int n, Wire bot, double inv_a1, double a2,
    const double *__restrict__ rt, const double *__restrict__ rb, double *__restrict__ f,
    const int *__restrict__ skip, const double *__restrict__ shift)
{
    if (skip && *skip) return;
    if (shift) {
        a2 = shift[0];
        inv_a1 = shift[1];
    }
    const int h = m / 2;
    const size_t hn = (size_t)h * n;
    auto w_at = [&](int i, int j) {
        const size_t k = (size_t)i * n + j;
        const double r = rt[k];
        const double s = wire_apply(bot, i, r, (i > 0) ? rt[k - n] : 0.0,
                                    (i + 1 < m) ? rt[k + n] : 0.0);
        return rb[k] + (s + a2 * r) * inv_a1;
    };
    const size_t k0 = (size_t)xcd_run_chunk(blockIdx.x, 0, gridDim.x) * TPB + threadIdx.x;
    for (size_t k = k0; k < hn; k += (size_t)gridDim.x * TPB) {
        const int i = (int)(k / n), j = (int)(k - (size_t)i * n);
        const double w0 = w_at(i, j), w1 = w_at(m - 1 - i, j);
        f[k] = w0 + w1;
        f[hn + k] = w0 - w1;
    }
}

__global__ __launch_bounds__(TPB) void k_unfold(const double *__restrict__ ys,
                                                const double *__restrict__ ya, int n, int h,
                                                double *__restrict__ xt, const int *__restrict__ skip)
{
    if (skip && *skip) return;
    const size_t nh = (size_t)n * h;
    const int m = 2 * h;
    for (size_t k = (size_t)blockIdx.x * TPB + threadIdx.x; k < nh; k += (size_t)gridDim.x * TPB) {
        const size_t j = k / h;
        const int i = (int)(k - j * h);
        const double s = ys[k], a = ya[k];
        xt[j * m + i] = s + a;
        xt[j * m + (m - 1 - i)] = s - a;
    }
}

__global__ __launch_bounds__(TPB) void k_precond_post(
    int m, int n, Wire top, double a1, double inv_a1,
    const double *__restrict__ zt, const double *__restrict__ rt, double *__restrict__ zb,
    const int *__restrict__ skip)
{
    if (skip && *skip) return;
    const size_t mn = (size_t)m * n;
    for (size_t k = (size_t)blockIdx.x * TPB + threadIdx.x; k < mn; k += (size_t)gridDim.x * TPB) {
        const int j = (int)(k % n);
        const double z = zt[k];
        const double s = wire_apply(top, j, z, (j > 0) ? zt[k - 1] : 0.0,
                                    (j + 1 < n) ? zt[k + 1] : 0.0);
        zb[k] = (s + a1 * z - rt[k]) * inv_a1;
    }
}

// ------------------------------------------------------------------ Krylov
// Krylov vectors have even length and 16-byte aligned starts, so these
// kernels stream them as double2 pairs (len2 = len / 2).
__global__ __launch_bounds__(TPB) void k_dot_partials(
    const double *__restrict__ x, const double *__restrict__ y, size_t len,
    double *__restrict__ partials)
{
    double acc[1] = {0.0};
    for (size_t k = (size_t)blockIdx.x * TPB + threadIdx.x; k < len; k += (size_t)gridDim.x * TPB)
        acc[0] += x[k] * y[k];
    block_sum<1>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

// One modified Gram-Schmidt step fused with the next projection:
//   h = <w, v_prev> (summed from the previous pass's partials); w -= h v_prev;
//   partial <w, v_next>  (or partial ||w||^2 when v_next is null).
__global__ __launch_bounds__(TPB) void k_mgs_step(
    double *__restrict__ w, const double *__restrict__ vprev, const double *__restrict__ vnext,
    size_t len2, const double *__restrict__ pin, int nb, double *__restrict__ pout,
    double *__restrict__ hout, const int *__restrict__ skip)
{
    if (skip && *skip) return;
    const double h = sum_partials(pin, nb);
    if (blockIdx.x == 0 && threadIdx.x == 0) hout[0] = h;
    double2 *w2 = reinterpret_cast<double2 *>(w);
    const double2 *p2 = reinterpret_cast<const double2 *>(vprev);
    const double2 *n2 = reinterpret_cast<const double2 *>(vnext);
    double acc[1] = {0.0};
    if (vnext) {
        for (size_t k = (size_t)blockIdx.x * TPB + threadIdx.x; k < len2; k += (size_t)gridDim.x * TPB) {
            double2 x = w2[k];
            const double2 p = p2[k], q = n2[k];
            x.x -= h * p.x;
            x.y -= h * p.y;
            w2[k] = x;
            acc[0] += x.x * q.x + x.y * q.y;
        }
    } else {
        for (size_t k = (size_t)blockIdx.x * TPB + threadIdx.x; k < len2; k += (size_t)gridDim.x * TPB) {
            double2 x = w2[k];
            const double2 p = p2[k];
            x.x -= h * p.x;
            x.y -= h * p.y;
            w2[k] = x;
            acc[0] += x.x * x.x + x.y * x.y;
        }
    }
    block_sum<1>(acc);
    if (threadIdx.x == 0) pout[blockIdx.x] = acc[0];
}

__global__ __launch_bounds__(TPB) void k_normalize(
    double *__restrict__ w, size_t len2, const double *__restrict__ pin, int nb,
    double *__restrict__ hout, const int *__restrict__ skip)
{
    if (skip && *skip) return;
    const double nrm = sqrt(sum_partials(pin, nb));
    if (blockIdx.x == 0 && threadIdx.x == 0) hout[0] = nrm;
    if (!(nrm > 0.0)) return;
    const double inv = 1.0 / nrm;
    double2 *w2 = reinterpret_cast<double2 *>(w);
    for (size_t k = (size_t)blockIdx.x * TPB + threadIdx.x; k < len2; k += (size_t)gridDim.x * TPB) {
        double2 x = w2[k];
        x.x *= inv;
        x.y *= inv;
        w2[k] = x;
    }
}

// ----------------------------- two-pass Gram-Schmidt (MGS, compact WY form)
// Modified Gram-Schmidt applies the elementary projections I - v_k v_k^T,
// k = 0..j, one after another.  Their product equals I - V T V^T with
// T^{-1} = I + L, L the strictly lower triangle of V^T V (for unit v_k), and
// MGS's coefficients are h = T (V^T w).  So one pass over the basis gives the
// projections s = V^T w, a forward substitution (I + L) h = s gives MGS's h,
// and a second pass forms w - V h.  L grows by one row per step: the second
// pass also leaves the products of the new vector with the basis.
//
// The basis is kept unnormalised: slot q holds u_q with v_q = sig_q u_q
// (sig_q = 1 / ||u_q||, sig_0 = 1).  The preconditioner is linear, so it is
// applied to u_j, and the Jacobian product is scaled by sig_j instead;
// the least-squares coefficients take the factors sig_j before the update.
//
// The two streaming passes leave per-block partials (value q at
// partials[q * gridDim.x + block]).  The update pass's blocks each sum the
// first pass's partials themselves (kProjBlocks of them per value); a
// one-block kernel after the update pass sums its partials and does the rest
// of the step's small dense work.

// Sums of nval values' partials (nb <= 1024 each, value q at p[q * nb +
// block]) by a block of 1024 threads: thread t loads partial t of every
// value at once, then a fixed-order tree; out[q] in LDS.
__device__ __forceinline__ void sum_partials_1024(const double *__restrict__ p, int nval, int nb,
                                                  double *out)
{
    __shared__ double red[kGsMaxV + 1][16];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double v[kGsMaxV + 1];
#pragma unroll
    for (int q = 0; q <= kGsMaxV; ++q) v[q] = (q < nval && t < nb) ? p[(size_t)q * nb + t] : 0.0;
#pragma unroll
    for (int q = 0; q <= kGsMaxV; ++q) {
        if (q < nval) {
            const double x = dev::wave_sum(v[q]);
            if (lane == 0) red[q][wave] = x;
        }
    }
    __syncthreads();
    if (t < nval) {
        double x = 0.0;
        for (int w = 0; w < 16; ++w) x += red[t][w];
        out[t] = x;
    }
    __syncthreads();
}

// Copy of the cycle control block (stop flag, steps done, reason) to the
// host's pinned snapshot slot (16-byte aligned), then the slot's marker
// (snap[4]) set to `epoch` with a release store at system scope: a host that
// reads the marker with acquire order sees the control block.
__device__ __forceinline__ void write_snapshot(int *snap, const int *ctl, int epoch)
{
    *reinterpret_cast<int4 *>(snap) = int4{ctl[0], ctl[1], ctl[2], ctl[3]};
    __hip_atomic_store(snap + 4, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Givens update of Hessenberg column j: apply rotations 0..j-1, then the
// rotation that zeroes h[j+1]; update g and stop the cycle when
// |g[j+1]| <= abs_tol (the GMRES residual).  Every thread of the block calls
// it (the column and the rotations are staged in LDS by all of them); thread
// 0 does the arithmetic.  hlast: the value of h[j+1].
__device__ void givens_block(double *__restrict__ H, int ldh, int j, double hlast,
                             double *__restrict__ g, double *__restrict__ cs,
                             double *__restrict__ sn, double abs_tol, int *__restrict__ ctl,
                             double *__restrict__ resid)
{
    __shared__ double hs[MCA_MAX_RESTART + 1], cz[MCA_MAX_RESTART], sz[MCA_MAX_RESTART];
    double *h = H + (size_t)j * ldh;
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        hs[i] = h[i];
        if (i < j) {
            cz[i] = cs[i];
            sz[i] = sn[i];
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double hj1 = hlast;
    bool bad = !isfinite(hj1);
    for (int i = 0; i <= j; ++i) bad = bad || !isfinite(hs[i]);
    if (bad) {
        ctl[0] = 1;
        ctl[2] = CYCLE_NONFINITE;
        return;
    }
    for (int i = 0; i < j; ++i) {   // rotation i mixes rows i and i + 1 <= j
        const double t = cz[i] * hs[i] + sz[i] * hs[i + 1];
        hs[i + 1] = -sz[i] * hs[i] + cz[i] * hs[i + 1];
        hs[i] = t;
    }
    for (int i = 0; i < j; ++i) h[i] = hs[i];
    const double r = hypot(hs[j], hj1);
    if (r == 0.0) {
        h[j] = hs[j];
        h[j + 1] = hj1;
        ctl[0] = 1;
        ctl[2] = CYCLE_BREAKDOWN;
        return;
    }
    const double c = hs[j] / r, sv = hj1 / r;
    cs[j] = c;
    sn[j] = sv;
    h[j] = r;
    h[j + 1] = 0.0;
    const double gj = g[j];
    g[j + 1] = -sv * gj;
    g[j] = c * gj;
    ctl[1] = j + 1;
    resid[j] = fabs(sv * gj);
    if (fabs(sv * gj) <= abs_tol) {   // includes hj1 == 0 (invariant subspace)
        ctl[0] = 1;
        ctl[2] = CYCLE_CONVERGED;
    }
}

// w = sig_j J z~_j (eq. (J); z~_j the preconditioned u_j) with the partials of
// <w, u_q>, q <= j.  POST: z~_j's bottom half comes from its top half here
// (the literal form's last step, eq. (block)): z_b = ((G_t + a1 I) z_t - r_t)
// / a1 with the arithmetic of k_precond_post, stored for the solution update.
// The bottom wire's stencil needs z_b at the rows above and below, so a POST
// thread walks a strip of kPostRows rows of one column and rolls z_t's row
// triple and z_b down it (each z_b formed (kPostRows + 2) / kPostRows times).
constexpr int kPostRows = 4;

template <int MAXV, int NT, bool POST>
__global__ __launch_bounds__(NT) void k_jacobian_proj(GsStep a)
{
    if (*a.ctl) return;
    const int m = a.m, n = a.n, j = a.j, nv = j + 1;
    const size_t mn = (size_t)m * n;
    const double sj = a.sig[j];
    double acc[MAXV];
#pragma unroll
    for (int q = 0; q < MAXV; ++q) acc[q] = 0.0;
    // one crosspoint: t = z_t, st = top stencil of z_t, b / bm / bp = z_b here,
    // one row up, one row down
    auto point = [&](size_t k, int i, double t, double st, double b, double bm, double bp) {
        const double sb = wire_apply(a.bot, i, b, bm, bp);
        const double c = a.d[k] * (t - b);
        const double y1 = sj * (st + c), y2 = sj * (sb - c);
        a.w[k] = y1;
        a.w[mn + k] = y2;
#pragma unroll
        for (int q = 0; q < MAXV; ++q)
            if (q < nv) acc[q] += y1 * a.V[q * a.ldv + k] + y2 * a.V[q * a.ldv + mn + k];
    };
    if constexpr (POST) {
        const double pa1 = a.shift ? a.shift[0] : a.post_a1;
        const double pinv = a.shift ? a.shift[1] : a.post_inv_a1;
        const int strips = (m + kPostRows - 1) / kPostRows;
        const size_t units = (size_t)strips * n;
#pragma unroll 1
        for (size_t u = (size_t)blockIdx.x * NT + threadIdx.x; u < units; u += (size_t)gridDim.x * NT) {
            const int sx = (int)(u / n), jj = (int)(u - (size_t)sx * n);
            const int i0 = sx * kPostRows, i1 = min(i0 + kPostRows, m);
            auto row = [&](int i, double &zl, double &zc, double &zr) {
                const size_t kk = (size_t)i * n + jj;
                zc = a.zt[kk];
                zl = (jj > 0) ? a.zt[kk - 1] : 0.0;
                zr = (jj + 1 < n) ? a.zt[kk + 1] : 0.0;
            };
            auto zb_of = [&](int i, double zl, double zc, double zr) {
                const double s = wire_apply(a.top, jj, zc, zl, zr);
                return (s + pa1 * zc - a.post_rt[(size_t)i * n + jj]) * pinv;
            };
            double cl, cc, cr;
            row(i0, cl, cc, cr);
            double bc = zb_of(i0, cl, cc, cr), bprev = 0.0;
            if (i0 > 0) {
                double pl, pc, pr;
                row(i0 - 1, pl, pc, pr);
                bprev = zb_of(i0 - 1, pl, pc, pr);
            }
#pragma unroll 1
            for (int i = i0; i < i1; ++i) {
                double nl = 0.0, nc = 0.0, nr = 0.0, bnext = 0.0;
                if (i + 1 < m) {
                    row(i + 1, nl, nc, nr);
                    bnext = zb_of(i + 1, nl, nc, nr);
                }
                const size_t k = (size_t)i * n + jj;
                a.zb_store[k] = bc;
                point(k, i, cc, wire_apply(a.top, jj, cc, cl, cr), bc, bprev, bnext);
                bprev = bc;
                bc = bnext;
                cl = nl;
                cc = nc;
                cr = nr;
            }
        }
    } else {
#pragma unroll 1
        for (size_t k = (size_t)blockIdx.x * NT + threadIdx.x; k < mn; k += (size_t)gridDim.x * NT) {
            const int i = (int)(k / n), jj = (int)(k - (size_t)i * n);
            const double t = a.zt[k];
            const double st = wire_apply(a.top, jj, t, (jj > 0) ? a.zt[k - 1] : 0.0,
                                         (jj + 1 < n) ? a.zt[k + 1] : 0.0);
            point(k, i, t, st, a.zb[k], (i > 0) ? a.zb[k - n] : 0.0,
                  (i + 1 < m) ? a.zb[k + n] : 0.0);
        }
    }
    dev::block_store_sums<MAXV, NT>(acc, nv, a.p1 + blockIdx.x, gridDim.x);
}

// Longer bases (j + 1 > kGsFusedMaxV): one block of 1024 threads forms
// s_q = sig_q <w, u_q> from the first pass's kGsBlocks partials, then
// (I + L) h = s by forward substitution with rows 0..j of L; h to H column j.
__global__ __launch_bounds__(1024) void k_gs_coef(GsStep a)
{
    if (*a.ctl) return;
    const int j = a.j, nv = j + 1;
    __shared__ double sv[kGsMaxV + 1];
    __shared__ double Ls[kGsMaxV][kGsMaxV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int e = threadIdx.x; e < nv * kGsMaxV; e += 1024) {
        const int r = e / kGsMaxV, k = e - r * kGsMaxV;
        if (k < r) Ls[r][k] = a.L[(size_t)r * a.ldl + k];
    }
    sum_partials_1024(a.p1, nv, kGsBlocks, sv);
    if (wave != 0) return;
    if (lane < nv) sv[lane] *= a.sig[lane];   // s_q = sig_q <w, u_q>
    double h = 0.0;     // lane k holds h_k
    for (int r = 0; r <= j; ++r) {
        // h_r = s_r - sum_{k < r} L[r][k] h_k
        double t = (lane < r) ? Ls[r][lane] * h : 0.0;
        t = dev::wave_sum(t);
        const double hr = sv[r] - t;
        if (lane == r) h = hr;
        if (lane == 0) a.hcol[r] = hr;
    }
}

// Second pass.  With PRO (j + 1 <= kGsFusedMaxV) every block first forms
// MGS's coefficients itself: s_q = sig_q <w, u_q> from the first pass's
// kProjBlocks partials (the same fixed order in every block), then
// (I + L) h = s by forward substitution with rows 0..j of L; block 0 stores h
// in H column j.  Without PRO, k_gs_coef has stored h.  Then
// x = w - sum_q h_q sig_q u_q (q <= j, in order) is stored as u_{j+1}, with
// the partials of <x, u_q> (values 0..j) and ||x||^2 (value j + 1).
template <int MAXV, bool PRO, int NT>
__global__ __launch_bounds__(NT) void k_gs_update(GsStep a)
{
    if (*a.ctl) return;
    const int j = a.j, nv = j + 1;
    __shared__ double hsh[kGsMaxV];
    if constexpr (!PRO) {
        for (int q = threadIdx.x; q < nv; q += NT) hsh[q] = a.hcol[q];
        __syncthreads();
    } else {
        __shared__ double sv[kGsMaxV];
        __shared__ double Ls[kGsMaxV][kGsMaxV];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        for (int q = wave; q < nv; q += NT / 64) {
            double x = 0.0;
#pragma unroll
            for (int u = 0; u < kProjBlocks / 64; ++u) x += a.p1[(size_t)q * kProjBlocks + lane + 64 * u];
            x = dev::wave_sum(x);
            if (lane == 0) sv[q] = a.sig[q] * x;
        }
        for (int e = threadIdx.x; e < nv * kGsMaxV; e += NT) {
            const int r = e / kGsMaxV, k = e - r * kGsMaxV;
            if (k < r) Ls[r][k] = a.L[(size_t)r * a.ldl + k];
        }
        __syncthreads();
        if (wave == 0) {
            double h = 0.0;     // lane k holds h_k
            for (int r = 0; r <= j; ++r) {
                // h_r = s_r - sum_{k < r} L[r][k] h_k
                double t = (lane < r) ? Ls[r][lane] * h : 0.0;
                t = dev::wave_sum(t);
                const double hr = sv[r] - t;
                if (lane == r) h = hr;
                if (lane == 0) {
                    hsh[r] = hr;
                    if (blockIdx.x == 0) a.hcol[r] = hr;
                }
            }
        }
        __syncthreads();
    }
    double c[MAXV], acc[MAXV + 1];
#pragma unroll
    for (int q = 0; q < MAXV; ++q) c[q] = (q < nv) ? hsh[q] * a.sig[q] : 0.0;
#pragma unroll
    for (int q = 0; q <= MAXV; ++q) acc[q] = 0.0;
    // pairs of elements (the vector length 2mn and the slot stride are even).
    // The grid walks the vectors from their end back to their start: the first
    // pass of this Arnoldi step read them front to back just before, so the
    // parts it read last are the likeliest still in the memory-side cache.
    double2 *w2 = reinterpret_cast<double2 *>(a.w);
    const double2 *V2 = reinterpret_cast<const double2 *>(a.V);
    const size_t len2 = (size_t)a.m * a.n, ldv2 = a.ldv / 2;
    const size_t first = (size_t)blockIdx.x * NT + threadIdx.x, stride = (size_t)gridDim.x * NT;
    // w -= sum_q c_q v_q at pair k, with the partial sums
    auto update = [&](size_t k) -> double2 {
        double2 vq[MAXV];
        double2 x = w2[k];
#pragma unroll
        for (int q = 0; q < MAXV; ++q) {
            vq[q] = (q < nv) ? V2[q * ldv2 + k] : double2{0.0, 0.0};
            x.x -= c[q] * vq[q].x;
            x.y -= c[q] * vq[q].y;
        }
        w2[k] = x;
#pragma unroll
        for (int q = 0; q < MAXV; ++q) acc[q] += x.x * vq[q].x + x.y * vq[q].y;
        acc[MAXV] += x.x * x.x + x.y * x.y;
        return x;
    };
    // as k_split: FP64 -> FP32 -> bfloat16 hi, lo = rest
    auto put = [&](int layer, size_t e, double v) {
        const float f = (float)v;
        if (a.prec == MCA_PREC_FP32) {
            static_cast<float *>(a.xp[layer][0])[e] = f;
        } else {
            const __bf16 hi = (__bf16)f;
            static_cast<__bf16 *>(a.xp[layer][0])[e] = hi;
            if (a.prec == MCA_PREC_BF16X3) static_cast<__bf16 *>(a.xp[layer][1])[e] = (__bf16)(f - (float)hi);
        }
    };
    if (a.xp[0][0] && a.fold_h) {
        // the folded chain's input: pairs of rows (i, m - 1 - i), written as
        // row i (sum) and row h + i (difference)
        const size_t half = (size_t)a.fold_h * a.n, mn = len2;
        if constexpr (MAXV <= 4) {
            // two columns at a time where n is even
            if (a.n % 2 == 0) {
                const int n2 = a.n / 2;
                const size_t half2 = half / 2, units = 2 * half2, layer2 = len2 / 2;
                const size_t steps = first < units ? (units - 1 - first) / stride + 1 : 0;
#pragma unroll 1
                for (size_t t = steps; t-- > 0;) {
                    const size_t u = first + t * stride;
                    const int layer = u < half2 ? 0 : 1;
                    const size_t r = u - layer * half2;
                    const int i = (int)(r / n2), c2 = (int)(r - (size_t)i * n2);
                    const double2 x0 = update(layer * layer2 + r);
                    const double2 x1 = update(layer * layer2 + (size_t)(a.m - 1 - i) * n2 + c2);
                    put(layer, 2 * r, x0.x + x1.x);
                    put(layer, 2 * r + 1, x0.y + x1.y);
                    put(layer, 2 * r + half, x0.x - x1.x);
                    put(layer, 2 * r + 1 + half, x0.y - x1.y);
                }
                goto folded_done;
            }
        }
        {
            // one element of each row per thread (a pair of double2 with eight
            // basis vectors would not fit the registers of 1024-thread blocks)
            const size_t units = 2 * half;
            const size_t steps = first < units ? (units - 1 - first) / stride + 1 : 0;
            auto update1 = [&](size_t e) -> double {
                double vq[MAXV];
                double x = a.w[e];
#pragma unroll
                for (int q = 0; q < MAXV; ++q) {
                    vq[q] = (q < nv) ? a.V[q * a.ldv + e] : 0.0;
                    x -= c[q] * vq[q];
                }
                a.w[e] = x;
#pragma unroll
                for (int q = 0; q < MAXV; ++q) acc[q] += x * vq[q];
                acc[MAXV] += x * x;
                return x;
            };
#pragma unroll 1
            for (size_t t = steps; t-- > 0;) {
                const size_t u = first + t * stride;
                const int layer = u < half ? 0 : 1;
                const size_t r = u - layer * half;
                const int i = (int)(r / a.n), jj = (int)(r - (size_t)i * a.n);
                const double x0 = update1(layer * mn + r);
                const double x1 = update1(layer * mn + (size_t)(a.m - 1 - i) * a.n + jj);
                put(layer, r, x0 + x1);
                put(layer, r + half, x0 - x1);
            }
        }
    folded_done:;
    } else {
        // pairs of elements (the vector length 2mn and the slot stride are even).
        // The grid walks the vectors from their end back to their start: the first
        // pass of this Arnoldi step read them front to back just before, so the
        // parts it read last are the likeliest still in the memory-side cache.
        const size_t steps = first < len2 ? (len2 - 1 - first) / stride + 1 : 0;
#pragma unroll 1
        for (size_t t = steps; t-- > 0;) {
            const size_t k = first + t * stride;
            const double2 x = update(k);
            if (a.xp[0][0]) {
                const size_t mn = (size_t)a.m * a.n;
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    size_t e = 2 * k + hh;
                    const int layer = e < mn ? 0 : 1;
                    e -= layer * mn;
                    put(layer, e, hh ? x.y : x.x);
                }
            }
        }
    }
    // block sums of <x, u_q> (q < nv) and ||x||^2 as values 0..nv
    __shared__ double sh[MAXV + 1][NT / 64];
    {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int q = 0; q <= MAXV; ++q) {
            if (q < nv || q == MAXV) {
                const double t = dev::wave_sum(acc[q]);
                if (lane == 0) sh[q][wave] = t;
            }
        }
    }
    __syncthreads();
    if ((int)threadIdx.x <= nv) {
        const int q = ((int)threadIdx.x < nv) ? (int)threadIdx.x : MAXV;
        double t = 0.0;
        for (int w = 0; w < NT / 64; ++w) t += sh[q][w];
        a.p2[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// One block of 1024 threads: ||x|| and <x, u_q> from the partials give
// H[j+1][j] = ||x||, sig_{j+1} and row j + 1 of L; then the Givens update of
// column j and the snapshot.  Every load the block needs (the stop flag, the
// partials, Hessenberg column j, the rotations, g[j], the scales) is issued
// before any of them is used: the kernel is a chain of dependent steps, and
// that keeps it to one memory round trip before the arithmetic.
// (the body runs in a block of 1024 threads, in k_gs_finish or as block 0 of
// k_finish_fold)
__device__ __forceinline__ void gs_finish_block(const GsStep &a)
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int j = a.j, nv = j + 1;
    const int nb = (nv <= kGsFusedMaxV) ? kProjBlocks : kGsBlocks;
    const int stop = a.ctl[0];
    double v[kGsMaxV + 1];
#pragma unroll
    for (int q = 0; q <= kGsMaxV; ++q) v[q] = (q <= nv && t < nb) ? a.p2[(size_t)q * nb + t] : 0.0;
    __shared__ double hs[MCA_MAX_RESTART + 1], cz[MCA_MAX_RESTART], sz[MCA_MAX_RESTART];
    __shared__ double sgs[kGsMaxV + 1], gj;
    if (t <= j) {
        hs[t] = a.hcol[t];
        sgs[t] = a.sig[t];
        if (t < j) {
            cz[t] = a.cs[t];
            sz[t] = a.sn[t];
        }
    }
    if (t == 0) gj = a.g[j];
    if (stop) {   // a stopped cycle: the snapshot only
        if (t == 0) write_snapshot(a.snap, a.ctl, a.epoch);
        return;
    }
    // fixed-order sums of the partials: waves, then the 16 wave sums
    __shared__ double red[kGsMaxV + 1][16];
    __shared__ double sv[kGsMaxV + 1];
#pragma unroll
    for (int q = 0; q <= kGsMaxV; ++q) {
        if (q <= nv) {
            const double x = dev::wave_sum(v[q]);
            if (lane == 0) red[q][wave] = x;
        }
    }
    __syncthreads();
    if (t <= nv) {
        double x = 0.0;
        for (int w = 0; w < 16; ++w) x += red[t][w];
        sv[t] = x;
    }
    __syncthreads();
    const double nrm = sqrt(sv[nv]);
    const double inv = (nrm > 0.0) ? 1.0 / nrm : 0.0;
    // row j + 1 of L: <v_{j+1}, v_q> = sig_q <x, u_q> / ||x||
    if (t < nv) a.L[(size_t)(j + 1) * a.ldl + t] = sv[t] * sgs[t] * inv;
    if (t != 0) return;
    a.sig[j + 1] = inv;
    // Givens update of column j (hs: h[0..j], h[j+1] = nrm)
    int *ctl = a.ctl;
    double *h = a.hcol;
    bool bad = !isfinite(nrm);
    for (int i = 0; i <= j; ++i) bad = bad || !isfinite(hs[i]);
    if (bad) {
        ctl[0] = 1;
        ctl[2] = CYCLE_NONFINITE;
    } else {
        for (int i = 0; i < j; ++i) {   // rotation i mixes rows i and i + 1 <= j
            const double u = cz[i] * hs[i] + sz[i] * hs[i + 1];
            hs[i + 1] = -sz[i] * hs[i] + cz[i] * hs[i + 1];
            hs[i] = u;
        }
        for (int i = 0; i < j; ++i) h[i] = hs[i];
        const double r = hypot(hs[j], nrm);
        if (r == 0.0) {
            h[j] = hs[j];
            h[j + 1] = nrm;
            ctl[0] = 1;
            ctl[2] = CYCLE_BREAKDOWN;
        } else {
            const double c = hs[j] / r, sn = nrm / r;
            a.cs[j] = c;
            a.sn[j] = sn;
            h[j] = r;
            h[j + 1] = 0.0;
            a.g[j + 1] = -sn * gj;
            a.g[j] = c * gj;
            ctl[1] = j + 1;
            a.resid[j] = fabs(sn * gj);
            if (fabs(sn * gj) <= (a.tol ? a.tol[0] : a.abs_tol)) {   // includes nrm == 0
                ctl[0] = 1;
                ctl[2] = CYCLE_CONVERGED;
            }
        }
    }
    write_snapshot(a.snap, ctl, a.epoch);
}

__global__ __launch_bounds__(1024) void k_gs_finish(GsStep a) { gs_finish_block(a); }

// The finish of Arnoldi step j - 1 (block 0, dispatched first) and the fold that starts step
// j's literal preconditioner (the other blocks, as k_precond_pre_fold) in one
// launch: the two are independent (the preconditioner is applied to the
// unnormalised u_j, which needs no sigma), and the finish, a chain of
// dependent steps in one workgroup, then no longer takes a launch of its own.
// The fold blocks skip on the stop flag as it stands when they start (the
// finish may set it meanwhile; the products after them read it again).
struct FoldArgs {
    int m, n;
    Wire bot;
    double inv_a1, a2;
    const double *shift;    // optional: a2 = shift[0], 1 / a1 = shift[1] (device)
    const double *rt, *rb;
    double *f;
    const int *skip;
};

__global__ __launch_bounds__(1024) void k_finish_fold(GsStep g, FoldArgs a)
{
    if (blockIdx.x == 0) {
        gs_finish_block(g);
        return;
    }
    if (a.skip && *a.skip) return;
    const int m = a.m, n = a.n, h = m / 2;
    const size_t hn = (size_t)h * n;
    const double a2 = a.shift ? a.shift[0] : a.a2, inv_a1 = a.shift ? a.shift[1] : a.inv_a1;
    auto w_at = [&](int i, int j) {
        const size_t k = (size_t)i * n + j;
        const double r = a.rt[k];
        const double s = wire_apply(a.bot, i, r, (i > 0) ? a.rt[k - n] : 0.0,
                                    (i + 1 < m) ? a.rt[k + n] : 0.0);
        return a.rb[k] + (s + a2 * r) * inv_a1;
    };
    // fold workgroups 1 .. F, in runs of rows per XCD
    const int F = gridDim.x - 1, chunk = xcd_run_chunk(blockIdx.x, 1, F);
    const size_t stride = (size_t)F * 1024;
    for (size_t k = (size_t)chunk * 1024 + threadIdx.x; k < hn; k += stride) {
        const int i = (int)(k / n), j = (int)(k - (size_t)i * n);
        const double w0 = w_at(i, j), w1 = w_at(m - 1 - i, j);
        a.f[k] = w0 + w1;
        a.f[hn + k] = w0 - w1;
    }
}

// ------------------------------------------- least squares on the device
// Control block of one GMRES cycle: ctl[0] stop flag (read by every kernel
// of later Arnoldi steps), ctl[1] iterations completed, ctl[2] reason.
// ls: g[R+1] (rotated right-hand side), cs[R], sn[R] (Givens rotations).
__global__ void k_cycle_init(int *__restrict__ ctl, double *__restrict__ g, int R, double beta,
                             double *__restrict__ sig)
{
    for (int i = threadIdx.x; i <= R; i += blockDim.x) g[i] = (i == 0) ? beta : 0.0;
    if (threadIdx.x == 0) {
        ctl[0] = 0;
        ctl[1] = 0;
        ctl[2] = CYCLE_RUNNING;
        if (sig) sig[0] = 1.0;
    }
}

// One Givens update of Hessenberg column j (givens_block), then the snapshot.
__global__ void k_givens(double *__restrict__ H, int ldh, int j, double *__restrict__ g,
                         double *__restrict__ cs, double *__restrict__ sn, double abs_tol,
                         int *__restrict__ ctl, double *__restrict__ resid, int *__restrict__ snap,
                         int epoch)
{
    if (ctl[0]) {
        if (threadIdx.x == 0) write_snapshot(snap, ctl, epoch);
        return;
    }
    const double hlast = H[(size_t)j * ldh + j + 1];
    givens_block(H, ldh, j, hlast, g, cs, sn, abs_tol, ctl, resid);
    if (threadIdx.x == 0) write_snapshot(snap, ctl, epoch);
}

// y = R^{-1} g over the ctl[1] completed columns (upper triangular R in H).
// With sig (an unnormalised basis, v_i = sig_i u_i) y_i is then scaled by
// sig_i: the update sums y_i sig_i times the preconditioned u_i.
__global__ void k_backsolve(const double *__restrict__ H, int ldh, const double *__restrict__ g,
                            const int *__restrict__ ctl, double *__restrict__ y,
                            const double *__restrict__ sig)
{
    if (threadIdx.x != 0) return;
    const int k = ctl[1];
    for (int i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int c = i + 1; c < k; ++c) t -= H[(size_t)c * ldh + i] * y[c];
        y[i] = t / H[(size_t)i * ldh + i];
    }
    if (sig)
        for (int i = 0; i < k; ++i) y[i] *= sig[i];
}

__global__ __launch_bounds__(TPB) void k_scale(const double *__restrict__ x, double alpha,
                                               double *__restrict__ y, size_t len)
{
    for (size_t k = (size_t)blockIdx.x * TPB + threadIdx.x; k < len; k += (size_t)gridDim.x * TPB)
        y[k] = alpha * x[k];
}

// x (+)= sum_{v < nvec} coef[v] Z_v, nvec = *kptr (device) when kptr is given
__global__ __launch_bounds__(TPB) void k_update(
    const double *__restrict__ Z, size_t zstride, const double *__restrict__ coef, int nvec,
    const int *__restrict__ kptr, size_t len2, double *__restrict__ x, int accumulate)
{
    if (kptr) nvec = *kptr;
    double2 *x2 = reinterpret_cast<double2 *>(x);
    for (size_t k = (size_t)blockIdx.x * TPB + threadIdx.x; k < len2; k += (size_t)gridDim.x * TPB) {
        double2 s = accumulate ? x2[k] : double2{0.0, 0.0};
        for (int v = 0; v < nvec; ++v) {
            const double2 z = reinterpret_cast<const double2 *>(Z + (size_t)v * zstride)[k];
            const double c = coef[v];
            s.x += c * z.x;
            s.y += c * z.y;
        }
        x2[k] = s;
    }
}

__global__ __launch_bounds__(TPB) void k_axpby(const double *__restrict__ a, double sc,
                                               const double *__restrict__ b,
                                               double *__restrict__ out, size_t len)
{
    for (size_t k = (size_t)blockIdx.x * TPB + threadIdx.x; k < len; k += (size_t)gridDim.x * TPB)
        out[k] = a[k] + sc * b[k];
}

__global__ __launch_bounds__(TPB) void k_neg_sum(const double *__restrict__ a,
                                                 const double *__restrict__ b,
                                                 double *__restrict__ out, size_t len)
{
    for (size_t k = (size_t)blockIdx.x * TPB + threadIdx.x; k < len; k += (size_t)gridDim.x * TPB)
        out[k] = -(a[k] + b[k]);
}

__global__ __launch_bounds__(TPB) void k_fill(double *__restrict__ x, double v, size_t len)
{
    for (size_t k = (size_t)blockIdx.x * TPB + threadIdx.x; k < len; k += (size_t)gridDim.x * TPB)
        x[k] = v;
}

int elementwise_blocks(size_t len)
{
    size_t b = (len + TPB - 1) / TPB;
    if (b > 8192) b = 8192;
    return b < 1 ? 1 : (int)b;
}

}  // namespace

int reduce_blocks(size_t len)
{
    size_t b = (len + 4 * TPB - 1) / (4 * TPB);
    if (b > (size_t)kMaxReduceBlocks) b = kMaxReduceBlocks;
    return b < 1 ? 1 : (int)b;
}

hipError_t launch_residual(const mca_plan *P, const double *g_dev, const double *v_in,
                           const double *vt, const double *vb, double *ft, double *fb,
                           double *d, double *partials, hipStream_t s)
{
    const int m = P->geom.m, n = P->geom.n;
    const size_t mn = (size_t)m * n;
    hipLaunchKernelGGL(k_residual, dim3(reduce_blocks(mn)), dim3(TPB), 0, s, m, n, P->top,
                       P->bot, P->geom.v0, P->geom.device_model == MCA_DEVICE_LINEAR ? 1 : 0,
                       g_dev, v_in, vt, vb, ft, fb, d, partials);
    return hipGetLastError();
}

hipError_t launch_reduce(const double *partials, int nblocks, int ncomp, double *out,
                         hipStream_t s, int *mark, int epoch)
{
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(TPB), 0, s, partials, nblocks, ncomp, out, mark,
                       epoch);
    return hipGetLastError();
}

hipError_t launch_jacobian(const mca_plan *P, const double *d, const double *xt,
                           const double *xb, double *yt, double *yb, hipStream_t s,
                           const double *v0, double *partials, const int *skip)
{
    const int m = P->geom.m, n = P->geom.n;
    const size_t mn = (size_t)m * n;
    // with a projection the grid matches the Krylov reductions of length 2mn
    const int blocks = v0 ? reduce_blocks(2 * mn) : elementwise_blocks(mn);
    hipLaunchKernelGGL(k_jacobian, dim3(blocks), dim3(TPB), 0, s, m, n, P->top, P->bot, d, xt,
                       xb, yt, yb, v0, v0 ? partials : nullptr, skip);
    return hipGetLastError();
}

hipError_t launch_precond_pre(const mca_plan *P, double a1, double a2, const double *rt,
                              const double *rb, double *w, hipStream_t s, const int *skip)
{
    const int m = P->geom.m, n = P->geom.n;
    hipLaunchKernelGGL(k_precond_pre, dim3(elementwise_blocks((size_t)m * n)), dim3(TPB), 0, s,
                       m, n, P->bot, 1.0 / a1, a2, rt, rb, w, skip);
    return hipGetLastError();
}

hipError_t launch_finish_fold(const GsStep &g, const mca_plan *P, double a1, double a2,
                              const double *rt, const double *rb, double *f, hipStream_t s,
                              const int *skip, const double *shift)
{
    const int nv = g.j + 1;
    if (g.j < 0 || nv > kGsMaxV || g.j + 1 >= g.ldl || g.j + 1 >= g.ldh) return hipErrorInvalidValue;
    FoldArgs a{};
    a.m = P->geom.m;
    a.n = P->geom.n;
    a.bot = P->bot;
    a.inv_a1 = shift ? 0.0 : 1.0 / a1;
    a.a2 = a2;
    a.shift = shift;
    a.rt = rt;
    a.rb = rb;
    a.f = f;
    a.skip = skip;
    const size_t hn = (size_t)(a.m / 2) * a.n;
    const int fold = (int)std::max<size_t>(1, std::min<size_t>((hn + 1023) / 1024, 512));
    hipLaunchKernelGGL(k_finish_fold, dim3(fold + 1), dim3(1024), 0, s, g, a);
    return hipGetLastError();
}

hipError_t launch_precond_pre_fold(const mca_plan *P, double a1, double a2, const double *rt,
                                   const double *rb, double *f, hipStream_t s, const int *skip)
{
    const int m = P->geom.m, n = P->geom.n;
    hipLaunchKernelGGL(k_precond_pre_fold, dim3(elementwise_blocks((size_t)(m / 2) * n)), dim3(TPB),
                       0, s, m, n, P->bot, 1.0 / a1, a2, rt, rb, f, skip, (const double *)nullptr);
    return hipGetLastError();
}

hipError_t launch_precond_pre_fold_dev(const mca_plan *P, const double *shift, const double *rt,
                                       const double *rb, double *f, hipStream_t s, const int *skip)
{
    const int m = P->geom.m, n = P->geom.n;
    hipLaunchKernelGGL(k_precond_pre_fold, dim3(elementwise_blocks((size_t)(m / 2) * n)), dim3(TPB),
                       0, s, m, n, P->bot, 0.0, 0.0, rt, rb, f, skip, shift);
    return hipGetLastError();
}

hipError_t launch_unfold(const double *ys, const double *ya, int n, int h, double *xt,
                         hipStream_t s, const int *skip)
{
    hipLaunchKernelGGL(k_unfold, dim3(elementwise_blocks((size_t)n * h)), dim3(TPB), 0, s, ys, ya,
                       n, h, xt, skip);
    return hipGetLastError();
}

hipError_t launch_precond_post(const mca_plan *P, double a1, const double *zt,
                               const double *rt, double *zb, hipStream_t s, const int *skip)
{
    const int m = P->geom.m, n = P->geom.n;
    hipLaunchKernelGGL(k_precond_post, dim3(elementwise_blocks((size_t)m * n)), dim3(TPB), 0, s,
                       m, n, P->top, a1, 1.0 / a1, zt, rt, zb, skip);
    return hipGetLastError();
}

hipError_t launch_dot_partials(const double *x, const double *y, size_t len, double *partials,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_partials, dim3(reduce_blocks(len)), dim3(TPB), 0, s, x, y, len,
                       partials);
    return hipGetLastError();
}

hipError_t launch_mgs_step(double *w, const double *v_prev, const double *v_next, size_t len,
                           const double *partials_in, double *partials_out, double *h_out,
                           hipStream_t s, const int *skip)
{
    const int nb = reduce_blocks(len);
    hipLaunchKernelGGL(k_mgs_step, dim3(nb), dim3(TPB), 0, s, w, v_prev, v_next, len / 2,
                       partials_in, nb, partials_out, h_out, skip);
    return hipGetLastError();
}

hipError_t launch_normalize(double *w, size_t len, const double *partials_in, double *h_out,
                            hipStream_t s, const int *skip)
{
    const int nb = reduce_blocks(len);
    hipLaunchKernelGGL(k_normalize, dim3(nb), dim3(TPB), 0, s, w, len / 2, partials_in, nb,
                       h_out, skip);
    return hipGetLastError();
}

hipError_t launch_gs_step(const GsStep &g, int pass, hipStream_t s)
{
    const int nv = g.j + 1;
    if (g.j < 0 || nv > kGsMaxV || g.j + 1 >= g.ldl || g.j + 1 >= g.ldh) return hipErrorInvalidValue;
    const bool fused = nv <= kGsFusedMaxV;
    const dim3 grid(kGsBlocks), b(TPB);
    if (pass == 0) {
        // short bases: kProjBlocks blocks of 1024 threads, whose partials every
        // update block sums; longer ones: kGsBlocks blocks of TPB threads
        const dim3 pg(kProjBlocks), pb(1024);
        if (g.post_rt) {
            if (nv <= 4) hipLaunchKernelGGL((k_jacobian_proj<4, 1024, true>), pg, pb, 0, s, g);
            else if (nv <= 8) hipLaunchKernelGGL((k_jacobian_proj<8, 1024, true>), pg, pb, 0, s, g);
            else if (nv <= 16) hipLaunchKernelGGL((k_jacobian_proj<16, TPB, true>), grid, b, 0, s, g);
            else hipLaunchKernelGGL((k_jacobian_proj<32, TPB, true>), grid, b, 0, s, g);
        } else {
            if (nv <= 4) hipLaunchKernelGGL((k_jacobian_proj<4, 1024, false>), pg, pb, 0, s, g);
            else if (nv <= 8) hipLaunchKernelGGL((k_jacobian_proj<8, 1024, false>), pg, pb, 0, s, g);
            else if (nv <= 16) hipLaunchKernelGGL((k_jacobian_proj<16, TPB, false>), grid, b, 0, s, g);
            else hipLaunchKernelGGL((k_jacobian_proj<32, TPB, false>), grid, b, 0, s, g);
        }
    } else if (pass == 1) {
        static_assert(kGsFusedMaxV == 8, "variants below");
        // short bases: kProjBlocks blocks of 1024 threads (each forms h itself)
        const dim3 pg(kProjBlocks), pb(1024);
        if (!fused) hipLaunchKernelGGL(k_gs_coef, dim3(1), dim3(1024), 0, s, g);
        if (nv <= 4) hipLaunchKernelGGL((k_gs_update<4, true, 1024>), pg, pb, 0, s, g);
        else if (nv <= 8) hipLaunchKernelGGL((k_gs_update<8, true, 1024>), pg, pb, 0, s, g);
        else if (nv <= 16) hipLaunchKernelGGL((k_gs_update<16, false, TPB>), grid, b, 0, s, g);
        else hipLaunchKernelGGL((k_gs_update<32, false, TPB>), grid, b, 0, s, g);
    } else {
        hipLaunchKernelGGL(k_gs_finish, dim3(1), dim3(1024), 0, s, g);
    }
    return hipGetLastError();
}

// The Newton scalars of a residual and the start of the first GMRES cycle
// on them (one thread; see launch_newton_next).
__global__ void k_newton_next(const double *__restrict__ sums, double mn, double gmres_tol,
                              double accept2, double conv2, double *__restrict__ nsc,
                              int *__restrict__ ctl, double *__restrict__ g, int R,
                              double *__restrict__ sig)
{
    for (int i = threadIdx.x + 1; i <= R; i += blockDim.x) g[i] = 0.0;
    if (threadIdx.x != 0) return;
    const double x = sums[0], ds = sums[1];
    const double a = ds / mn, beta = sqrt(x);
    nsc[0] = a;
    nsc[1] = 1.0 / a;
    nsc[2] = beta;
    nsc[3] = -1.0 / beta;
    nsc[4] = gmres_tol * beta;
    const bool ok = isfinite(x) && isfinite(ds) && x <= accept2 && !(x <= conv2);
    g[0] = beta;
    ctl[0] = ok ? 0 : 1;
    ctl[1] = 0;
    ctl[2] = CYCLE_RUNNING;
    ctl[3] = 0;
    if (sig) sig[0] = 1.0;
}

hipError_t launch_newton_next(const double *sums, double mn, double gmres_tol, double accept2,
                              double conv2, double *nsc, int *ctl, double *g, int R, double *sig,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_newton_next, dim3(1), dim3(64), 0, s, sums, mn, gmres_tol, accept2, conv2,
                       nsc, ctl, g, R, sig);
    return hipGetLastError();
}

__global__ __launch_bounds__(TPB) void k_scale_dev(const double *__restrict__ x,
                                                   const double *__restrict__ alpha,
                                                   double *__restrict__ y, size_t len)
{
    const double al = alpha[0];
    for (size_t k = (size_t)blockIdx.x * TPB + threadIdx.x; k < len; k += (size_t)gridDim.x * TPB)
        y[k] = al * x[k];
}

hipError_t launch_scale_dev(const double *x, const double *alpha, double *y, size_t len,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_dev, dim3(elementwise_blocks(len)), dim3(TPB), 0, s, x, alpha, y, len);
    return hipGetLastError();
}

hipError_t launch_cycle_init(int *ctl, double *g, int R, double beta, hipStream_t s,
                             double *sig)
{
    hipLaunchKernelGGL(k_cycle_init, dim3(1), dim3(64), 0, s, ctl, g, R, beta, sig);
    return hipGetLastError();
}

hipError_t launch_givens(double *H, int ldh, int j, double *g, double *cs, double *sn,
                         double abs_tol, int *ctl, double *resid, int *snap, int epoch,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, s, H, ldh, j, g, cs, sn, abs_tol, ctl,
                       resid, snap, epoch);
    return hipGetLastError();
}

hipError_t launch_backsolve(const double *H, int ldh, const double *g, const int *ctl,
                            double *y, hipStream_t s, const double *sig)
{
    hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(64), 0, s, H, ldh, g, ctl, y, sig);
    return hipGetLastError();
}

hipError_t launch_scale(const double *x, double alpha, double *y, size_t len, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale, dim3(elementwise_blocks(len)), dim3(TPB), 0, s, x, alpha, y, len);
    return hipGetLastError();
}

hipError_t launch_update(const double *Z, size_t zstride, const double *coef, int k,
                         const int *kptr, size_t len, double *x, int accumulate, hipStream_t s)
{
    hipLaunchKernelGGL(k_update, dim3(elementwise_blocks(len / 2)), dim3(TPB), 0, s, Z, zstride,
                       coef, k, kptr, len / 2, x, accumulate);
    return hipGetLastError();
}

hipError_t launch_axpby(const double *a, double sc, const double *b, double *out, size_t len,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_axpby, dim3(elementwise_blocks(len)), dim3(TPB), 0, s, a, sc, b, out,
                       len);
    return hipGetLastError();
}

hipError_t launch_neg_sum(const double *a, const double *b, double *out, size_t len,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_neg_sum, dim3(elementwise_blocks(len)), dim3(TPB), 0, s, a, b, out, len);
    return hipGetLastError();
}

hipError_t launch_fill(double *x, double v, size_t len, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3(elementwise_blocks(len)), dim3(TPB), 0, s, x, v, len);
    return hipGetLastError();
}

}  // namespace mca
