// batch.hip -- many crossbars of different sizes solved together (Monte-Carlo
// device variation): every Newton / flexible-GMRES step of every crossbar runs
// in the same kernel launches.
//
// Layout: crossbar b's m*n arrays start at element ox_b = sum_{c<b} m_c n_c of
// the concatenated arrays; its Krylov vectors (top layer then bottom layer,
// 2 m n values) start at 2 ox_b of each batch-wide vector; its drives at
// orow_b = sum_{c<b} m_c.  Streaming kernels run over a block table: block t
// covers crosspoints [c*CH, (c+1)*CH) of crossbar table[t].x (c = table[t].y),
// so per-block partial sums of one crossbar are contiguous and every block of
// that crossbar reduces them in the same fixed order.
//
// Control lives on the device: one state record per crossbar (Newton status,
// tolerances, line-search step, GMRES cycle flags), updated by one-thread-per-
// crossbar kernels; kernels skip crossbars whose flag says so.  The host only
// reads counters (crossbars still active, still in a GMRES cycle, still in the
// line search) to decide how many launches to enqueue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "device_common.h"

namespace mca {
namespace {

using dev::block_sum;
using dev::sinh_cosh;
using dev::TPB;
using dev::wire_apply;

constexpr int CH = 2048;   // crosspoints per block of the streaming kernels

struct BInst {             // device descriptor of one crossbar
    int m, n, linear, blk0, nblk;
    int fold;              // its preconditioner chain is folded (persymmetric rows)
    Wire top, bot;
    double v0, g_src;
    long long ox, orow;
};

struct BState {            // device control record of one crossbar
    double ynorm, fnorm, dsum, a, beta, abs_tol, step, fn_trial, ds_trial;
    int active;            // Newton still iterating
    int status;            // final mca_status
    int newton, krylov, backtracks, restarts;
    int gm_todo;           // in the current Newton step's GMRES solve
    int restart;           // the GMRES cycle ended unconverged: restart
    int first;             // next X update overwrites (first cycle of the step)
    int upd;               // columns of the last cycle to add into X
    int kry_step;          // GMRES iterations in this Newton step
    int ls_todo, accept, halvings;
    int guess;             // started from the caller's guess
    int reject;            // the guess is dropped for V = 0
    int vsel;              // the current voltages sit in T (1) or in Vc (0)
    int pad_;
};
constexpr int kStateInts = sizeof(BState) / sizeof(int);
static_assert(sizeof(BState) % sizeof(double) == 0, "state record");

__device__ __forceinline__ bool on(const int *flag, int b)
{
    return flag == nullptr || flag[(size_t)b * kStateInts] != 0;
}

// crossbar b, crosspoint range of block t; false when the block has nothing to do
__device__ __forceinline__ bool block_range(const BInst *__restrict__ I, const int2 *__restrict__ bt,
                                            const int *flag, int &b, int &k0, int &k1)
{
    const int2 e = bt[blockIdx.x];
    b = e.x;
    const int mn = I[b].m * I[b].n;
    k0 = e.y * CH;
    k1 = min(k0 + CH, mn);
    return on(flag, b);
}

// The same for a launch whose blocks run from the table's end back to its
// start (logical block = last one first); returns the logical block.
__device__ __forceinline__ int block_range_rev(const BInst *__restrict__ I, const int2 *__restrict__ bt,
                                               int &b, int &k0, int &k1)
{
    const int L = gridDim.x - 1 - blockIdx.x;
    const int2 e = bt[L];
    b = e.x;
    const int mn = I[b].m * I[b].n;
    k0 = e.y * CH;
    k1 = min(k0 + CH, mn);
    return L;
}

// Sum of crossbar b's per-block partials (component c of nc), fixed order.
__device__ __forceinline__ double inst_sum(const BInst &I, const double *__restrict__ p, int nc, int c)
{
    double v[1] = {0.0};
    for (int t = threadIdx.x; t < I.nblk; t += TPB) v[0] += p[(size_t)(I.blk0 + t) * nc + c];
    block_sum<1>(v);
    return v[0];
}

// --------------------------------------------------------------- streaming
// (with S given: the voltages of crossbar b are Va, or Vb when S[b].vsel is set)
__global__ __launch_bounds__(TPB) void bk_residual(
    const BInst *__restrict__ I, const int2 *__restrict__ bt, const int *flag,
    const double *__restrict__ g_dev, const double *__restrict__ v_in,
    const double *__restrict__ Va, const double *__restrict__ Vb, const BState *__restrict__ S,
    double *__restrict__ F, double *__restrict__ D, double *__restrict__ part)
{
    int b, k0, k1;
    if (!block_range(I, bt, flag, b, k0, k1)) return;
    const BInst in = I[b];
    const int m = in.m, n = in.n;
    const size_t mn = (size_t)m * n;
    const double *V = (S && S[b].vsel) ? Vb : Va;
    const double *vt = V + 2 * in.ox, *vb = vt + mn;
    double *ft = F + 2 * in.ox, *fb = ft + mn;
    double acc[2] = {0.0, 0.0};
    for (int k = k0 + threadIdx.x; k < k1; k += TPB) {
        const int i = k / n, j = k - i * n;
        const double t = vt[k], bv = vb[k];
        double st = (j > 0) ? in.top.g * (t - vt[k - 1]) : in.top.end0 * (t - v_in[in.orow + i]);
        st += (j + 1 < n) ? in.top.g * (t - vt[k + 1]) : in.top.end1 * t;
        const double sb = wire_apply(in.bot, i, bv, (i > 0) ? vb[k - n] : 0.0,
                                     (i + 1 < m) ? vb[k + n] : 0.0);
        const double u = t - bv, g = g_dev[in.ox + k];
        double cur, slope;
        if (in.linear) {
            cur = g * u;
            slope = g;
        } else {
            double sh, ch;
            sinh_cosh(u / in.v0, sh, ch);
            cur = g * in.v0 * sh;
            slope = g * ch;
        }
        const double f1 = st + cur, f2 = sb - cur;
        ft[k] = f1;
        fb[k] = f2;
        D[in.ox + k] = slope;
        acc[0] += f1 * f1 + f2 * f2;
        acc[1] += slope;
    }
    block_sum<2>(acc);
    if (threadIdx.x == 0) {
        part[2 * (size_t)blockIdx.x] = acc[0];
        part[2 * (size_t)blockIdx.x + 1] = acc[1];
    }
}

// J x at crosspoint k of a crossbar (eq. (J)): (top row, bottom row); x in
// FP64 or FP32 (the preconditioned vectors), the arithmetic in FP64
template <typename T>
__device__ __forceinline__ void jac_point(const BInst &in, const T *__restrict__ xt,
                                          const T *__restrict__ xb, double d, int k,
                                          double &y1, double &y2)
{
    const int m = in.m, n = in.n;
    const int i = k / n, j = k - i * n;
    const double t = xt[k], bv = xb[k];
    const double st = wire_apply(in.top, j, t, (j > 0) ? (double)xt[k - 1] : 0.0,
                                 (j + 1 < n) ? (double)xt[k + 1] : 0.0);
    const double sb = wire_apply(in.bot, i, bv, (i > 0) ? (double)xb[k - n] : 0.0,
                                 (i + 1 < m) ? (double)xb[k + n] : 0.0);
    const double c = d * (t - bv);
    y1 = st + c;
    y2 = sb - c;
}

// y = J x per crossbar (x: the FP32 preconditioned vector); with v0,
// per-block partials of <y, v0>.
__global__ __launch_bounds__(TPB) void bk_jacobian(
    const BInst *__restrict__ I, const int2 *__restrict__ bt, const int *__restrict__ ctl,
    const double *__restrict__ D, const float *__restrict__ X, double *__restrict__ Y,
    const double *__restrict__ v0, double *__restrict__ part)
{
    int b, k0, k1;
    if (!block_range(I, bt, nullptr, b, k0, k1)) return;
    if (ctl[4 * b]) return;
    const BInst in = I[b];
    const size_t mn = (size_t)in.m * in.n;
    const float *xt = X + 2 * in.ox, *xb = xt + mn;
    double *yt = Y + 2 * in.ox, *yb = yt + mn;
    const double *d = D + in.ox;
    double acc[1] = {0.0};
    for (int k = k0 + threadIdx.x; k < k1; k += TPB) {
        double y1, y2;
        jac_point(in, xt, xb, d[k], k, y1, y2);
        yt[k] = y1;
        yb[k] = y2;
        acc[0] += y1 * v0[2 * in.ox + k] + y2 * v0[2 * in.ox + mn + k];
    }
    block_sum<1>(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// GMRES restart of the flagged crossbars: r = -(F + J X) into R, with
// per-block partials of ||r||^2.
__global__ __launch_bounds__(TPB) void bk_restart_residual(
    const BInst *__restrict__ I, const int2 *__restrict__ bt, const int *flag,
    const double *__restrict__ D, const double *__restrict__ X, const double *__restrict__ F,
    double *__restrict__ Rv, double *__restrict__ part)
{
    int b, k0, k1;
    if (!block_range(I, bt, flag, b, k0, k1)) return;
    const BInst in = I[b];
    const size_t mn = (size_t)in.m * in.n, base = 2 * in.ox;
    const double *xt = X + base, *xb = xt + mn;
    const double *d = D + in.ox;
    double acc[1] = {0.0};
    for (int k = k0 + threadIdx.x; k < k1; k += TPB) {
        double y1, y2;
        jac_point(in, xt, xb, d[k], k, y1, y2);
        const double r1 = -(F[base + k] + y1), r2 = -(F[base + mn + k] + y2);
        Rv[base + k] = r1;
        Rv[base + mn + k] = r2;
        acc[0] += r1 * r1 + r2 * r2;
    }
    block_sum<1>(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// One MGS step of every running crossbar: h = <w, v_prev> (from pin),
// w -= h v_prev, partial <w, v_next> (or ||w||^2).  H is per crossbar,
// column-major with leading dimension ldh; h goes to H_b[col][row].
__global__ __launch_bounds__(TPB) void bk_mgs_step(
    const BInst *__restrict__ I, const int2 *__restrict__ bt, const int *__restrict__ ctl,
    double *__restrict__ W, const double *__restrict__ Vp, const double *__restrict__ Vn,
    const double *__restrict__ pin, double *__restrict__ pout, double *__restrict__ H, int ldh,
    int hsize, int col, int row)
{
    int b, k0, k1;
    if (!block_range(I, bt, nullptr, b, k0, k1)) return;
    if (ctl[4 * b]) return;
    const BInst in = I[b];
    const size_t mn = (size_t)in.m * in.n, base = 2 * in.ox;
    const double h = inst_sum(in, pin, 1, 0);
    if (k0 == 0 && threadIdx.x == 0) H[(size_t)b * hsize + (size_t)col * ldh + row] = h;
    double acc[1] = {0.0};
    for (int k = k0 + threadIdx.x; k < k1; k += TPB) {
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            const size_t e = base + l * mn + k;
            const double x = W[e] - h * Vp[e];
            W[e] = x;
            acc[0] += x * (Vn ? Vn[e] : x);
        }
    }
    block_sum<1>(acc);
    if (threadIdx.x == 0) pout[blockIdx.x] = acc[0];
}

// Two-pass Gram-Schmidt of Arnoldi step j for every crossbar in its cycle
// (modified Gram-Schmidt in compact WY form, as in mca_solve): the basis is
// unnormalised (slot q holds u_q, v_q = sig_q u_q), the first kernel forms
// w = sig_j J z~_j with the projections on the basis, the second w -= V h
// with the products of the new vector with the basis.  After each pass a
// kernel with one block per crossbar reduces that crossbar's partials and
// does its small dense work.  Partials of crossbar b, value q, its block t:
//   p[(blk0 * NVAL) + q * nblk + t]   (NVAL = kGsMaxV or kGsMaxV + 1).
struct BGs {
    const BInst *I;
    const int2 *bt;
    int *ctl;                   // per crossbar: stop flag first (stride 4)
    const double *D;
    const float *Z;             // slot j of Z: the preconditioned u_j (FP32)
    double *W;                  // slot j + 1 of V
    const double *V;            // slot 0 of V
    const double *v0;           // where u_0 is read: slot 0 of V, or F (sig_0 = -1 / beta)
    size_t len;                 // slot stride
    double *sig;                // per crossbar R + 1 scales
    double *L;                  // per crossbar (R + 1)^2, row-major
    double *H;                  // per crossbar hsize, column-major ld ldh
    int R, ldh, hsize, j;
    double *p1, *p2;
    // with xp[0] set, the update pass also writes the new vector in the
    // preconditioner's operand format (FP32, or bfloat16 hi [+ lo]), the
    // conversion the next step's chain would otherwise make of it; for a
    // crossbar with a folded chain it writes the folded rows into xf instead
    // (row i < m/2: x_i + x_{m-1-i}, row m/2 + i: x_i - x_{m-1-i}), the input
    // of that chain's first product
    void *xp[2];
    void *xf[2];
    int prec;
    double *g, *cs, *sn;        // Givens state, per crossbar
    const BState *S;
    int *run;                   // per crossbar: 1 while its cycle runs
};

template <int MAXV>
__global__ __launch_bounds__(TPB) void bk_jacobian_proj(BGs a)
{
    int b, k0, k1;
    if (!block_range(a.I, a.bt, nullptr, b, k0, k1)) return;
    if (a.ctl[4 * b]) return;
    const BInst in = a.I[b];
    const int j = a.j, nv = j + 1, R1 = a.R + 1;
    const size_t mn = (size_t)in.m * in.n, base = 2 * in.ox;
    const float *zt = a.Z + base, *zb = zt + mn;
    const double *d = a.D + in.ox;
    const double *sg = a.sig + (size_t)b * R1;
    const double sj = sg[j];
    double acc[MAXV];
#pragma unroll
    for (int q = 0; q < MAXV; ++q) acc[q] = 0.0;
    // (w = sig_j J z~_j is not stored: the update pass forms it again, with the
    // same arithmetic, from z~_j and D, which it reads in place of w)
    for (int k = k0 + threadIdx.x; k < k1; k += TPB) {
        double y1, y2;
        jac_point(in, zt, zb, d[k], k, y1, y2);
        y1 *= sj;
        y2 *= sj;
#pragma unroll
        for (int q = 0; q < MAXV; ++q)
            if (q < nv) {
                const double *u = (q == 0) ? a.v0 : a.V + q * a.len;
                acc[q] += y1 * u[base + k] + y2 * u[base + mn + k];
            }
    }
    block_sum<MAXV>(acc);
    const int t = blockIdx.x - in.blk0;
    double *p = a.p1 + (size_t)in.blk0 * kGsMaxV;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < MAXV; ++q)
            if (q < nv) p[(size_t)q * in.nblk + t] = acc[q];
    }
}

// Sum of p[u] over u = lane, lane + 64, ... < n (one wave; the result in
// every lane), with eight loads in flight per lane and a fixed order.
__device__ __forceinline__ double wave_strided_sum(const double *__restrict__ p, int n, int lane)
{
    double x[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int u = lane;
    for (; u + 7 * 64 < n; u += 8 * 64) {
#pragma unroll
        for (int t = 0; t < 8; ++t) x[t] += p[u + t * 64];
    }
    for (int t = 0; u < n; u += 64, ++t) x[t & 7] += p[u];
    return dev::wave_sum(((x[0] + x[1]) + (x[2] + x[3])) + ((x[4] + x[5]) + (x[6] + x[7])));
}

// One block per crossbar: s_q = sig_q <w, u_q> from the crossbar's partials,
// then (I + L) h = s by forward substitution; h to the crossbar's H column j.
__global__ __launch_bounds__(TPB) void bk_gs_coef(BGs a)
{
    const int b = blockIdx.x;
    if (a.ctl[4 * b]) return;
    const BInst in = a.I[b];
    const int j = a.j, nv = j + 1, R1 = a.R + 1;
    const double *p = a.p1 + (size_t)in.blk0 * kGsMaxV;
    const double *sg = a.sig + (size_t)b * R1;
    __shared__ double sv[kGsMaxV];
    __shared__ double Ls[kGsMaxV][kGsMaxV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = wave; q < nv; q += TPB / 64) {
        const double x = wave_strided_sum(p + (size_t)q * in.nblk, in.nblk, lane);
        if (lane == 0) sv[q] = sg[q] * x;
    }
    const double *Lb = a.L + (size_t)b * R1 * R1;
    for (int e = threadIdx.x; e < nv * kGsMaxV; e += TPB) {
        const int r = e / kGsMaxV, k = e - r * kGsMaxV;
        if (k < r) Ls[r][k] = Lb[(size_t)r * R1 + k];
    }
    __syncthreads();
    if (wave != 0) return;
    double *hcol = a.H + (size_t)b * a.hsize + (size_t)j * a.ldh;
    double h = 0.0;     // lane k holds h_k
    for (int r = 0; r <= j; ++r) {
        double x = (lane < r) ? Ls[r][lane] * h : 0.0;
        x = dev::wave_sum(x);
        const double hr = sv[r] - x;
        if (lane == r) h = hr;
        if (lane == 0) hcol[r] = hr;
    }
}

// The blocks run in reverse table order: the projection pass just before read
// the vectors front to back, so the parts it read last are the likeliest still
// in the memory-side cache.
// x in the preconditioner's operand format at element e: FP64 -> FP32 ->
// bfloat16 hi, lo = the rest (as k_split)
__device__ __forceinline__ void put_operand(void *const (&xp)[2], int prec, size_t e, double x)
{
    const float f = (float)x;
    if (prec == MCA_PREC_FP32) {
        static_cast<float *>(xp[0])[e] = f;
    } else {
        const __bf16 hi = (__bf16)f;
        static_cast<__bf16 *>(xp[0])[e] = hi;
        if (prec == MCA_PREC_BF16X3) static_cast<__bf16 *>(xp[1])[e] = (__bf16)(f - (float)hi);
    }
}

template <int MAXV>
__global__ __launch_bounds__(TPB) void bk_gs_update(BGs a)
{
    int b, k0, k1;
    const int L = block_range_rev(a.I, a.bt, b, k0, k1);
    if (a.ctl[4 * b]) return;
    const BInst in = a.I[b];
    const int j = a.j, nv = j + 1, R1 = a.R + 1;
    const size_t mn = (size_t)in.m * in.n, base = 2 * in.ox;
    double *sg = a.sig + (size_t)b * R1;
    double *hcol = a.H + (size_t)b * a.hsize + (size_t)j * a.ldh;
    double c[MAXV], acc[MAXV + 1];
#pragma unroll
    for (int q = 0; q < MAXV; ++q) c[q] = (q < nv) ? hcol[q] * sg[q] : 0.0;
#pragma unroll
    for (int q = 0; q <= MAXV; ++q) acc[q] = 0.0;
    // w = sig_j J z~_j at crosspoint k (both layers), as the projection pass
    // formed it
    const float *zt = a.Z + base, *zb = zt + mn;
    const double *d = a.D + in.ox;
    const double sj = sg[j];
    auto jw = [&](size_t k, double &y1, double &y2) {
        jac_point(in, zt, zb, d[k], (int)k, y1, y2);
        y1 *= sj;
        y2 *= sj;
    };
    // w -= sum_q c_q v_q at element e (w there: x); accumulates <w, v_q> and ||w||^2
    auto update = [&](size_t e, double x) -> double {
        double vq[MAXV];
#pragma unroll
        for (int q = 0; q < MAXV; ++q) {
            vq[q] = (q < nv) ? ((q == 0) ? a.v0 : a.V + q * a.len)[e] : 0.0;
            x -= c[q] * vq[q];
        }
        a.W[e] = x;
#pragma unroll
        for (int q = 0; q < MAXV; ++q) acc[q] += x * vq[q];
        acc[MAXV] += x * x;
        return x;
    };
    if (a.xp[0] && in.fold) {
        // pairs of rows (i, m - 1 - i): this block takes pairs k0/2 .. k1/2 of
        // the m/2 x n half (k0, k1 and m n are even) and writes both folded rows
        const int n = in.n, h = in.m / 2;
        const size_t half = (size_t)h * n;
        for (int q = k0 / 2 + threadIdx.x; q < k1 / 2; q += TPB) {
            const int i = q / n, jj = q - i * n;
            const size_t p0 = (size_t)i * n + jj, p1 = (size_t)(in.m - 1 - i) * n + jj;
            double w0[2], w1[2];
            jw(p0, w0[0], w0[1]);
            jw(p1, w1[0], w1[1]);
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                const size_t o = base + l * mn;
                const double x0 = update(o + p0, w0[l]), x1 = update(o + p1, w1[l]);
                put_operand(a.xf, a.prec, o + q, x0 + x1);
                put_operand(a.xf, a.prec, o + half + q, x0 - x1);
            }
        }
    } else {
        for (int k = k0 + threadIdx.x; k < k1; k += TPB) {
            double w[2];
            jw(k, w[0], w[1]);
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                const size_t e = base + l * mn + k;
                const double x = update(e, w[l]);
                if (a.xp[0]) put_operand(a.xp, a.prec, e, x);
            }
        }
    }
    block_sum<MAXV + 1>(acc);
    const int t = L - in.blk0;
    double *p = a.p2 + (size_t)in.blk0 * (kGsMaxV + 1);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < MAXV; ++q)
            if (q < nv) p[(size_t)q * in.nblk + t] = acc[q];
        p[(size_t)nv * in.nblk + t] = acc[MAXV];
    }
}

__global__ __launch_bounds__(TPB) void bk_normalize(
    const BInst *__restrict__ I, const int2 *__restrict__ bt, const int *__restrict__ ctl,
    double *__restrict__ W, const double *__restrict__ pin, double *__restrict__ H, int ldh,
    int hsize, int col, int row)
{
    int b, k0, k1;
    if (!block_range(I, bt, nullptr, b, k0, k1)) return;
    if (ctl[4 * b]) return;
    const BInst in = I[b];
    const size_t mn = (size_t)in.m * in.n, base = 2 * in.ox;
    const double nrm = sqrt(inst_sum(in, pin, 1, 0));
    if (k0 == 0 && threadIdx.x == 0) H[(size_t)b * hsize + (size_t)col * ldh + row] = nrm;
    if (!(nrm > 0.0)) return;
    const double inv = 1.0 / nrm;
    for (int k = k0 + threadIdx.x; k < k1; k += TPB) {
        W[base + k] *= inv;
        W[base + mn + k] *= inv;
    }
}

// dst = alpha_b * src (+ beta * src2), per crossbar scalars from the state
// record (field offset in doubles), for crossbars whose flag is set.
__global__ __launch_bounds__(TPB) void bk_axpy(
    const BInst *__restrict__ I, const int2 *__restrict__ bt, const int *flag,
    const BState *__restrict__ S, int mode, const double *__restrict__ x,
    const double *__restrict__ y, double *__restrict__ out)
{
    int b, k0, k1;
    if (!block_range(I, bt, flag, b, k0, k1)) return;
    const BInst in = I[b];
    const size_t mn = (size_t)in.m * in.n, base = 2 * in.ox;
    const BState s = S[b];
    for (int k = k0 + threadIdx.x; k < k1; k += TPB) {
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            const size_t e = base + l * mn + k;
            double v;
            switch (mode) {
            case 0: v = -x[e] / s.beta; break;            // v0 = -F / beta
            case 1: v = x[e] + s.step * y[e]; break;       // trial = V + step X
            case 2: v = -(x[e] + y[e]); break;             // r = -(F + J X)
            case 3: v = x[e] / s.beta; break;              // v0 = r / beta
            case 5: v = 0.0; break;                        // start from V = 0
            default: v = x[e]; break;                      // copy
            }
            out[e] = v;
        }
    }
}

// Line-search trial of the flagged crossbars: into the buffer that does not
// hold the current voltages, trial = current + step X.
__global__ __launch_bounds__(TPB) void bk_trial(const BInst *__restrict__ I,
                                                const int2 *__restrict__ bt, const int *flag,
                                                const BState *__restrict__ S,
                                                const double *__restrict__ X,
                                                double *__restrict__ Vc, double *__restrict__ T)
{
    int b, k0, k1;
    if (!block_range(I, bt, flag, b, k0, k1)) return;
    const BInst in = I[b];
    const size_t mn = (size_t)in.m * in.n, base = 2 * in.ox;
    const BState s = S[b];
    const double *cur = s.vsel ? T : Vc;
    double *nxt = s.vsel ? Vc : T;
    for (int k = k0 + threadIdx.x; k < k1; k += TPB) {
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            const size_t e = base + l * mn + k;
            nxt[e] = cur[e] + s.step * X[e];
        }
    }
}

// D copy for accepted crossbars (m n values per crossbar)
__global__ __launch_bounds__(TPB) void bk_copy_cross(
    const BInst *__restrict__ I, const int2 *__restrict__ bt, const int *flag,
    const double *__restrict__ src, double *__restrict__ dst)
{
    int b, k0, k1;
    if (!block_range(I, bt, flag, b, k0, k1)) return;
    const size_t ox = I[b].ox;
    for (int k = k0 + threadIdx.x; k < k1; k += TPB) dst[ox + k] = src[ox + k];
}

// X (+)= sum_{i < upd_b} y_b[i] Z_i for crossbars with upd_b > 0 or first_b set
__global__ __launch_bounds__(TPB) void bk_update(
    const BInst *__restrict__ I, const int2 *__restrict__ bt, const BState *__restrict__ S,
    const float *__restrict__ Z, size_t zstride, const double *__restrict__ Y, int R,
    double *__restrict__ X)
{
    int b, k0, k1;
    if (!block_range(I, bt, nullptr, b, k0, k1)) return;
    const int k = S[b].upd;
    const int overwrite = S[b].first;   // first cycle of a Newton step (k = 0 writes zeros)
    if (k <= 0 && !overwrite) return;
    const BInst in = I[b];
    const size_t mn = (size_t)in.m * in.n, base = 2 * in.ox;
    const double *y = Y + (size_t)b * R;
    for (int kk = k0 + threadIdx.x; kk < k1; kk += TPB) {
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            const size_t e = base + l * mn + kk;
            double s = overwrite ? 0.0 : X[e];
            // four vectors' loads in flight at a time, added in order
            int v = 0;
            for (; v + 4 <= k; v += 4) {
                float z4[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) z4[u] = Z[(size_t)(v + u) * zstride + e];
#pragma unroll
                for (int u = 0; u < 4; ++u) s += y[v + u] * (double)z4[u];
            }
            for (; v < k; ++v) s += y[v] * (double)Z[(size_t)v * zstride + e];
            X[e] = s;
        }
    }
}

// scatter the iterate into the caller's v_t / v_b, or gather a guess from them
// (to the user: the current voltages, Vc or, with vsel set, T)
__global__ __launch_bounds__(TPB) void bk_user_io(const BInst *__restrict__ I,
                                                  const int2 *__restrict__ bt,
                                                  const BState *__restrict__ S, double *Vc,
                                                  const double *T, double *vt, double *vb,
                                                  int to_user)
{
    int b, k0, k1;
    if (!block_range(I, bt, nullptr, b, k0, k1)) return;
    const BInst in = I[b];
    double *V = (to_user && S[b].vsel) ? const_cast<double *>(T) : Vc;
    const size_t mn = (size_t)in.m * in.n;
    const bool zero = to_user && S[b].ynorm == 0.0;
    for (int k = k0 + threadIdx.x; k < k1; k += TPB) {
        if (to_user) {
            vt[in.ox + k] = zero ? 0.0 : V[2 * in.ox + k];
            vb[in.ox + k] = zero ? 0.0 : V[2 * in.ox + mn + k];
        } else {
            V[2 * in.ox + k] = vt[in.ox + k];
            V[2 * in.ox + mn + k] = vb[in.ox + k];
        }
    }
}

// ------------------------------------------------------- per-crossbar sums
// One block per crossbar: sums of its block partials into state fields.
// what: 0 = (fnorm, dsum) from residual partials, 1 = (fn_trial, ds_trial),
//       2 = beta from <r, r> partials.
__global__ __launch_bounds__(TPB) void bk_inst_norms(const BInst *__restrict__ I, int count,
                                                     const int *flag,
                                                     const double *__restrict__ part, int what,
                                                     BState *__restrict__ S)
{
    const int b = blockIdx.x;
    if (b >= count || !on(flag, b)) return;
    const BInst in = I[b];
    if (what == 2) {
        const double s = inst_sum(in, part, 1, 0);
        if (threadIdx.x == 0) S[b].beta = sqrt(s);
        return;
    }
    const double f2 = inst_sum(in, part, 2, 0);
    const double ds = inst_sum(in, part, 2, 1);
    if (threadIdx.x == 0) {
        if (what == 0) {
            S[b].fnorm = sqrt(f2);
            S[b].dsum = ds;
        } else {
            S[b].fn_trial = sqrt(f2);
            S[b].ds_trial = ds;
        }
    }
}

// ||Y_b|| = g_src ||v_in_b||; state initialisation
__global__ __launch_bounds__(TPB) void bk_init(const BInst *__restrict__ I, int count,
                                               const double *__restrict__ v_in,
                                               BState *__restrict__ S)
{
    const int b = blockIdx.x;
    if (b >= count) return;
    const BInst in = I[b];
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < in.m; i += TPB) {
        const double x = v_in[in.orow + i];
        v[0] += x * x;
    }
    block_sum<1>(v);
    if (threadIdx.x == 0) {
        BState s{};
        s.ynorm = in.g_src * sqrt(v[0]);
        if (!isfinite(s.ynorm)) {
            s.status = MCA_ERR_NONFINITE;
        } else if (s.ynorm == 0.0) {
            s.status = MCA_OK;   // no drive: V = 0 solves F = 0 exactly
        } else {
            s.active = 1;
            s.status = MCA_ERR_NOT_CONVERGED;
        }
        S[b] = s;
    }
}

// Newton step k begins: convergence test, history, GMRES set-up.
__global__ void bk_newton_begin(const BInst *__restrict__ I, int count, BState *__restrict__ S,
                                int k, int max_newton, double tol, double gtol,
                                double *__restrict__ rhist, int *__restrict__ counter)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    int act = 0;
    if (b < count) {
        BState &s = S[b];
        if (s.active) {
            const double rel = s.ynorm > 0.0 ? s.fnorm / s.ynorm : 0.0;
            rhist[(size_t)b * (MCA_MAX_NEWTON + 1) + k] = rel;
            if (!isfinite(s.fnorm) || !isfinite(s.dsum)) {
                s.active = 0;
                s.status = MCA_ERR_NONFINITE;
            } else if (s.fnorm <= tol * s.ynorm) {
                s.active = 0;
                s.status = MCA_OK;
            } else if (k >= max_newton) {
                s.active = 0;
                s.status = MCA_ERR_NOT_CONVERGED;
            } else {
                s.a = s.dsum / ((double)I[b].m * I[b].n);
                s.beta = s.fnorm;
                s.abs_tol = gtol * s.fnorm;
                s.gm_todo = 1;
                s.first = 1;
                s.kry_step = 0;
                s.restart = 0;
                s.upd = 0;
            }
        }
        act = s.active;
    }
    // count in a fixed order: one block of up to 1024 threads per launch
    __shared__ int sh[1024];
    sh[threadIdx.x] = act;
    __syncthreads();
    if (threadIdx.x == 0) {
        int c = 0;
        for (int t = 0; t < (int)blockDim.x; ++t) c += sh[t];
        counter[blockIdx.x] = c;
    }
}

// sum of per-block counters (one thread)
// out[0] = sum of c[0..n); with host_out (the device address of pinned host
// memory) also written through to the host.
// Sum of the per-block counters into out[0] and, with host_out, into a pinned
// host flag slot as (1 << 32) | sum in one release store at system scope (the
// host cleared the slot before enqueueing this kernel and spins on it).
// (one wave: each lane sums every 64th value, then the lanes' sums)
__global__ void bk_sum_counters(const int *__restrict__ c, int n, int *__restrict__ out,
                                long long *__restrict__ host_out)
{
    if (blockIdx.x != 0 || threadIdx.x >= 64) return;
    int s = 0;
    for (int i = threadIdx.x; i < n; i += 64) s += c[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x != 0) return;
    out[0] = s;
    if (host_out)
        __hip_atomic_store(host_out, (long long)((1ULL << 32) | (unsigned)s), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_SYSTEM);
}

// GMRES cycle start for crossbars in their Newton step's GMRES solve
// With from_f set, a crossbar's first cycle of a Newton step takes u_0 = F
// unscaled (sig_0 = -1 / beta, so that sig_0 u_0 = -F / beta); otherwise v_0
// is stored normalised.
__global__ void bk_cycle_init(int count, BState *__restrict__ S, int *__restrict__ ctl,
                              double *__restrict__ g, int R, int max_krylov,
                              double *__restrict__ sig, int from_f)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    BState &s = S[b];
    if (sig) sig[(size_t)b * (R + 1)] = (from_f && s.first) ? -1.0 / s.beta : 1.0;
    s.restart = 0;
    const bool run = s.gm_todo && s.kry_step < max_krylov;
    ctl[4 * b + 0] = run ? 0 : 1;
    ctl[4 * b + 1] = 0;
    ctl[4 * b + 2] = CYCLE_RUNNING;
    ctl[4 * b + 3] = run ? (max_krylov - s.kry_step) : 0;   // iterations allowed
    double *gb = g + (size_t)b * (R + 1);
    for (int i = 0; i <= R; ++i) gb[i] = (i == 0) ? s.beta : 0.0;
}

// Givens rotations of Hessenberg column j, per running crossbar.
// Givens update of crossbar b's Hessenberg column j (one thread); returns 1
// while the crossbar's cycle keeps running.
__device__ int batch_givens(int b, const BState *__restrict__ S, double *__restrict__ H, int ldh,
                            int hsize, int j, double *__restrict__ g, double *__restrict__ cs,
                            double *__restrict__ sn, int R, int *__restrict__ ctl)
{
    int *c = ctl + 4 * b;
    if (c[0]) return 0;
    double *h = H + (size_t)b * hsize + (size_t)j * ldh;
    double *gb = g + (size_t)b * (R + 1), *cb = cs + (size_t)b * R, *sb = sn + (size_t)b * R;
    bool bad = false;
    for (int i = 0; i <= j + 1; ++i) bad = bad || !isfinite(h[i]);
    if (bad) {
        c[0] = 1;
        c[2] = CYCLE_NONFINITE;
    } else {
        for (int i = 0; i < j; ++i) {
            const double t = cb[i] * h[i] + sb[i] * h[i + 1];
            h[i + 1] = -sb[i] * h[i] + cb[i] * h[i + 1];
            h[i] = t;
        }
        const double hn = h[j + 1];
        const double r = hypot(h[j], hn);
        if (r == 0.0) {
            c[0] = 1;
            c[2] = CYCLE_BREAKDOWN;
        } else {
            cb[j] = h[j] / r;
            sb[j] = hn / r;
            h[j] = r;
            h[j + 1] = 0.0;
            gb[j + 1] = -sb[j] * gb[j];
            gb[j] = cb[j] * gb[j];
            c[1] = j + 1;
            if (fabs(gb[j + 1]) <= S[b].abs_tol) {
                c[0] = 1;
                c[2] = CYCLE_CONVERGED;
            } else if (j + 1 >= c[3]) {
                c[0] = 1;   // iteration budget of this Newton step spent
            }
        }
    }
    return c[0] ? 0 : 1;
}

__global__ void bk_givens(int count, const BState *__restrict__ S, double *__restrict__ H,
                          int ldh, int hsize, int j, double *__restrict__ g,
                          double *__restrict__ cs, double *__restrict__ sn, int R,
                          int *__restrict__ ctl, int *__restrict__ counter)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int running = (b < count) ? batch_givens(b, S, H, ldh, hsize, j, g, cs, sn, R, ctl) : 0;
    __shared__ int sh[1024];
    sh[threadIdx.x] = running;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int t = 0; t < (int)blockDim.x; ++t) s += sh[t];
        counter[blockIdx.x] = s;
    }
}

// One block per crossbar after the second pass: ||x|| and <x, u_q> from the
// partials give H[j+1][j], sig_{j+1} and row j + 1 of L; then the crossbar's
// Givens update.  run[b] = 1 while its cycle keeps running.
__global__ __launch_bounds__(TPB) void bk_gs_finish(BGs a)
{
    const int b = blockIdx.x;
    if (a.ctl[4 * b]) {
        if (threadIdx.x == 0) a.run[b] = 0;
        return;
    }
    const BInst in = a.I[b];
    const int j = a.j, nv = j + 1, R1 = a.R + 1;
    const double *p = a.p2 + (size_t)in.blk0 * (kGsMaxV + 1);
    double *sg = a.sig + (size_t)b * R1;
    __shared__ double sv[kGsMaxV + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = wave; q <= nv; q += TPB / 64) {
        const double x = wave_strided_sum(p + (size_t)q * in.nblk, in.nblk, lane);
        if (lane == 0) sv[q] = x;
    }
    __syncthreads();
    const double nrm = sqrt(sv[nv]);
    const double inv = (nrm > 0.0) ? 1.0 / nrm : 0.0;
    // row j + 1 of L: <v_{j+1}, v_q> = sig_q <x, u_q> / ||x||
    if (threadIdx.x < nv)
        a.L[(size_t)b * R1 * R1 + (size_t)(j + 1) * R1 + threadIdx.x] =
            sv[threadIdx.x] * sg[threadIdx.x] * inv;
    if (threadIdx.x == 0) {
        sg[j + 1] = inv;
        a.H[(size_t)b * a.hsize + (size_t)j * a.ldh + j + 1] = nrm;
        a.run[b] = batch_givens(b, a.S, a.H, a.ldh, a.hsize, j, a.g, a.cs, a.sn, a.R, a.ctl);
    }
}

// End of a GMRES cycle: least squares, bookkeeping, restart decision.
__global__ void bk_cycle_end(int count, BState *__restrict__ S, const double *__restrict__ H,
                             int ldh, int hsize, const double *__restrict__ g, int R,
                             const int *__restrict__ ctl, double *__restrict__ Y, int max_krylov,
                             int *__restrict__ counter, const double *__restrict__ sig)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    int again = 0;
    if (b < count) {
        BState &s = S[b];
        s.upd = 0;
        if (s.gm_todo) {
            const int *c = ctl + 4 * b;
            const int k = c[1];
            const double *Hb = H + (size_t)b * hsize;
            const double *gb = g + (size_t)b * (R + 1);
            double *y = Y + (size_t)b * R;
            if (k <= kGsMaxV) {
                // back substitution with y in registers (the loops run to the
                // bound so that every index is a constant)
                double yl[kGsMaxV];
#pragma unroll
                for (int i = kGsMaxV - 1; i >= 0; --i) {
                    yl[i] = 0.0;
                    if (i < k) {
                        double t = gb[i];
#pragma unroll
                        for (int cc = i + 1; cc < kGsMaxV; ++cc)
                            if (cc < k) t -= Hb[(size_t)cc * ldh + i] * yl[cc];
                        yl[i] = t / Hb[(size_t)i * ldh + i];
                    }
                }
#pragma unroll
                for (int i = 0; i < kGsMaxV; ++i)
                    if (i < k) y[i] = yl[i];
            } else {
                for (int i = k - 1; i >= 0; --i) {
                    double t = gb[i];
                    for (int cc = i + 1; cc < k; ++cc) t -= Hb[(size_t)cc * ldh + i] * y[cc];
                    y[i] = t / Hb[(size_t)i * ldh + i];
                }
            }
            if (sig)   // an unnormalised basis: the update takes y_i sig_i
                for (int i = 0; i < k; ++i) y[i] *= sig[(size_t)b * (R + 1) + i];
            s.upd = k;
            s.kry_step += k;
            s.krylov += k;
            if (c[2] == CYCLE_NONFINITE) {
                s.gm_todo = 0;
                s.active = 0;
                s.status = MCA_ERR_NONFINITE;
                s.upd = 0;
                s.first = 0;
            } else if (c[2] == CYCLE_CONVERGED || c[2] == CYCLE_BREAKDOWN || k == 0 ||
                       s.kry_step >= max_krylov) {
                s.gm_todo = 0;
            } else {
                s.restart = 1;
                s.restarts += 1;
                again = 1;
            }
        }
    }
    __shared__ int sh[1024];
    sh[threadIdx.x] = again;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += sh[i];
        counter[blockIdx.x] = t;
    }
}

// after the X update of a cycle: later cycles of the Newton step accumulate
__global__ void bk_after_update(int count, BState *__restrict__ S)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    S[b].first = 0;
    S[b].upd = 0;
}

// restart: with beta = ||r|| of the new residual, stop (converged or not
// finite) or keep the restart flag for the scaling v_0 = r / beta
__global__ void bk_restart_check(int count, BState *__restrict__ S)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    BState &s = S[b];
    if (!s.restart) return;
    if (!isfinite(s.beta)) {
        s.gm_todo = 0;
        s.active = 0;
        s.status = MCA_ERR_NONFINITE;
        s.restart = 0;
    } else if (s.beta <= s.abs_tol) {
        s.gm_todo = 0;
        s.restart = 0;
    }
}

// guesses no better than V = 0 (whose residual is ||Y||) are dropped
__global__ void bk_check_guess(int count, BState *__restrict__ S, int fallback)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    BState &s = S[b];
    s.guess = 1;
    s.reject = 0;
    if (fallback && s.active && !(s.fnorm < s.ynorm && isfinite(s.dsum))) {
        s.reject = 1;
        s.guess = 0;
    }
}

__global__ void bk_ls_init(int count, BState *__restrict__ S, int *__restrict__ khist, int k)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    BState &s = S[b];
    s.ls_todo = s.active;
    s.step = 1.0;
    s.halvings = 0;
    s.accept = 0;
    if (s.active) khist[(size_t)b * MCA_MAX_NEWTON + k] = s.kry_step;
}

// damped update: accept when ||F(V + s X)|| <= (1 - 1e-4 s) ||F(V)||
__global__ void bk_ls_check(int count, BState *__restrict__ S, int *__restrict__ counter)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    int todo = 0;
    if (b < count) {
        BState &s = S[b];
        if (s.ls_todo) {
            const bool fin = isfinite(s.fn_trial) && isfinite(s.ds_trial);
            if (fin && s.fn_trial <= (1.0 - 1e-4 * s.step) * s.fnorm) {
                s.ls_todo = 0;
                s.accept = 1;
            } else if (s.halvings >= 30) {
                s.ls_todo = 0;
                s.accept = fin && s.fn_trial < s.fnorm;
            } else {
                s.step *= 0.5;
                s.halvings += 1;
                s.backtracks += 1;
            }
        }
        todo = s.ls_todo;
    }
    __shared__ int sh[1024];
    sh[threadIdx.x] = todo;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += sh[i];
        counter[blockIdx.x] = t;
    }
}

__global__ void bk_ls_finish(int count, BState *__restrict__ S)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    BState &s = S[b];
    if (!s.active) return;
    if (s.accept) {
        s.fnorm = s.fn_trial;
        s.dsum = s.ds_trial;
        s.newton += 1;
        s.vsel ^= 1;   // the trial buffer now holds the current voltages
    } else {
        // no decrease: the rounding floor (accepted below 1e-12 ||Y||) or a failure
        s.active = 0;
        s.status = (s.fnorm <= 1e-12 * s.ynorm) ? MCA_OK : MCA_ERR_NOT_CONVERGED;
    }
}

int cblocks(int count) { return (count + 1023) / 1024; }

}  // namespace

// Arnoldi steps captured as HIP graphs (MCA_FLAG_GRAPH): one executable graph
// per step index j (step j runs j + 1 projection passes), built on first use
// and replayed by later cycles and later solves.  The kernels' pointers
// depend on the workspace address, the precision, the restart length and the
// uploaded batch block, so a change of any of them drops the cache.
// HIP events around the four products of the preconditioner chains
// (MCA_FLAG_TIMING: every chain; MCA_FLAG_TIMING_SAMPLED: every fourth), eager
// launches only, at most kMaxPairs chains per solve.
struct ChainTimer {
    static constexpr int kMaxPairs = 1024;
    bool on = false;
    int stride = 1;
    unsigned chains = 0;
    std::vector<hipEvent_t> ev;   // start, end of each timed chain
    ~ChainTimer()
    {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    // the events for the next chain, or nullptr when it is not timed
    hipError_t next(hipEvent_t (&pair)[2])
    {
        pair[0] = pair[1] = nullptr;
        if (!on || chains++ % stride != 0 || (int)ev.size() >= 2 * kMaxPairs) return hipSuccess;
        for (int i = 0; i < 2; ++i) {
            hipEvent_t e = nullptr;
            const hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            ev.push_back(e);
            pair[i] = e;
        }
        return hipSuccess;
    }
    // after the stream has completed the timed chains
    hipError_t total(double &ms) const
    {
        ms = 0.0;
        for (size_t i = 0; i + 1 < ev.size(); i += 2) {
            float t = 0.f;
            const hipError_t r = hipEventElapsedTime(&t, ev[i], ev[i + 1]);
            if (r != hipSuccess) return r;
            ms += t;
        }
        return hipSuccess;
    }
};

struct StepGraphs {
    void *ws = nullptr;
    const void *dev = nullptr;
    int precision = -1, restart = 0;
    int two_pass = -1;                  // Gram-Schmidt form the steps were captured with
    hipStream_t cap = nullptr;          // private stream that the steps are captured on
    std::vector<hipGraphExec_t> exec;
    void clear()
    {
        for (hipGraphExec_t &e : exec)
            if (e) (void)hipGraphExecDestroy(e);
        exec.clear();
        ws = nullptr;
        dev = nullptr;
    }
    void release()
    {
        clear();
        if (cap) (void)hipStreamDestroy(cap);
        cap = nullptr;
    }
};

}  // namespace mca

// ====================================================================== host
struct mca_batch {
    std::vector<mca_geometry> geoms;
    std::vector<mca_plan *> plans;          // host eigen data per distinct geometry
    std::vector<int> pidx;                  // plan of each crossbar
    std::vector<long long> ox, orow;        // offsets (count + 1 entries)
    std::vector<int2> btab;                 // block table
    std::vector<int2> ftab;                 // (crossbar, chunk) of the folded crossbars' row folds
    std::vector<mca::BInst> inst;
    size_t len = 0;                         // sum 2 m n
    size_t dev_bytes = 0;
    void *dev_buf = nullptr;
    // device pointers (inside dev_buf)
    mca::BInst *d_inst = nullptr;
    int2 *d_btab = nullptr;
    int2 *d_ftab = nullptr;
    mca::LpDesc *d_desc[2][4] = {};         // [fp32 | bf16][step]
    int4 *d_tiles[4] = {};
    int ntiles[4] = {};
    int tile = 64;                          // tile edge of the grouped products
    // state kept between solves: pinned counters read back by the host, and
    // the captured Arnoldi steps (calls on one batch must not overlap)
    mutable int *host = nullptr;
    mutable mca::StepGraphs graphs;
};

namespace mca {
namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct BCarver {
    char *base;
    size_t off = 0;
    explicit BCarver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count)
    {
        off = align256(off);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t size() const { return align256(off); }
};

// device block of a batch: descriptors, tables and the eigenbases of every
// distinct geometry (crossbars that share a geometry share them)
struct BatchLayout {
    BInst *inst;
    int2 *btab;
    int2 *ftab;
    LpDesc *desc[2][4];
    int4 *tiles[4];
    std::vector<float *> q32[4];                  // per plan: QnT, QmT, Qm, Qn
    std::vector<uint16_t *> qh[4], ql[4];
    std::vector<double *> lt, lb;
    size_t bytes;
};

// A crossbar's reduced-precision chain is folded (its Q_m-side products at half
// depth, see the single-crossbar chain) when its G_bot is persymmetric and each
// half is a whole number of the batch's product tiles.
bool plan_fold(const mca_plan *P, int tile) { return P->persym && (P->geom.m / 2) % tile == 0; }

// Tile edge of a batch's grouped products: 128 (four times the operand reuse)
// when every crossbar's sides are at least 256 and the batch still gives 256 or
// more 128-tiles per product; else 64.
int choose_tile(const std::vector<mca_geometry> &geoms)
{
    long t128 = 0;
    for (const mca_geometry &g : geoms) {
        if (g.m < 256 || g.n < 256) return 64;
        t128 += (long)((g.m + 127) / 128) * ((g.n + 127) / 128);
    }
    return t128 >= 256 ? 128 : 64;
}

BatchLayout batch_layout(const mca_batch *B, void *base)
{
    BCarver c(base);
    BatchLayout L;
    const size_t cnt = B->geoms.size();
    L.inst = c.take<BInst>(cnt);
    L.btab = c.take<int2>(B->btab.size());
    L.ftab = c.take<int2>(std::max<size_t>(1, B->ftab.size()));
    for (auto &p : L.desc)
        for (auto &d : p) d = c.take<LpDesc>(cnt);
    for (int s = 0; s < 4; ++s) L.tiles[s] = c.take<int4>(B->ntiles[s]);
    const size_t np = B->plans.size();
    for (int s = 0; s < 4; ++s) {
        L.q32[s].resize(np);
        L.qh[s].resize(np);
        L.ql[s].resize(np);
    }
    L.lt.resize(np);
    L.lb.resize(np);
    for (size_t b = 0; b < np; ++b) {
        const size_t m = B->plans[b]->geom.m, n = B->plans[b]->geom.n;
        const size_t sz[4] = {n * n, m * m, m * m, n * n};   // QnT, QmT, Qm, Qn
        for (int s = 0; s < 4; ++s) {
            L.q32[s][b] = c.take<float>(sz[s]);
            L.qh[s][b] = c.take<uint16_t>(sz[s]);
            L.ql[s][b] = c.take<uint16_t>(sz[s]);
        }
        L.lt[b] = c.take<double>(n);
        L.lb[b] = c.take<double>(m);
    }
    L.bytes = c.size();
    return L;
}

struct BatchWs {
    double *V, *X, *Vc, *T, *F, *Ft, *D, *Dt;
    float *Z;   // the preconditioned vectors: FP32, as the products form them
    double *pa, *pb;
    double *pg1, *pg2, *sig, *Lg;   // two-pass Gram-Schmidt
    int *run;
    double *H, *g, *cs, *sn, *Y;
    int *ctl, *counter;
    BState *S;
    double *rhist;
    int *khist;
    LpPlanes x, u, w;
    size_t bytes;
};

BatchWs batch_ws(const mca_batch *B, const mca_options *o, void *base)
{
    const size_t cnt = B->geoms.size(), len = B->len, R = o->restart;
    const size_t nblk = B->btab.size();
    BCarver c(base);
    BatchWs w;
    w.V = c.take<double>((R + 1) * len);
    w.Z = c.take<float>(R * len);
    w.X = c.take<double>(len);
    w.Vc = c.take<double>(len);
    w.T = c.take<double>(len);
    w.F = c.take<double>(len);
    w.Ft = c.take<double>(len);
    w.D = c.take<double>(len / 2);
    w.Dt = c.take<double>(len / 2);
    w.pa = c.take<double>(2 * nblk);
    w.pb = c.take<double>(2 * nblk);
    w.pg1 = c.take<double>(nblk * kGsMaxV);
    w.pg2 = c.take<double>(nblk * (kGsMaxV + 1));
    w.sig = c.take<double>(cnt * (R + 1));
    w.Lg = c.take<double>(cnt * (R + 1) * (R + 1));
    w.run = c.take<int>(cnt);
    w.H = c.take<double>(cnt * (R + 1) * R);
    w.g = c.take<double>(cnt * (R + 1));
    w.cs = c.take<double>(cnt * R);
    w.sn = c.take<double>(cnt * R);
    w.Y = c.take<double>(cnt * R);
    w.ctl = c.take<int>(4 * cnt);
    w.counter = c.take<int>(cblocks((int)cnt) + 8);
    w.S = c.take<BState>(cnt);
    w.rhist = c.take<double>(cnt * (MCA_MAX_NEWTON + 1));
    w.khist = c.take<int>(cnt * MCA_MAX_NEWTON);
    for (LpPlanes *p : {&w.x, &w.u, &w.w}) {
        if (o->precision == MCA_PREC_FP32) {
            p->p[0] = c.take<float>(len);
            p->p[1] = nullptr;
        } else {
            p->p[0] = c.take<uint16_t>(len);
            p->p[1] = c.take<uint16_t>(len);
        }
    }
    w.bytes = c.size();
    return w;
}

#define MCA_BTRY(expr)                  \
    do {                                \
        hipError_t e_ = (expr);         \
        if (e_ != hipSuccess) {         \
            set_hip_error(#expr, e_);   \
            return MCA_ERR_HIP;         \
        }                               \
    } while (0)

mca_status batch_options_ok(const mca_options *o)
{
    if (!(o->newton_tol >= 0.0) || !(o->gmres_tol > 0.0) || !(o->gmres_tol < 1.0))
        return MCA_ERR_INVALID_ARG;
    if (o->restart < 1 || o->restart > MCA_MAX_RESTART) return MCA_ERR_INVALID_ARG;
    if (o->max_newton < 1 || o->max_newton > MCA_MAX_NEWTON) return MCA_ERR_INVALID_ARG;
    if (o->max_krylov < 1) return MCA_ERR_INVALID_ARG;
    if (o->precond != MCA_PRECOND_PERMODE) return MCA_ERR_INVALID_ARG;
    if (o->precision != MCA_PREC_FP32 && o->precision != MCA_PREC_BF16X3 &&
        o->precision != MCA_PREC_BF16)
        return MCA_ERR_INVALID_ARG;
    if (o->flags & ~(MCA_FLAG_INITIAL_GUESS | MCA_FLAG_TIMING | MCA_FLAG_GUESS_FALLBACK |
                     MCA_FLAG_SWEEP_START | MCA_FLAG_GRAPH | MCA_FLAG_MGS_PASSES |
                     MCA_FLAG_TIMING_SAMPLED))
        return MCA_ERR_INVALID_ARG;
    if ((o->flags & MCA_FLAG_INITIAL_GUESS) && (o->flags & MCA_FLAG_SWEEP_START))
        return MCA_ERR_INVALID_ARG;
    return MCA_OK;
}

}  // namespace
}  // namespace mca

using namespace mca;

extern "C" {

mca_status mca_batch_create(int32_t count, const mca_geometry *geoms, mca_batch **out)
{
    if (!out || count < 1 || !geoms) return MCA_ERR_INVALID_ARG;
    *out = nullptr;
    mca_batch *B = new (std::nothrow) mca_batch();
    if (!B) return MCA_ERR_INVALID_ARG;
    B->geoms.assign(geoms, geoms + count);
    // one plan per distinct geometry (bitwise equal records share it)
    std::vector<int> first;                  // a crossbar of each distinct geometry
    {
        std::map<std::string, int> seen;
        B->pidx.resize(count);
        for (int b = 0; b < count; ++b) {
            const std::string key(reinterpret_cast<const char *>(&geoms[b]), sizeof(mca_geometry));
            auto it = seen.find(key);
            if (it == seen.end()) {
                it = seen.emplace(key, (int)first.size()).first;
                first.push_back(b);
            }
            B->pidx[b] = it->second;
        }
    }
    const int np = (int)first.size();
    B->plans.assign(np, nullptr);
    // eigen set-up of the two wires of every distinct geometry, spread over host threads
    std::vector<mca_status> st(np, MCA_OK);
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nt; ++t)
        pool.emplace_back([&, t]() {
            for (int u = (int)t; u < np; u += (int)nt)
                st[u] = mca_plan_create(&geoms[first[u]], &B->plans[u]);
        });
    for (auto &th : pool) th.join();
    for (int u = 0; u < np; ++u)
        if (st[u] != MCA_OK) {
            mca_batch_destroy(B);
            return st[u];
        }
    B->ox.assign(count + 1, 0);
    B->orow.assign(count + 1, 0);
    for (int b = 0; b < count; ++b) {
        B->ox[b + 1] = B->ox[b] + (long long)geoms[b].m * geoms[b].n;
        B->orow[b + 1] = B->orow[b] + geoms[b].m;
    }
    B->len = 2 * (size_t)B->ox[count];
    B->inst.resize(count);
    for (int b = 0; b < count; ++b) {
        const mca_plan *P = B->plans[B->pidx[b]];
        BInst &I = B->inst[b];
        I.m = geoms[b].m;
        I.n = geoms[b].n;
        I.linear = geoms[b].device_model == MCA_DEVICE_LINEAR;
        I.top = P->top;
        I.bot = P->bot;
        I.v0 = geoms[b].v0;
        I.g_src = geoms[b].g_src;
        I.ox = B->ox[b];
        I.orow = B->orow[b];
        I.blk0 = (int)B->btab.size();
        const int nb = (int)((((size_t)I.m * I.n) + CH - 1) / CH);
        I.nblk = nb;
        for (int c = 0; c < nb; ++c) B->btab.push_back(int2{b, c});
    }
    // tiles of the four products: steps 1, 2 are n x m, steps 3, 4 are m x n
    B->tile = choose_tile(B->geoms);
    const int T = B->tile;
    for (int s = 0; s < 4; ++s) {
        int t = 0;
        for (int b = 0; b < count; ++b) {
            const int M = (s < 2) ? geoms[b].n : geoms[b].m, N = (s < 2) ? geoms[b].m : geoms[b].n;
            t += ((M + T - 1) / T) * ((N + T - 1) / T);
        }
        B->ntiles[s] = t;
    }
    // the folded crossbars' row folds, in chunks of kFoldChunk (m/2) x n elements
    for (int b = 0; b < count; ++b)
        B->inst[b].fold = plan_fold(B->plans[B->pidx[b]], T) ? 1 : 0;
    for (int b = 0; b < count; ++b)
        if (B->inst[b].fold) {
            const size_t half = (size_t)geoms[b].m / 2 * geoms[b].n;
            for (size_t c = 0; c * kFoldChunk < half; ++c) B->ftab.push_back(int2{b, (int)c});
        }
    B->dev_bytes = batch_layout(B, nullptr).bytes;
    *out = B;
    return MCA_OK;
}

void mca_batch_destroy(mca_batch *B)
{
    if (!B) return;
    for (mca_plan *p : B->plans) mca_plan_destroy(p);
    B->graphs.release();
    if (B->host) (void)hipHostFree(B->host);
    delete B;
}

mca_status mca_batch_offsets(const mca_batch *B, int64_t *cross_offsets, int64_t *row_offsets)
{
    if (!B) return MCA_ERR_INVALID_ARG;
    for (size_t b = 0; b < B->ox.size(); ++b) {
        if (cross_offsets) cross_offsets[b] = B->ox[b];
        if (row_offsets) row_offsets[b] = B->orow[b];
    }
    return MCA_OK;
}

size_t mca_batch_device_bytes(const mca_batch *B) { return B ? B->dev_bytes : 0; }

int32_t mca_batch_product_tile(const mca_batch *B) { return B ? B->tile : 0; }

mca_status mca_batch_upload(mca_batch *B, void *dev_buf, size_t bytes, void *stream)
{
    if (!B || !dev_buf || (reinterpret_cast<uintptr_t>(dev_buf) & 255)) return MCA_ERR_INVALID_ARG;
    if (bytes < B->dev_bytes) return MCA_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t cnt = B->geoms.size();
    B->graphs.clear();
    std::vector<char> img(B->dev_bytes);
    BatchLayout H = batch_layout(B, img.data());   // host image, same offsets
    BatchLayout D = batch_layout(B, dev_buf);      // device addresses
    std::memcpy(H.inst, B->inst.data(), cnt * sizeof(BInst));
    std::memcpy(H.btab, B->btab.data(), B->btab.size() * sizeof(int2));
    if (!B->ftab.empty()) std::memcpy(H.ftab, B->ftab.data(), B->ftab.size() * sizeof(int2));
    // every plan's operand planes, spread over host threads (disjoint parts of the image)
    const size_t np = B->plans.size();
    auto convert = [&](size_t first, size_t stride) {
        std::vector<double> tmp;
        for (size_t u = first; u < np; u += stride) {
            const mca_plan *P = B->plans[u];
            const size_t m = P->geom.m, n = P->geom.n;
            // QnT, QmT, Qm, Qn in FP64 from the host eigenvectors; a folded
            // chain's QmT and Qm are [U_s^T; U_a^T] and [U_s; U_a] (m x m/2) and
            // its eigenvalues of G_bot run symmetric modes first
            const bool fold = plan_fold(P, B->tile);
            const size_t h = m / 2;
            for (int q = 0; q < 4; ++q) {
                const size_t L = (q == 0 || q == 3) ? n : m;
                const std::vector<double> &src = (q == 0 || q == 3) ? P->Qn : P->Qm;
                const bool tr = (q == 0 || q == 1);
                size_t cnt = L * L;
                tmp.resize(L * L);
                if (fold && (q == 1 || q == 2)) {
                    cnt = m * h;
                    for (int part = 0; part < 2; ++part) {
                        const std::vector<double> &U = part ? P->Ua : P->Us;
                        for (size_t i = 0; i < h; ++i)
                            for (size_t k = 0; k < h; ++k)
                                tmp[(part * h + i) * h + k] = (q == 1) ? U[k * h + i] : U[i * h + k];
                    }
                } else {
                    for (size_t i = 0; i < L; ++i)
                        for (size_t j = 0; j < L; ++j) tmp[i * L + j] = tr ? src[j * L + i] : src[i * L + j];
                }
                split_host(tmp.data(), cnt, MCA_PREC_FP32, H.q32[q][u], nullptr);
                split_host(tmp.data(), cnt, MCA_PREC_BF16X3, H.qh[q][u], H.ql[q][u]);
            }
            std::memcpy(H.lt[u], P->lt.data(), n * sizeof(double));
            if (fold) {
                std::memcpy(H.lb[u], P->ls.data(), h * sizeof(double));
                std::memcpy(H.lb[u] + h, P->la.data(), h * sizeof(double));
            } else {
                std::memcpy(H.lb[u], P->lb.data(), m * sizeof(double));
            }
        }
    };
    {
        const size_t nt = std::max<size_t>(1, std::min<size_t>({16, np, std::thread::hardware_concurrency()}));
        std::vector<std::thread> pool;
        size_t started = 0;
        try {
            for (; started + 1 < nt; ++started) pool.emplace_back(convert, started + 1, nt);
        } catch (...) {   // fewer threads than asked: this thread takes the rest
        }
        convert(0, nt);
        for (size_t t = started + 1; t < nt; ++t) convert(t, nt);
        for (auto &th : pool) th.join();
    }
    for (size_t b = 0; b < cnt; ++b) {
        const int u = B->pidx[b];
        const size_t m = B->geoms[b].m, n = B->geoms[b].n;
        // descriptors of the four products
        const int Ms[4] = {(int)n, (int)n, (int)m, (int)m}, Ns[4] = {(int)m, (int)m, (int)n, (int)n};
        const int Ks[4] = {(int)n, (int)m, (int)m, (int)n};
        for (int f = 0; f < 2; ++f)
            for (int st = 0; st < 4; ++st) {
                LpDesc d{};
                d.M = Ms[st];
                d.N = Ns[st];
                d.K = Ks[st];
                d.inst = (int)b;
                if (f == 0) {
                    d.Q[0] = D.q32[st][u];
                    d.Q[1] = nullptr;
                } else {
                    d.Q[0] = D.qh[st][u];
                    d.Q[1] = D.ql[st][u];
                }
                d.off_data = d.off_out = 2 * (size_t)B->ox[b];
                d.mn = m * n;
                d.lam_row = (st < 2) ? D.lt[u] : nullptr;
                d.lam_col = (st < 2) ? D.lb[u] : nullptr;
                if (plan_fold(B->plans[u], B->tile)) {
                    const int h = (int)m / 2;
                    if (st == 0) d.alt = 1;   // reads the folded rows
                    if (st == 1) {            // symmetric / antisymmetric modes from the two halves
                        d.K = h;
                        d.lda = (int)m;
                        d.split = 1;
                    }
                    if (st == 2) {            // rows of both halves, interleaved by 16
                        d.K = h;
                        d.ldb = (int)m;
                        d.split = 2;
                        d.ileave = 1;
                    }
                    if (st == 3) d.unfold = 1;
                }
                // data rows are m*n-offset slices: aligned when 2 ox and mn are multiples of 8
                d.vec = (d.K % 8 == 0) && (d.lda % 8 == 0) && (d.ldb % 8 == 0) &&
                        ((2 * (size_t)B->ox[b]) % 8 == 0) && (d.mn % 8 == 0);
                H.desc[f][st][b] = d;
            }
    }
    for (int st = 0; st < 4; ++st) {
        int t = 0;
        for (size_t b = 0; b < cnt; ++b) {
            const int M = H.desc[0][st][b].M, N = H.desc[0][st][b].N;
            const int T = B->tile;
            for (int i = 0; i < (M + T - 1) / T; ++i)
                for (int j = 0; j < (N + T - 1) / T; ++j) H.tiles[st][t++] = int4{(int)b, i * T, j * T, 0};
        }
    }
    MCA_BTRY(hipMemcpyAsync(dev_buf, img.data(), B->dev_bytes, hipMemcpyHostToDevice, s));
    MCA_BTRY(hipStreamSynchronize(s));
    B->dev_buf = dev_buf;
    B->d_inst = D.inst;
    B->d_btab = D.btab;
    B->d_ftab = D.ftab;
    for (int f = 0; f < 2; ++f)
        for (int st = 0; st < 4; ++st) B->d_desc[f][st] = D.desc[f][st];
    for (int st = 0; st < 4; ++st) B->d_tiles[st] = D.tiles[st];
    return MCA_OK;
}

size_t mca_batch_workspace_bytes(const mca_batch *B, const mca_options *opts)
{
    if (!B) return 0;
    mca_options o;
    if (opts) o = *opts;
    else {
        mca_options_default(&o);
        o.precond = MCA_PRECOND_PERMODE;
        o.precision = MCA_PREC_BF16X3;
    }
    if (batch_options_ok(&o) != MCA_OK) return 0;
    return batch_ws(B, &o, nullptr).bytes;
}

mca_status mca_solve_batched(const mca_batch *B, const double *g_dev, const double *v_in,
                             double *v_t, double *v_b, const mca_options *opts, void *ws,
                             size_t ws_bytes, mca_stats *stats, void *stream)
{
    if (!B || !g_dev || !v_in || !v_t || !v_b) return MCA_ERR_INVALID_ARG;
    const int cnt = (int)B->geoms.size();
    if (stats) std::memset(stats, 0, sizeof(mca_stats) * cnt);
    mca_options o;
    if (opts) o = *opts;
    else {
        mca_options_default(&o);
        o.precond = MCA_PRECOND_PERMODE;
        o.precision = MCA_PREC_BF16X3;
    }
    mca_status st = batch_options_ok(&o);
    if (st != MCA_OK) return st;
    if (!B->dev_buf) return MCA_ERR_WORKSPACE;
    BatchWs w = batch_ws(B, &o, ws);
    if (!ws || ws_bytes < w.bytes) return MCA_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int R = o.restart, ldh = R + 1, hsize = (R + 1) * R;
    const size_t len = B->len;
    const int nblk = (int)B->btab.size();
    const dim3 gridB(nblk), blk(TPB);
    const int cb = cblocks(cnt), ct = std::min(cnt, 1024);
    const int *actf = &w.S[0].active, *lsf = &w.S[0].ls_todo, *rsf = &w.S[0].restart;
    const int *accf = &w.S[0].accept;
    if (!B->host)
        MCA_BTRY(hipHostMalloc((void **)&B->host, 4096 * sizeof(int),
                               hipHostMallocMapped | hipHostMallocCoherent));
    int *host = B->host, *host_dev = nullptr;
    MCA_BTRY(hipHostGetDevicePointer((void **)&host_dev, host, 0));
    const bool graph = (o.flags & MCA_FLAG_GRAPH) != 0;
    ChainTimer ctm;
    ctm.on = !graph && (o.flags & (MCA_FLAG_TIMING | MCA_FLAG_TIMING_SAMPLED)) != 0;
    ctm.stride = (o.flags & MCA_FLAG_TIMING) ? 1 : 4;
    // the Gram-Schmidt form decides which kernels an Arnoldi step holds
    const bool two_pass = !(o.flags & MCA_FLAG_MGS_PASSES) && R <= kGsMaxV;
    StepGraphs &G = B->graphs;
    if (graph) {
        if (G.ws != ws || G.dev != B->dev_buf || G.precision != o.precision || G.restart != R ||
            G.two_pass != (int)two_pass)
            G.clear();
        if (!G.cap) MCA_BTRY(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
        G.ws = ws;
        G.dev = B->dev_buf;
        G.precision = o.precision;
        G.restart = R;
        G.two_pass = (int)two_pass;
        G.exec.resize(R + 1, nullptr);   // [R]: step 0 of a restart cycle (see below)
    }
    // pinned flag slots (64-bit, from int 16 of the host block): slot j for
    // Arnoldi step j, slot kCountSlot for count_now
    long long *flag = reinterpret_cast<long long *>(host + 16);
    long long *flag_dev = reinterpret_cast<long long *>(host_dev + 16);
    constexpr int kCountSlot = 127;

    // read the sum of the per-block counters written by the last control kernel
    auto count_now = [&](int *out) -> mca_status {
        __atomic_store_n(&flag[kCountSlot], 0LL, __ATOMIC_RELAXED);
        hipLaunchKernelGGL(bk_sum_counters, dim3(1), dim3(64), 0, s, w.counter, cb, w.counter + cb,
                           flag_dev + kCountSlot);
        MCA_BTRY(hipGetLastError());
        return wait_flag64(&flag[kCountSlot], s, out);
    };

    GroupedChain gc{};
    const int f = (o.precision == MCA_PREC_FP32) ? 0 : 1;
    for (int q = 0; q < 4; ++q) {
        gc.descs[q] = B->d_desc[f][q];
        gc.tiles[q] = B->d_tiles[q];
        gc.ntiles[q] = B->ntiles[q];
    }
    gc.len = len;
    gc.tile = B->tile;
    gc.fold_tab = B->d_ftab;
    gc.fold_blocks = (int)B->ftab.size();
    gc.x = w.x;
    gc.u = w.u;
    gc.w = w.w;
    gc.a_inst = &w.S[0].a;
    gc.a_stride = (int)(sizeof(BState) / sizeof(double));
    gc.ctl = w.ctl;

    BGs gs{};
    gs.I = B->d_inst;
    gs.bt = B->d_btab;
    gs.ctl = w.ctl;
    gs.D = w.D;
    gs.V = w.V;
    gs.v0 = w.V;
    gs.len = len;
    gs.sig = w.sig;
    gs.L = w.Lg;
    gs.H = w.H;
    gs.R = R;
    gs.ldh = ldh;
    gs.hsize = hsize;
    gs.p1 = w.pg1;
    gs.p2 = w.pg2;
    gs.g = w.g;
    gs.cs = w.cs;
    gs.sn = w.sn;
    gs.S = w.S;
    gs.run = w.run;
    gs.xp[0] = w.x.p[0];
    gs.xp[1] = w.x.p[1];
    gs.xf[0] = w.w.p[0];
    gs.xf[1] = w.w.p[1];
    gs.prec = o.precision;
    // Arnoldi step j of every crossbar still in its cycle: preconditioner,
    // Jacobian product fused with <w, v_0>, the projection passes, the
    // normalisation, the Givens update, and the count of running cycles
    // written to flag slot j
    auto enqueue_step = [&](int j, hipStream_t q) -> hipError_t {
        double *vj = w.V + (size_t)j * len;
        float *zj = w.Z + (size_t)j * len;
        double *wv = w.V + (size_t)(j + 1) * len;
        GroupedChain c = gc;
        c.r = (j == 0) ? gs.v0 : vj;
        c.z = zj;
        {
            const hipError_t e = ctm.next(c.ev);
            if (e != hipSuccess) return e;
        }
        // the previous update pass converted v_j (and folded it for the folded chains)
        c.r_split = (two_pass && j > 0) ? 1 : 0;
        c.r_folded = c.r_split;
        hipError_t e = launch_precond_lowprec_grouped(o.precision, c, q);
        if (e != hipSuccess) return e;
        if (two_pass) {
            BGs a = gs;
            a.Z = zj;
            a.W = wv;
            a.j = j;
            const int nv = j + 1;
            if (nv <= 4) hipLaunchKernelGGL(bk_jacobian_proj<4>, gridB, blk, 0, q, a);
            else if (nv <= 8) hipLaunchKernelGGL(bk_jacobian_proj<8>, gridB, blk, 0, q, a);
            else if (nv <= 16) hipLaunchKernelGGL(bk_jacobian_proj<16>, gridB, blk, 0, q, a);
            else hipLaunchKernelGGL(bk_jacobian_proj<32>, gridB, blk, 0, q, a);
            hipLaunchKernelGGL(bk_gs_coef, dim3(cnt), blk, 0, q, a);
            if (nv <= 4) hipLaunchKernelGGL(bk_gs_update<4>, gridB, blk, 0, q, a);
            else if (nv <= 8) hipLaunchKernelGGL(bk_gs_update<8>, gridB, blk, 0, q, a);
            else if (nv <= 16) hipLaunchKernelGGL(bk_gs_update<16>, gridB, blk, 0, q, a);
            else hipLaunchKernelGGL(bk_gs_update<32>, gridB, blk, 0, q, a);
            hipLaunchKernelGGL(bk_gs_finish, dim3(cnt), blk, 0, q, a);
            hipLaunchKernelGGL(bk_sum_counters, dim3(1), dim3(64), 0, q, w.run, cnt,
                               w.counter + cb + 1, flag_dev + j);
        } else {
            hipLaunchKernelGGL(bk_jacobian, gridB, blk, 0, q, B->d_inst, B->d_btab, w.ctl, w.D, zj,
                               wv, w.V, w.pa);
            double *pin = w.pa, *pout = w.pb;
            for (int i = 0; i <= j; ++i) {
                const double *vn = (i < j) ? w.V + (size_t)(i + 1) * len : nullptr;
                hipLaunchKernelGGL(bk_mgs_step, gridB, blk, 0, q, B->d_inst, B->d_btab, w.ctl, wv,
                                   w.V + (size_t)i * len, vn, pin, pout, w.H, ldh, hsize, j, i);
                std::swap(pin, pout);
            }
            hipLaunchKernelGGL(bk_normalize, gridB, blk, 0, q, B->d_inst, B->d_btab, w.ctl, wv, pin,
                               w.H, ldh, hsize, j, j + 1);
            hipLaunchKernelGGL(bk_givens, dim3(cb), dim3(ct), 0, q, cnt, w.S, w.H, ldh, hsize, j,
                               w.g, w.cs, w.sn, R, w.ctl, w.counter);
            hipLaunchKernelGGL(bk_sum_counters, dim3(1), dim3(64), 0, q, w.counter, cb,
                               w.counter + cb + 1, flag_dev + j);
        }
        return hipGetLastError();
    };

    // initial state and iterate
    hipLaunchKernelGGL(bk_init, dim3(cnt), blk, 0, s, B->d_inst, cnt, v_in, w.S);
    if (o.flags & MCA_FLAG_SWEEP_START) {
        for (int b = 0; b < cnt; ++b) {
            const BInst &in = B->inst[b];
            if (in.m > kSweepMaxLen || in.n > kSweepMaxLen) return MCA_ERR_INVALID_ARG;
        }
        for (int b = 0; b < cnt; ++b) {
            const BInst &in = B->inst[b];
            const size_t mn = (size_t)in.m * in.n;
            double *vt = w.Vc + 2 * in.ox;
            MCA_BTRY(launch_sweep_guess(in.top, in.bot, in.m, in.n, in.g_src, g_dev + in.ox,
                                        v_in + in.orow, vt, vt + mn, s));
        }
    } else if (o.flags & MCA_FLAG_INITIAL_GUESS)
        hipLaunchKernelGGL(bk_user_io, gridB, blk, 0, s, B->d_inst, B->d_btab, w.S, w.Vc, w.T, v_t,
                           v_b, 0);
    else
        MCA_BTRY(launch_fill(w.Vc, 0.0, len, s));
    hipLaunchKernelGGL(bk_residual, gridB, blk, 0, s, B->d_inst, B->d_btab, (const int *)nullptr, g_dev,
                       v_in, w.Vc, (const double *)nullptr, (const BState *)nullptr, w.F, w.D, w.pa);
    hipLaunchKernelGGL(bk_inst_norms, dim3(cnt), blk, 0, s, B->d_inst, cnt, (const int *)nullptr,
                       w.pa, 0, w.S);
    if (o.flags & (MCA_FLAG_INITIAL_GUESS | MCA_FLAG_SWEEP_START)) {
        const int *rjf = &w.S[0].reject;
        hipLaunchKernelGGL(bk_check_guess, dim3(cb), dim3(ct), 0, s, cnt, w.S,
                           (o.flags & MCA_FLAG_GUESS_FALLBACK) ? 1 : 0);
        hipLaunchKernelGGL(bk_axpy, gridB, blk, 0, s, B->d_inst, B->d_btab, rjf, w.S, 5,
                           (const double *)nullptr, (const double *)nullptr, w.Vc);
        hipLaunchKernelGGL(bk_residual, gridB, blk, 0, s, B->d_inst, B->d_btab, rjf, g_dev, v_in,
                           w.Vc, (const double *)nullptr, (const BState *)nullptr, w.F, w.D, w.pa);
        hipLaunchKernelGGL(bk_inst_norms, dim3(cnt), blk, 0, s, B->d_inst, cnt, rjf, w.pa, 0, w.S);
    }
    MCA_BTRY(hipGetLastError());

    for (int k = 0; k <= o.max_newton; ++k) {
        hipLaunchKernelGGL(bk_newton_begin, dim3(cb), dim3(ct), 0, s, B->d_inst, cnt, w.S, k,
                           o.max_newton, o.newton_tol, o.gmres_tol, w.rhist, w.counter);
        int active = 0;
        if ((st = count_now(&active)) != MCA_OK) return st;
        if (active == 0) break;
        // flexible GMRES for every active crossbar: v_0 = -F / beta, or with
        // the two-pass form (eager launches) u_0 = F read in place, sig_0 =
        // -1 / beta; restart cycles keep v_0 = r / beta in slot 0
        const bool v0_from_f = two_pass;
        if (!v0_from_f)
            hipLaunchKernelGGL(bk_axpy, gridB, blk, 0, s, B->d_inst, B->d_btab, actf, w.S, 0, w.F,
                               (const double *)nullptr, w.V);
        for (bool first_cycle = true;; first_cycle = false) {
            gs.v0 = (v0_from_f && first_cycle) ? w.F : w.V;
            hipLaunchKernelGGL(bk_cycle_init, dim3(cb), dim3(ct), 0, s, cnt, w.S, w.ctl, w.g, R,
                               o.max_krylov, two_pass ? w.sig : nullptr, v0_from_f ? 1 : 0);
            for (int j = 0; j < R; ++j) {
                // (every kernel that wrote slot j before has completed: the last
                // wait of the previous cycle came after it in stream order)
                __atomic_store_n(&flag[j], 0LL, __ATOMIC_RELAXED);
                if (graph) {
                    // step 0 reads u_0 from F in a Newton step's first cycle and
                    // from slot 0 of V in its restarts: one graph each
                    hipGraphExec_t &ex = G.exec[(j == 0 && gs.v0 != w.F) ? R : j];
                    if (!ex) {
                        MCA_BTRY(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
                        const hipError_t e1 = enqueue_step(j, G.cap);
                        hipGraph_t gph = nullptr;
                        const hipError_t e2 = hipStreamEndCapture(G.cap, &gph);
                        hipError_t e3 = hipErrorInvalidValue;
                        if (e1 == hipSuccess && e2 == hipSuccess && gph)
                            e3 = hipGraphInstantiate(&ex, gph, nullptr, nullptr, 0);
                        if (gph) (void)hipGraphDestroy(gph);
                        if (e3 != hipSuccess) {
                            ex = nullptr;
                            const hipError_t e = (e1 != hipSuccess) ? e1 : (e2 != hipSuccess) ? e2 : e3;
                            set_hip_error("capture of an Arnoldi step", e);
                            (void)hipGetLastError();
                            return MCA_ERR_HIP;
                        }
                    }
                    MCA_BTRY(hipGraphLaunch(ex, s));
                } else {
                    MCA_BTRY(enqueue_step(j, s));
                }
                if (j > 0) {
                    // step j runs while the host reads step j-1's count of crossbars
                    // still in their cycle
                    int running = 0;
                    if ((st = wait_flag64(&flag[j - 1], s, &running)) != MCA_OK) return st;
                    if (running == 0) break;   // every crossbar's cycle has stopped
                }
            }
            hipLaunchKernelGGL(bk_cycle_end, dim3(cb), dim3(ct), 0, s, cnt, w.S, w.H, ldh, hsize, w.g,
                               R, w.ctl, w.Y, o.max_krylov, w.counter,
                               two_pass ? (const double *)w.sig : nullptr);
            hipLaunchKernelGGL(bk_update, gridB, blk, 0, s, B->d_inst, B->d_btab, w.S, w.Z, len, w.Y,
                               R, w.X);
            hipLaunchKernelGGL(bk_after_update, dim3(cb), dim3(ct), 0, s, cnt, w.S);
            int again = 0;
            if ((st = count_now(&again)) != MCA_OK) return st;
            if (again == 0) break;
            // restart from the true residual r = -F - J X for the crossbars that need it
            hipLaunchKernelGGL(bk_restart_residual, gridB, blk, 0, s, B->d_inst, B->d_btab, rsf,
                               w.D, w.X, w.F, w.V, w.pb);
            hipLaunchKernelGGL(bk_inst_norms, dim3(cnt), blk, 0, s, B->d_inst, cnt, rsf, w.pb, 2,
                               w.S);
            hipLaunchKernelGGL(bk_restart_check, dim3(cb), dim3(ct), 0, s, cnt, w.S);
            hipLaunchKernelGGL(bk_axpy, gridB, blk, 0, s, B->d_inst, B->d_btab, rsf, w.S, 3, w.V,
                               (const double *)nullptr, w.V);
            MCA_BTRY(hipGetLastError());
        }
        // damped update with a per-crossbar line search
        hipLaunchKernelGGL(bk_ls_init, dim3(cb), dim3(ct), 0, s, cnt, w.S, w.khist, k);
        for (int round = 0; round < 32; ++round) {
            hipLaunchKernelGGL(bk_trial, gridB, blk, 0, s, B->d_inst, B->d_btab, lsf, w.S, w.X, w.Vc,
                               w.T);
            hipLaunchKernelGGL(bk_residual, gridB, blk, 0, s, B->d_inst, B->d_btab, lsf, g_dev,
                               v_in, w.T, w.Vc, w.S, w.Ft, w.Dt, w.pa);
            hipLaunchKernelGGL(bk_inst_norms, dim3(cnt), blk, 0, s, B->d_inst, cnt, lsf, w.pa, 1,
                               w.S);
            hipLaunchKernelGGL(bk_ls_check, dim3(cb), dim3(ct), 0, s, cnt, w.S, w.counter);
            int todo = 0;
            if ((st = count_now(&todo)) != MCA_OK) return st;
            if (todo == 0) break;
        }
        // accepted crossbars move to the trial point: their voltages by the
        // buffer flag (bk_ls_finish), F and D by exchanging the arrays (every
        // crossbar still active has accepted; the others no longer read them),
        // or with captured steps, which hold D's address, by copies
        if (graph) {
            hipLaunchKernelGGL(bk_axpy, gridB, blk, 0, s, B->d_inst, B->d_btab, accf, w.S, 4, w.Ft,
                               (const double *)nullptr, w.F);
            hipLaunchKernelGGL(bk_copy_cross, gridB, blk, 0, s, B->d_inst, B->d_btab, accf, w.Dt,
                               w.D);
        } else {
            std::swap(w.F, w.Ft);
            std::swap(w.D, w.Dt);
            gs.D = w.D;
        }
        hipLaunchKernelGGL(bk_ls_finish, dim3(cb), dim3(ct), 0, s, cnt, w.S);
        MCA_BTRY(hipGetLastError());
    }
    hipLaunchKernelGGL(bk_user_io, gridB, blk, 0, s, B->d_inst, B->d_btab, w.S, w.Vc, w.T, v_t, v_b, 1);
    MCA_BTRY(hipGetLastError());
    // per-crossbar results
    std::vector<BState> S(cnt);
    std::vector<double> rh((size_t)cnt * (MCA_MAX_NEWTON + 1));
    std::vector<int> kh((size_t)cnt * MCA_MAX_NEWTON);
    MCA_BTRY(hipMemcpyAsync(S.data(), w.S, cnt * sizeof(BState), hipMemcpyDeviceToHost, s));
    MCA_BTRY(hipMemcpyAsync(rh.data(), w.rhist, rh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    MCA_BTRY(hipMemcpyAsync(kh.data(), w.khist, kh.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    MCA_BTRY(hipStreamSynchronize(s));
    if (stats && ctm.on) {
        double ms = 0.0;
        MCA_BTRY(ctm.total(ms));
        stats[0].kernel_ms[MCA_KCLASS_GEMM] = ms;
        stats[0].kernel_launches[MCA_KCLASS_GEMM] = 4 * (int)(ctm.ev.size() / 2);
    }
    mca_status result = MCA_OK;
    for (int b = 0; b < cnt; ++b) {
        const BState &x = S[b];
        int status = x.status;
        if (x.active) status = MCA_ERR_NOT_CONVERGED;
        if (status != MCA_OK && result == MCA_OK) result = status;
        if (stats) {
            mca_stats &t = stats[b];
            t.newton_iters = x.newton;
            t.krylov_iters = x.krylov;
            t.backtracks = x.backtracks;
            t.restarts = x.restarts;
            t.rel_residual = x.ynorm > 0 ? x.fnorm / x.ynorm : 0.0;
            t.a_last = x.a;
            t.start = x.guess;
            const mca_plan *P = B->plans[B->pidx[b]];
            t.err_bound = x.fnorm / std::min(P->lt[0], P->lb[0]);
            for (int i = 0; i <= std::min(x.newton, MCA_MAX_NEWTON); ++i)
                t.residual_history[i] = rh[(size_t)b * (MCA_MAX_NEWTON + 1) + i];
            for (int i = 0; i < std::min(x.newton, MCA_MAX_NEWTON); ++i)
                t.krylov_history[i] = kh[(size_t)b * MCA_MAX_NEWTON + i];
        }
    }
    return result;
}

}  // extern "C"
