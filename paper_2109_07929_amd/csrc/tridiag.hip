// tridiag.hip -- the paper's approximate preconditioner on the GPU: batched
// tridiagonal solves with the shifted wire matrices, and the point-Jacobi
// baseline.
//
// Approximating the Schur complement M of eq. (M) by Mhat = G2hat (x) G1
// (eq. (Mhat)) is the same as dropping P's -a2 I block: the Schur complement
// of [[G_t + a1 I, -a1 I], [0, G_b + a2 I]] is (G_b + a2 I)(G_t + a1 I)/a1 =
// Mhat exactly.  So the paper's evaluation (eqs. (block), (2matrix4)) equals
// the block back-substitution
//     z_b = (G_b + a2 I)^{-1} r_b                 (G2 = G_bot + a2 I down every column)
//     z_t = (G_t + a1 I)^{-1} (r_t + a1 z_b)      (G1 = G_top + a1 I along every row)
// which never divides a difference by a1.  Every line of one launch has the
// same matrix T, so its factorisation is built once per shift (once per
// Newton step) into tables, and each right-hand side then costs a few FMAs
// per element:
//  * lines of up to kChunkMaxLen elements: Thomas elimination split into
//    16-element chunks, one per thread, held in registers.  A chunk runs the
//    forward elimination and the back substitution as if its neighbours were
//    zero; the true values differ from those by a multiple of the value
//    carried in from the neighbouring chunk (the products of the
//    elimination multipliers across the chunk, tabulated), and the carries
//    themselves are one short recurrence over the chunks of a line, in LDS.
//    One pass over the data: each element is read once and written once.
//  * longer lines: parallel cyclic reduction held in LDS: level l (stride
//    s = 2^l) replaces equation k by itself plus alpha_k * (equation k - s) +
//    gamma_k * (equation k + s), eliminating the couplings to k -+ s; after
//    ceil(log2 len) levels every equation is diagonal.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"

namespace mca {
namespace {

using dev::TPB;

constexpr int kLds = kTridiagMaxLen;        // doubles of one workgroup's lines (PCR)

// diagonal / couplings of (wire + shift I) at level 0
__global__ __launch_bounds__(TPB) void k_pcr_init(Wire w, double shift, double *__restrict__ a,
                                                  double *__restrict__ b, double *__restrict__ c)
{
    const int len = w.len;
    for (int k = blockIdx.x * TPB + threadIdx.x; k < len; k += gridDim.x * TPB) {
        b[k] = ((k > 0) ? w.g : w.end0) + ((k + 1 < len) ? w.g : w.end1) + shift;
        a[k] = (k > 0) ? -w.g : 0.0;
        c[k] = (k + 1 < len) ? -w.g : 0.0;
    }
}

// one PCR level of the matrix (a, b, c) with stride s -> (a2, b2, c2) and the
// level's multipliers
__global__ __launch_bounds__(TPB) void k_pcr_level(int len, int s, const double *__restrict__ a,
                                                   const double *__restrict__ b,
                                                   const double *__restrict__ c,
                                                   double *__restrict__ a2, double *__restrict__ b2,
                                                   double *__restrict__ c2,
                                                   double *__restrict__ alpha,
                                                   double *__restrict__ gamma)
{
    for (int k = blockIdx.x * TPB + threadIdx.x; k < len; k += gridDim.x * TPB) {
        const bool lo = k - s >= 0, hi = k + s < len;
        const double al = lo ? -a[k] / b[k - s] : 0.0;
        const double ga = hi ? -c[k] / b[k + s] : 0.0;
        a2[k] = lo ? al * a[k - s] : 0.0;
        c2[k] = hi ? ga * c[k + s] : 0.0;
        b2[k] = b[k] + (lo ? al * c[k - s] : 0.0) + (hi ? ga * a[k + s] : 0.0);
        alpha[k] = al;
        gamma[k] = ga;
    }
}

__global__ __launch_bounds__(TPB) void k_pcr_final(int len, const double *__restrict__ b,
                                                   double *__restrict__ invb)
{
    for (int k = blockIdx.x * TPB + threadIdx.x; k < len; k += gridDim.x * TPB) invb[k] = 1.0 / b[k];
}

// Workgroup ids are dispatched round-robin over the 8 XCDs; this order gives
// every XCD a contiguous run of ids.
__device__ __forceinline__ int xcd_order(int bid, int nwg)
{
    return (nwg % 8 == 0) ? (bid % 8) * (nwg / 8) + bid / 8 : bid;
}

// Solve T x = in (+ in2_scale * in2) for `lines` lines of length len.
// Element k of line l sits at l * line_stride + k * elem_stride.  A workgroup
// holds lpw consecutive lines in LDS, ordered as in memory: line-major when the
// lines are contiguous (rows), element-major when consecutive lines are
// adjacent in memory (columns), so loads and stores stay coalesced.
struct PcrSolveArgs {
    int len, levels, lines, lpw, rows;
    size_t line_stride, elem_stride;
    const double *alpha, *gamma, *invb;   // levels x len, levels x len, len
    const double *in, *in2;
    double in2_scale;
    double *out;
    const int *skip;
};

// NT threads of EPT elements each (E = len * lpw <= EPT * NT); LDS sized to E
// at launch.  Workgroups are taken in XCD order, so the lpw-line groups that
// share cache lines (adjacent columns) are solved on one XCD (one L2).  Each thread's (k, line) pairs are fixed for the whole solve, and the
// next level's multipliers are loaded while the current level is applied.
template <int EPT, int NT>
__global__ __launch_bounds__(NT) void k_pcr_solve(PcrSolveArgs p)
{
    if (p.skip && *p.skip) return;
    extern __shared__ double d[];
    const int len = p.len, lpw = p.lpw, E = len * lpw;
    const int line0 = xcd_order(blockIdx.x, gridDim.x) * lpw;
    const int kst = p.rows ? 1 : lpw;      // LDS distance between elements k and k + 1
    int kk[EPT];
    bool valid[EPT];
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
        const int e = threadIdx.x + r * NT;
        int k = 0, l = 0;
        if (e < E) {
            if (p.rows) {
                l = e / len;
                k = e - l * len;
            } else {
                k = e / lpw;
                l = e - k * lpw;
            }
        }
        kk[r] = k;
        valid[r] = e < E && line0 + l < p.lines;
        double v = 0.0;
        if (valid[r]) {
            const size_t g = (size_t)(line0 + l) * p.line_stride + (size_t)k * p.elem_stride;
            v = p.in[g];
            if (p.in2) v += p.in2_scale * p.in2[g];
        }
        if (e < E) d[e] = v;
    }
    double al[EPT], ga[EPT];
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
        al[r] = (p.levels > 0) ? p.alpha[kk[r]] : 0.0;
        ga[r] = (p.levels > 0) ? p.gamma[kk[r]] : 0.0;
    }
    __syncthreads();
    int s = 1;
    for (int lev = 0; lev < p.levels; ++lev, s <<= 1) {
        double nd[EPT];
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            const int e = threadIdx.x + r * NT;
            if (e < E) {
                const int k = kk[r];
                double v = d[e];
                if (k - s >= 0) v += al[r] * d[e - s * kst];
                if (k + s < len) v += ga[r] * d[e + s * kst];
                nd[r] = v;
            }
        }
        if (lev + 1 < p.levels) {
            const double *an = p.alpha + (size_t)(lev + 1) * len;
            const double *gn = p.gamma + (size_t)(lev + 1) * len;
#pragma unroll
            for (int r = 0; r < EPT; ++r) {
                al[r] = an[kk[r]];
                ga[r] = gn[kk[r]];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            const int e = threadIdx.x + r * NT;
            if (e < E) d[e] = nd[r];
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
        const int e = threadIdx.x + r * NT;
        if (valid[r]) {
            const int l = p.rows ? e / len : e - kk[r] * lpw;
            p.out[(size_t)(line0 + l) * p.line_stride + (size_t)kk[r] * p.elem_stride] =
                d[e] * p.invb[kk[r]];
        }
    }
}

// ---- chunked Thomas ------------------------------------------------------
// Thomas elimination of T (diagonal b_k, both couplings -g), in terms of the
// inverse pivots q_k = 1 / delta_k (delta_0 = b_0, delta_k = b_k -
// g^2 q_{k-1}):
//   forward    d'_k = d_k + g q_{k-1} d'_{k-1}
//   backward   x_k  = q_k (d'_k + g x_{k+1})            (x_len = 0)
// A chunk s..e run with zero neighbours gives d'loc and xloc; then
//   d'_k = d'loc_k + fpi_k d'_{s-1},  fpi_s = g q_{s-1},  fpi_k = g q_{k-1} fpi_{k-1}
//   x_k  = xloc_k + bsig_k x_{e+1},    bsig_e = g q_e,      bsig_k = g q_k bsig_{k+1}
// so one table, q, serves every line (element (i, c) of chunk c at i P + c,
// so that the 16 chunks one instruction touches are 16 consecutive doubles;
// zero past the line, which ends the back substitution and the carries).
constexpr int kChunkLines = 4;      // lines per wave: lanes = 4 lines x 16 chunks
constexpr int kChunkWavesMax = 8;
static_assert(kChunkMaxLen == 16 * 16 * kChunkWavesMax, "chunked lines: 8 waves of 16 chunks of 16");

// elements per thread (8 measured no faster at 1024: 7.8 / 9.5 us per column
// / row launch against 7.9 / 9.3 us)
int chunk_len(int) { return 16; }

int chunk_cols(int len)   // chunks per line, a whole number of waves' worth
{
    const int K = chunk_len(len), p = (len + K - 1) / K;
    return (p + 15) / 16 * 16;
}

struct ChunkSetupArgs {
    struct One {
        Wire w;
        double shift;
        int len, K, P;
        double *q;
    } w[2];
};

// One workgroup per wire.  delta_k = theta_k / theta_{k-1} with theta the
// leading principal minors, theta_k = b_k theta_{k-1} - g^2 theta_{k-2}
// (theta_0 = b_0, theta_{-1} = 1): a linear recurrence with one FMA per step
// on its dependency chain (the pivot recurrence would put a division there),
// run by one thread and rescaled by a power of two after every 16 steps; the
// stored pairs (theta_k, theta_{k-1}) keep the scale of their step.  Every
// computed theta_k is exact for b_k and g^2 perturbed by a rounding, as with
// the pivot recurrence.  Then all threads write q.
__global__ __launch_bounds__(TPB) void k_chunk_setup(ChunkSetupArgs p)
{
    __shared__ double th[kChunkMaxLen], thp[kChunkMaxLen];
    const ChunkSetupArgs::One &o = p.w[blockIdx.x];
    const Wire w = o.w;
    const int len = o.len, P = o.P;
    const double g2 = w.g * w.g;
    if (threadIdx.x == 0) {
        const double b0 = w.end0 + ((len > 1) ? w.g : w.end1) + o.shift;
        const double bint = 2.0 * w.g + o.shift, blast = w.g + w.end1 + o.shift;
        double t1 = b0, t0 = 1.0;
        th[0] = t1;
        thp[0] = t0;
        auto step = [&](int k, double b) {
            const double x = fma(b, t1, -g2 * t0);
            t0 = t1;
            t1 = x;
            th[k] = t1;
            thp[k] = t0;
        };
        auto rescale = [&]() {
            int e = 0;
            frexp(fmax(fabs(t0), fabs(t1)), &e);
            t0 = ldexp(t0, -e);
            t1 = ldexp(t1, -e);
        };
        int k = 1;
        for (; k + 16 <= len - 1; k += 16) {   // interior k = 1 .. len - 2
#pragma unroll
            for (int i = 0; i < 16; ++i) step(k + i, bint);
            rescale();
        }
        for (; k < len - 1; ++k) step(k, bint);
        if (len > 1) step(len - 1, blast);
    }
    __syncthreads();
    const int K = o.K;
    for (int k = threadIdx.x; k < K * P; k += TPB) o.q[(k % K) * P + k / K] = (k < len) ? thp[k] / th[k] : 0.0;
}

struct ChunkSolveArgs {
    int len, P, lines, vec;
    size_t line_stride, elem_stride;
    double g;
    const double *q;
    const double *in, *in2;
    double in2_scale;
    double *out;
    const int *skip;
};

// W waves of 4 lines x 16 chunks of K: a workgroup holds 4 whole lines of up
// to 16 K W elements.  ROWS: elements of a line are contiguous (16-byte loads and
// stores where vec says the rows allow them); else consecutive lines are
// adjacent in memory and the 4 lines of a chunk read 32 contiguous bytes.
template <int K, int W, bool ROWS>
__global__ __launch_bounds__(64 * W) void k_chunk_solve(ChunkSolveArgs p)
{
    if (p.skip && *p.skip) return;
    constexpr int P = 16 * W;
    // per wave and line: the carry map (x -> A + B x) across the wave's chunks
    __shared__ double totA[2][W][kChunkLines], totB[2][W][kChunkLines];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l = lane & 3, c = wave * 16 + (lane >> 2);
    const int line = xcd_order(blockIdx.x, gridDim.x) * kChunkLines + l;
    const bool lv = line < p.lines;
    const int len = p.len, k0 = c * K;
    const double g = p.g;
    const size_t base = (size_t)(lv ? line : 0) * p.line_stride;
    const bool whole = lv && k0 + K <= len;
    // q of the chunk's elements, and g q of the element before it
    double q[K], gq[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        q[i] = p.q[i * P + c];
        gq[i] = g * q[i];
    }
    const double gqp = (c > 0) ? g * p.q[(K - 1) * P + c - 1] : 0.0;
    // Loads without branches between them (a branch per element made the
    // compiler wait for each load in turn): addresses are clamped into the
    // line, and what lies past it is zeroed afterwards.
    double v[K];
    if (ROWS && whole && p.vec) {
        const double2 *a = reinterpret_cast<const double2 *>(p.in + base + k0);
#pragma unroll
        for (int i = 0; i < K / 2; ++i) {
            const double2 x = a[i];
            v[2 * i] = x.x;
            v[2 * i + 1] = x.y;
        }
        if (p.in2) {
            const double2 *b = reinterpret_cast<const double2 *>(p.in2 + base + k0);
#pragma unroll
            for (int i = 0; i < K / 2; ++i) {
                const double2 y = b[i];
                v[2 * i] += p.in2_scale * y.x;
                v[2 * i + 1] += p.in2_scale * y.y;
            }
        }
    } else {
        size_t gi[K];
#pragma unroll
        for (int i = 0; i < K; ++i) gi[i] = base + (size_t)min(k0 + i, len - 1) * p.elem_stride;
#pragma unroll
        for (int i = 0; i < K; ++i) v[i] = p.in[gi[i]];
        if (p.in2) {
#pragma unroll
            for (int i = 0; i < K; ++i) v[i] += p.in2_scale * p.in2[gi[i]];
        }
        if (!whole) {
#pragma unroll
            for (int i = 0; i < K; ++i) v[i] = (lv && k0 + i < len) ? v[i] : 0.0;
        }
    }
    // The carries: chunk c maps the value carried into it to the value it
    // carries on, x -> A_c + B_c x; the maps of a line are composed by a scan
    // over its chunks (lanes 4 apart within a wave, then over the waves).
    auto carry = [&](double A, double B, bool fwd) -> double {
#pragma unroll
        for (int off = 4; off < 64; off <<= 1) {
            const double Ap = fwd ? __shfl_up(A, off, 64) : __shfl_down(A, off, 64);
            const double Bp = fwd ? __shfl_up(B, off, 64) : __shfl_down(B, off, 64);
            if (fwd ? lane >= off : lane + off < 64) {
                A += B * Ap;
                B *= Bp;
            }
        }
        // the composition over the chunks before this one within the wave
        const double Ae0 = fwd ? __shfl_up(A, 4, 64) : __shfl_down(A, 4, 64);
        const double Be0 = fwd ? __shfl_up(B, 4, 64) : __shfl_down(B, 4, 64);
        const bool first = fwd ? lane < 4 : lane >= 60;
        const double Ae = first ? 0.0 : Ae0, Be = first ? 1.0 : Be0;
        const int d = fwd ? 0 : 1;
        if (fwd ? lane >= 60 : lane < 4) {
            totA[d][wave][l] = A;
            totB[d][wave][l] = B;
        }
        __syncthreads();
        double cw = 0.0;   // carried into this wave's chunks from the other waves
        if (fwd) {
            for (int u = 0; u < wave; ++u) cw = totA[0][u][l] + totB[0][u][l] * cw;
        } else {
            for (int u = W - 1; u > wave; --u) cw = totA[1][u][l] + totB[1][u][l] * cw;
        }
        return Ae + Be * cw;
    };
    // forward elimination inside the chunk, zero carried in; pi = fpi
    double t = v[0], pi = gqp;
#pragma unroll
    for (int i = 1; i < K; ++i) {
        t = fma(gq[i - 1], t, v[i]);
        v[i] = t;
        pi *= gq[i - 1];
    }
    const double cf = carry(t, pi, true);   // d' just before the chunk
    pi = gqp;
    v[0] = fma(pi, cf, v[0]);
#pragma unroll
    for (int i = 1; i < K; ++i) {
        pi *= gq[i - 1];
        v[i] = fma(pi, cf, v[i]);
    }
    // back substitution inside the chunk, zero carried in; sg = bsig
    t = 0.0;
    double sg = 1.0;
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
        t = q[i] * fma(g, t, v[i]);
        v[i] = t;
        sg *= gq[i];
    }
    const double cb = carry(t, sg, false);   // x just after the chunk
    sg = 1.0;
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
        sg *= gq[i];
        v[i] = fma(sg, cb, v[i]);
    }
    if (ROWS && whole && p.vec) {
        double2 *o = reinterpret_cast<double2 *>(p.out + base + k0);
#pragma unroll
        for (int i = 0; i < K / 2; ++i) o[i] = double2{v[2 * i], v[2 * i + 1]};
    } else if (whole) {
#pragma unroll
        for (int i = 0; i < K; ++i) p.out[base + (size_t)(k0 + i) * p.elem_stride] = v[i];
    } else {
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (lv && k0 + i < len) p.out[base + (size_t)(k0 + i) * p.elem_stride] = v[i];
    }
}

// Jacobi: z = r ./ diag(J), diag(J) = wire diagonal + D on each layer
__global__ __launch_bounds__(TPB) void k_jacobi(int m, int n, Wire top, Wire bot,
                                                const double *__restrict__ D,
                                                const double *__restrict__ rt,
                                                const double *__restrict__ rb,
                                                double *__restrict__ zt, double *__restrict__ zb,
                                                const int *skip)
{
    if (skip && *skip) return;
    const size_t mn = (size_t)m * n;
    for (size_t k = (size_t)blockIdx.x * TPB + threadIdx.x; k < mn; k += (size_t)gridDim.x * TPB) {
        const int i = (int)(k / n), j = (int)(k - (size_t)i * n);
        const double dt = ((j > 0) ? top.g : top.end0) + ((j + 1 < n) ? top.g : top.end1);
        const double db = ((i > 0) ? bot.g : bot.end0) + ((i + 1 < m) ? bot.g : bot.end1);
        zt[k] = rt[k] / (dt + D[k]);
        zb[k] = rb[k] / (db + D[k]);
    }
}

// Tridiagonal solves whose diagonal varies along every line: (wire + diag(shunt))
// x = rhs, by PCR with the coefficients (a, b, c) reduced level by level in
// LDS next to the right-hand side (no shared tables: every line differs).
// rhs_k = [k == 0] r0_scale r0[line] + shunt_k rhs1_k (either part optional).
constexpr int kVarMax = 2048;   // elements per workgroup: four LDS arrays of doubles
constexpr int kVarEpt = kVarMax / TPB;

struct LineSolveArgs {
    int len, levels, lines, lpw, rows;
    size_t line_stride, elem_stride;
    Wire w;
    const double *shunt, *r0, *rhs1;
    double r0_scale;
    double *out;
};

__global__ __launch_bounds__(TPB) void k_line_solve(LineSolveArgs p)
{
    __shared__ double sa[kVarMax], sb[kVarMax], sc[kVarMax], sd[kVarMax];
    const int len = p.len, lpw = p.lpw, E = len * lpw;
    const int line0 = xcd_order(blockIdx.x, gridDim.x) * lpw;
    const int kst = p.rows ? 1 : lpw;
    auto coords = [&](int e, int &k, int &l) {
        if (p.rows) {
            l = e / len;
            k = e - l * len;
        } else {
            k = e / lpw;
            l = e - k * lpw;
        }
    };
    for (int e = threadIdx.x; e < E; e += TPB) {
        int k, l;
        coords(e, k, l);
        double a = 0.0, b = 1.0, c = 0.0, d = 0.0;
        if (line0 + l < p.lines) {
            const size_t g = (size_t)(line0 + l) * p.line_stride + (size_t)k * p.elem_stride;
            const double sh = p.shunt[g];
            b = ((k > 0) ? p.w.g : p.w.end0) + ((k + 1 < len) ? p.w.g : p.w.end1) + sh;
            a = (k > 0) ? -p.w.g : 0.0;
            c = (k + 1 < len) ? -p.w.g : 0.0;
            if (k == 0 && p.r0) d = p.r0_scale * p.r0[line0 + l];
            if (p.rhs1) d += sh * p.rhs1[g];
        }
        sa[e] = a;
        sb[e] = b;
        sc[e] = c;
        sd[e] = d;
    }
    __syncthreads();
    int s = 1;
    for (int lev = 0; lev < p.levels; ++lev, s <<= 1) {
        double na[kVarEpt], nb[kVarEpt], nc[kVarEpt], nd[kVarEpt];
#pragma unroll
        for (int r = 0; r < kVarEpt; ++r) {
            const int e = threadIdx.x + r * TPB;
            if (e < E) {
                int k, l;
                coords(e, k, l);
                double a2 = 0.0, c2 = 0.0, b2 = sb[e], d2 = sd[e];
                if (k - s >= 0) {
                    const int q = e - s * kst;
                    const double al = -sa[e] / sb[q];
                    a2 = al * sa[q];
                    b2 += al * sc[q];
                    d2 += al * sd[q];
                }
                if (k + s < len) {
                    const int q = e + s * kst;
                    const double ga = -sc[e] / sb[q];
                    c2 = ga * sc[q];
                    b2 += ga * sa[q];
                    d2 += ga * sd[q];
                }
                na[r] = a2;
                nb[r] = b2;
                nc[r] = c2;
                nd[r] = d2;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kVarEpt; ++r) {
            const int e = threadIdx.x + r * TPB;
            if (e < E) {
                sa[e] = na[r];
                sb[e] = nb[r];
                sc[e] = nc[r];
                sd[e] = nd[r];
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < E; e += TPB) {
        int k, l;
        coords(e, k, l);
        if (line0 + l < p.lines)
            p.out[(size_t)(line0 + l) * p.line_stride + (size_t)k * p.elem_stride] = sd[e] / sb[e];
    }
}

int pcr_levels(int len)
{
    int l = 0;
    while ((1 << l) < len) ++l;
    return l;
}

int grid_for(size_t count) { return (int)std::max<size_t>(1, std::min<size_t>((count + TPB - 1) / TPB, 1024)); }

// lines per workgroup: as many as fit in LDS, but keep >= ~512 workgroups
// lines per workgroup: as many as fit in `cap` elements while keeping about
// 512 workgroups or more (measured best at 1024 x 1024)
int lines_per_wg(int len, int lines, int cap = kLds)
{
    int lpw = 1;
    while (2 * lpw * len <= cap && 2 * lpw <= std::max(1, lines / 512)) lpw *= 2;
    return lpw;
}

hipError_t line_solve(const Wire &w, int lines, int len, bool rows, size_t line_stride,
                      size_t elem_stride, const double *shunt, const double *r0, double r0_scale,
                      const double *rhs1, double *out, hipStream_t s)
{
    if (len < 1 || len > kVarMax || lines < 1) return hipErrorInvalidValue;
    LineSolveArgs p{};
    p.len = len;
    p.levels = pcr_levels(len);
    p.lines = lines;
    p.lpw = lines_per_wg(len, lines, kVarMax);
    p.rows = rows ? 1 : 0;
    p.line_stride = line_stride;
    p.elem_stride = elem_stride;
    p.w = w;
    p.shunt = shunt;
    p.r0 = r0;
    p.rhs1 = rhs1;
    p.r0_scale = r0_scale;
    p.out = out;
    hipLaunchKernelGGL(k_line_solve, dim3((lines + p.lpw - 1) / p.lpw), dim3(TPB), 0, s, p);
    return hipGetLastError();
}

}  // namespace

size_t tridiag_table_doubles(int len)
{
    if (len <= kChunkMaxLen) return (size_t)chunk_len(len) * chunk_cols(len);
    return (size_t)(2 * pcr_levels(len) + 1 + 6) * len;
}

TridiagTables tridiag_carve(double *base, int len, double g)
{
    TridiagTables t{};
    t.len = len;
    t.g = g;
    if (len <= kChunkMaxLen) {
        t.K = chunk_len(len);
        t.P = chunk_cols(len);
        t.q = base;
        return t;
    }
    t.levels = pcr_levels(len);
    t.alpha = base;
    t.gamma = base + (size_t)t.levels * len;
    t.invb = base + (size_t)2 * t.levels * len;
    t.work = t.invb + len;
    return t;
}

hipError_t launch_tridiag_setup(const Wire &w, double shift, const TridiagTables &t, hipStream_t s)
{
    const int len = t.len;
    if (t.P > 0) {
        ChunkSetupArgs a{};
        a.w[0] = ChunkSetupArgs::One{w, shift, len, t.K, t.P, t.q};
        hipLaunchKernelGGL(k_chunk_setup, dim3(1), dim3(TPB), 0, s, a);
        return hipGetLastError();
    }
    const int grid = grid_for(len);
    double *a = t.work, *b = a + len, *c = b + len, *a2 = c + len, *b2 = a2 + len, *c2 = b2 + len;
    hipLaunchKernelGGL(k_pcr_init, dim3(grid), dim3(TPB), 0, s, w, shift, a, b, c);
    for (int lev = 0, st = 1; lev < t.levels; ++lev, st <<= 1) {
        hipLaunchKernelGGL(k_pcr_level, dim3(grid), dim3(TPB), 0, s, len, st, a, b, c, a2, b2, c2,
                           t.alpha + (size_t)lev * len, t.gamma + (size_t)lev * len);
        std::swap(a, a2);
        std::swap(b, b2);
        std::swap(c, c2);
    }
    hipLaunchKernelGGL(k_pcr_final, dim3(grid), dim3(TPB), 0, s, len, b, t.invb);
    return hipGetLastError();
}

hipError_t launch_tridiag_setup2(const Wire &w1, double shift1, const TridiagTables &t1,
                                 const Wire &w2, double shift2, const TridiagTables &t2,
                                 hipStream_t s)
{
    if (t1.P > 0 && t2.P > 0) {   // both chunked: one launch, one workgroup each
        ChunkSetupArgs a{};
        a.w[0] = ChunkSetupArgs::One{w1, shift1, t1.len, t1.K, t1.P, t1.q};
        a.w[1] = ChunkSetupArgs::One{w2, shift2, t2.len, t2.K, t2.P, t2.q};
        hipLaunchKernelGGL(k_chunk_setup, dim3(2), dim3(TPB), 0, s, a);
        return hipGetLastError();
    }
    hipError_t e = launch_tridiag_setup(w1, shift1, t1, s);
    return e == hipSuccess ? launch_tridiag_setup(w2, shift2, t2, s) : e;
}

namespace {

template <int K, int W>
void chunk_launch(const ChunkSolveArgs &p, bool rows, int grid, hipStream_t s)
{
    if (rows)
        hipLaunchKernelGGL((k_chunk_solve<K, W, true>), dim3(grid), dim3(64 * W), 0, s, p);
    else
        hipLaunchKernelGGL((k_chunk_solve<K, W, false>), dim3(grid), dim3(64 * W), 0, s, p);
}

template <int K>
bool chunk_dispatch(const ChunkSolveArgs &p, bool rows, int grid, hipStream_t s)
{
    switch (p.P / 16) {
    case 1: chunk_launch<K, 1>(p, rows, grid, s); return true;
    case 2: chunk_launch<K, 2>(p, rows, grid, s); return true;
    case 3: chunk_launch<K, 3>(p, rows, grid, s); return true;
    case 4: chunk_launch<K, 4>(p, rows, grid, s); return true;
    case 5: chunk_launch<K, 5>(p, rows, grid, s); return true;
    case 6: chunk_launch<K, 6>(p, rows, grid, s); return true;
    case 7: chunk_launch<K, 7>(p, rows, grid, s); return true;
    case 8: chunk_launch<K, 8>(p, rows, grid, s); return true;
    default: return false;
    }
}

}  // namespace

hipError_t launch_tridiag_solve(const TridiagTables &t, int lines, bool rows, size_t line_stride,
                                size_t elem_stride, const double *in, const double *in2,
                                double in2_scale, double *out, const int *skip, hipStream_t s)
{
    if (t.len > kTridiagMaxLen || t.len < 1 || lines < 1) return hipErrorInvalidValue;
    if (t.P > 0) {
        ChunkSolveArgs p{};
        p.len = t.len;
        p.P = t.P;
        p.lines = lines;
        p.line_stride = line_stride;
        p.elem_stride = elem_stride;
        p.q = t.q;
        p.g = t.g;
        p.in = in;
        p.in2 = in2;
        p.in2_scale = in2_scale;
        p.out = out;
        p.skip = skip;
        auto al16 = [](const void *q) { return q == nullptr || (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
        p.vec = rows && elem_stride == 1 && line_stride % 2 == 0 && al16(in) && al16(in2) && al16(out);
        const int grid = (lines + kChunkLines - 1) / kChunkLines;
        if (t.K != 16 || !chunk_dispatch<16>(p, rows, grid, s)) return hipErrorInvalidValue;
        return hipGetLastError();
    }
    PcrSolveArgs p{};
    p.len = t.len;
    p.levels = t.levels;
    p.lines = lines;
    p.lpw = lines_per_wg(t.len, lines);
    p.rows = rows ? 1 : 0;
    p.line_stride = line_stride;
    p.elem_stride = elem_stride;
    p.alpha = t.alpha;
    p.gamma = t.gamma;
    p.invb = t.invb;
    p.in = in;
    p.in2 = in2;
    p.in2_scale = in2_scale;
    p.out = out;
    p.skip = skip;
    const size_t lds = (size_t)t.len * p.lpw * sizeof(double);
    const dim3 grid((lines + p.lpw - 1) / p.lpw);
    // (loading every level's multipliers up front measured slower; so did
    // 32 elements per thread, which spills)
    const int E = t.len * p.lpw;
    if (E <= 8 * TPB)
        hipLaunchKernelGGL((k_pcr_solve<8, TPB>), grid, dim3(TPB), lds, s, p);
    else if (E <= 8 * 512)
        hipLaunchKernelGGL((k_pcr_solve<8, 512>), grid, dim3(512), lds, s, p);
    else
        hipLaunchKernelGGL((k_pcr_solve<8, 1024>), grid, dim3(1024), lds, s, p);
    return hipGetLastError();
}

hipError_t launch_sweep_guess(const Wire &top, const Wire &bot, int m, int n, double g_src,
                              const double *g_dev, const double *v_in, double *vt, double *vb,
                              hipStream_t s)
{
    // rows: (G_top + diag(g_dev[i, :])) V_t[i, :] = Y_t[i, :], Y_t[i, 0] = g_src v_in[i]
    hipError_t e = line_solve(top, m, n, true, (size_t)n, 1, g_dev, v_in, g_src, nullptr, vt, s);
    // columns: (G_bot + diag(g_dev[:, j])) V_b[:, j] = g_dev[:, j] V_t[:, j]
    if (e == hipSuccess)
        e = line_solve(bot, n, m, false, 1, (size_t)n, g_dev, nullptr, 0.0, vt, vb, s);
    return e;
}

hipError_t launch_jacobi(const mca_plan *P, const double *D, const double *rt, const double *rb,
                         double *zt, double *zb, const int *skip, hipStream_t s)
{
    const size_t mn = (size_t)P->geom.m * P->geom.n;
    hipLaunchKernelGGL(k_jacobi, dim3(grid_for(mn)), dim3(TPB), 0, s, P->geom.m, P->geom.n,
                       P->top, P->bot, D, rt, rb, zt, zb, skip);
    return hipGetLastError();
}

}  // namespace mca
