// tridiag.hip -- the paper's approximate preconditioner on the GPU: batched
// tridiagonal solves with the shifted wire matrices, by parallel cyclic
// reduction (PCR), and the point-Jacobi baseline.
//
// Approximating the Schur complement M of eq. (M) by Mhat = G2hat (x) G1
// (eq. (Mhat)) is the same as dropping P's -a2 I block: the Schur complement
// of [[G_t + a1 I, -a1 I], [0, G_b + a2 I]] is (G_b + a2 I)(G_t + a1 I)/a1 =
// Mhat exactly.  So the paper's evaluation (eqs. (block), (2matrix4)) equals
// the block back-substitution
//     z_b = (G_b + a2 I)^{-1} r_b                 (G2 = G_bot + a2 I down every column)
//     z_t = (G_t + a1 I)^{-1} (r_t + a1 z_b)      (G1 = G_top + a1 I along every row)
// which never divides a difference by a1.  Each line solve is PCR held in
// LDS: level l (stride s = 2^l) replaces equation k by itself plus
// alpha_k * (equation k - s) + gamma_k * (equation k + s), eliminating the
// couplings to k -+ s; after ceil(log2 len) levels every equation is
// diagonal.  The multipliers depend only on the matrix, so they are built
// once per shift (once per Newton step) and every right-hand side is then
// log2(len) LDS sweeps of two FMAs per element.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"

namespace mca {
namespace {

using dev::TPB;

constexpr int kLds = kPcrMaxLen;            // doubles of one workgroup's lines

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

size_t pcr_table_doubles(int len)
{
    return (size_t)(2 * pcr_levels(len) + 1 + 6) * len;
}

PcrTables pcr_carve(double *base, int len)
{
    PcrTables t{};
    t.len = len;
    t.levels = pcr_levels(len);
    t.alpha = base;
    t.gamma = base + (size_t)t.levels * len;
    t.invb = base + (size_t)2 * t.levels * len;
    t.work = t.invb + len;
    return t;
}

hipError_t launch_pcr_setup(const Wire &w, double shift, const PcrTables &t, hipStream_t s)
{
    const int len = t.len, grid = grid_for(len);
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

hipError_t launch_pcr_solve(const PcrTables &t, int lines, bool rows, size_t line_stride,
                            size_t elem_stride, const double *in, const double *in2,
                            double in2_scale, double *out, const int *skip, hipStream_t s)
{
    if (t.len > kPcrMaxLen || t.len < 1) return hipErrorInvalidValue;
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
