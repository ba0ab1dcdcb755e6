// device_common.h -- small device helpers shared by the kernel files.
#pragma once

#include "mca_internal.h"

namespace mca {
namespace dev {

constexpr int TPB = 256;   // threads per block of the streaming kernels

// sinh x and cosh x from one expm1 of |x|: with e = expm1(|x|) >= 0 and p = 1 + e,
// sinh |x| = e (2 + e) / (2 p) = (e / 2)(1 + 1/p) and cosh x = (p + 1/p) / 2 (no
// cancellation for small |x|, none in p for large |x|; a few ulps each).
__device__ __forceinline__ void sinh_cosh(double x, double &sh, double &ch)
{
    const double e = expm1(fabs(x)), p = 1.0 + e, r = 1.0 / p;
    sh = copysign(0.5 * e * (1.0 + r), x);
    ch = 0.5 * (p + r);
}

// Product of one wire matrix (eq. (G) with end terminations) with x at node k
// of the wire, in branch-current form:
//   sum over the node's segments of g (x_k - x_neighbour)
//   + end conductance * x_k at the wire's first / last node.
__device__ __forceinline__ double wire_apply(const Wire w, int k, double xk, double xm, double xp)
{
    double s = (k > 0) ? w.g * (xk - xm) : w.end0 * xk;
    s += (k + 1 < w.len) ? w.g * (xk - xp) : w.end1 * xk;
    return s;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over an NT-thread block in a fixed order; the result is valid in every thread.
template <int NC, int NT = TPB>
__device__ __forceinline__ void block_sum(double (&v)[NC])
{
    __shared__ double sh[NC][NT / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double w = wave_sum(v[c]);
        if (lane == 0) sh[c][wave] = w;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s += sh[c][w];
        v[c] = s;
    }
    __syncthreads();
}

// Block sums of the first nc of NC per-thread values, in a fixed order, stored
// by threads 0..nc-1: out[c * stride] = sum over the NT-thread block of v[c].
template <int NC, int NT>
__device__ __forceinline__ void block_store_sums(const double (&v)[NC], int nc, double *out,
                                                 size_t stride)
{
    __shared__ double sh[NC][NT / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double w = wave_sum(v[c]);
        if (lane == 0) sh[c][wave] = w;
    }
    __syncthreads();
    if ((int)threadIdx.x < nc) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += sh[threadIdx.x][w];
        out[threadIdx.x * stride] = s;
    }
}

// Sum of nb per-block partials p[0..nb), identical in every block (fixed order).
__device__ __forceinline__ double sum_partials(const double *__restrict__ p, int nb)
{
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += TPB) v[0] += p[b];
    block_sum<1>(v);
    return v[0];
}


// Workgroups go to the eight XCDs (each with its own L2) in turn: workgroup x
// runs on XCD x mod 8.  For the F workgroups x0 .. x0 + F - 1 of a launch over
// F chunks of a stencil, this gives each XCD's workgroups one contiguous run
// of chunks, so that the rows above and below a chunk, which the stencil also
// reads, are mostly in that XCD's L2.
__device__ __forceinline__ int xcd_run_chunk(int x, int x0, int F)
{
    const int c = x & 7;
    int before = 0;
    for (int cc = 0; cc < c; ++cc) {
        const int f = (cc - x0) & 7;   // first workgroup of XCD cc, counted from x0
        before += (F > f) ? (F - f + 7) / 8 : 0;
    }
    return before + (x - x0 - ((c - x0) & 7)) / 8;
}

}  // namespace dev
}  // namespace mca
