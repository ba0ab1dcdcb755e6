// gemm.hip -- eigenbasis transforms of the preconditioner on FP64 MFMA (gfx950).
//
// The paper evaluates M^{-1} v through Kronecker products of the wire matrices
// and a reshape of v into an m x n matrix (eqs. (2matrix1)-(2matrix4)).  Here
// the wire matrices are diagonalised once (G = Q diag(lambda) Q^T), so every
// Kronecker factor becomes one dense transform on each side of the m x n
// array, e.g. M^{-1} W = Q_m [(Q_m^T W Q_n) ./ mu] Q_n^T.
//
// Every transform is the single product shape  O = L^T R  with
//   L : K x M row-major  (the data array, contracted over its rows),
//   R : K x N row-major  (an eigenbasis matrix, N = its column count),
//   O : M x N row-major.
// A transform along the rows of an m x n array writes its result transposed
// (n x m), and the following transform along the former columns contracts
// over the rows of that transposed array, so both operands are always read
// along contiguous rows and the output is written along contiguous rows.
//
// Tiling: 64 x 64 output tile per 256-thread workgroup, four waves of 32 x 32,
// each wave a 2 x 2 grid of v_mfma_f64_16x16x4 accumulators; K is staged
// through LDS in double-buffered 16-deep slices.  A second batch (the bottom
// layer) may share the same R tile: the per-mode 2x2 solve of the block
// formula (eq. (block)) then runs in the epilogue on both accumulators.
#include "mca_internal.h"

namespace mca {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, PAD = 2;
constexpr int GTPB = 256;

template <int NB, int EPI>
__global__ __launch_bounds__(GTPB) void k_gemm_tn_f64(GemmArgs a)
{
    __shared__ double Ls[2][NB][BK][BM + PAD];
    __shared__ double Rs[2][BK][BN + PAD];

    const int M = a.M, N = a.N, K = a.K;
    const int tiles_n = (N + BN - 1) / BN;
    const int tile = blockIdx.x;
    const int m0 = (tile / tiles_n) * BM, n0 = (tile % tiles_n) * BN;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

    const double *Lb[2] = {a.L0, a.L1};

    // global -> register staging: row kk of the K slice, 4 consecutive columns
    const int lk = tid >> 4, lc = (tid & 15) * 4;
    double lreg[NB][4], rreg[4];

    auto load = [&](int k0) {
        const int gk = k0 + lk;
        const bool krow = gk < K;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const double *src = Lb[b] + (size_t)gk * M;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gm = m0 + lc + e;
                lreg[b][e] = (krow && gm < M) ? src[gm] : 0.0;
            }
        }
        const double *rsrc = a.R + (size_t)gk * N;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int gn = n0 + lc + e;
            rreg[e] = (krow && gn < N) ? rsrc[gn] : 0.0;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) Ls[buf][b][lk][lc + e] = lreg[b][e];
#pragma unroll
        for (int e = 0; e < 4; ++e) Rs[buf][lk][lc + e] = rreg[e];
    };

    d4 acc[NB][2][2];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[b][i][j] = d4{0.0, 0.0, 0.0, 0.0};

    const int nk = (K + BK - 1) / BK;
    load(0);
    stash(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
        for (int k4 = 0; k4 < BK / 4; ++k4) {
            const int kr = k4 * 4 + (lane >> 4);
            double af[NB][2], bf[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
#pragma unroll
                for (int b = 0; b < NB; ++b) af[b][i] = Ls[buf][b][kr][wm + i * 16 + (lane & 15)];
                bf[i] = Rs[buf][kr][wn + i * 16 + (lane & 15)];
            }
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[b][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[b][i], bf[j],
                                                                             acc[b][i][j], 0, 0, 0);
        }
        if (kt + 1 < nk) stash(buf ^ 1);
        __syncthreads();
    }

    // epilogue: accumulator element r of lane l is row l/16 + 4r, column l%16
    // (the f64 16x16x4 layout, checked on gfx950)
    const double inv_a1 = (EPI != EPI_STORE) ? 1.0 / a.a1 : 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + i * 16 + (lane >> 4) + 4 * r;
                const int col = n0 + wn + j * 16 + (lane & 15);
                if (row >= M || col >= N) continue;
                const size_t o = (size_t)row * N + col;
                if constexpr (EPI == EPI_STORE) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) (b == 0 ? a.O0 : a.O1)[o] = acc[b][i][j][r];
                } else if constexpr (EPI == EPI_DIV_MU) {
                    // eigenvalue of M (eq. (M)) for mode (row, col), summed without cancellation
                    const double lb = a.lb[row], lt = a.lt[col];
                    const double mu = lb * lt * inv_a1 + lb + a.a2 * inv_a1 * lt;
                    a.O0[o] = acc[0][i][j][r] / mu;
                } else {
                    // per-mode block solve [[lt + a1, -a1], [-a2, lb + a2]] x = r
                    const double lb = a.lb[row], lt = a.lt[col];
                    const double det = lt * lb + a.a2 * lt + a.a1 * lb;
                    const double rt = acc[0][i][j][r], rb = acc[NB - 1][i][j][r];
                    a.O0[o] = ((lb + a.a2) * rt + a.a1 * rb) / det;
                    a.O1[o] = (a.a2 * rt + (lt + a.a1) * rb) / det;
                }
            }
}

}  // namespace

hipError_t launch_gemm_f64(const GemmArgs &a, int epi, hipStream_t s)
{
    const int tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
    const bool dual = a.L1 != nullptr;
    if (epi == EPI_PERMODE && !dual) return hipErrorInvalidValue;
    if (dual) {
        if (epi == EPI_PERMODE)
            hipLaunchKernelGGL((k_gemm_tn_f64<2, EPI_PERMODE>), dim3(tiles), dim3(GTPB), 0, s, a);
        else if (epi == EPI_STORE)
            hipLaunchKernelGGL((k_gemm_tn_f64<2, EPI_STORE>), dim3(tiles), dim3(GTPB), 0, s, a);
        else
            return hipErrorInvalidValue;
    } else {
        if (epi == EPI_DIV_MU)
            hipLaunchKernelGGL((k_gemm_tn_f64<1, EPI_DIV_MU>), dim3(tiles), dim3(GTPB), 0, s, a);
        else if (epi == EPI_STORE)
            hipLaunchKernelGGL((k_gemm_tn_f64<1, EPI_STORE>), dim3(tiles), dim3(GTPB), 0, s, a);
        else
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mca
