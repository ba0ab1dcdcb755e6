// gemm_lp.hip -- reduced-precision eigenbasis transforms for the mixed-precision
// preconditioner (flexible GMRES absorbs their rounding).
//
// Every transform here has the shape  O = A B^T  with both operands stored
// row-major with K contiguous (A: M x K, B: N x K).  The per-mode
// preconditioner (the block formula of eq. (block) applied per Kronecker
// eigenmode) then becomes four such products without any transpose:
//   U^T   = Q_n^T . X^T      A = Q_n^T,  B = X      (contract over j)
//   W^T   = U^T . Q_m        A = U^T,    B = Q_m^T  (contract over i), + 2x2 solve
//   Y     = Q_m . X^hat      A = Q_m,    B = X^hat^T (contract over p)
//   Z     = Y . Q_n^T        A = Y,      B = Q_n    (contract over q)
// (X is the m x n input, hats mark the eigenbasis.)  Operands are converted
// to FP32 while they are staged into LDS; in the BF16 modes each value is
// also split into hi + lo bfloat16 halves (v = hi + lo to ~16 bits), and the
// product uses hi.hi (BF16) or hi.hi + hi.lo + lo.hi (BF16X3), accumulated in
// FP32 by v_mfma_f32_16x16x32_bf16.  The FP32 mode uses v_mfma_f32_16x16x4f32.
//
// Tiling: 64 x 64 output tile per 256-thread workgroup (four waves of 32 x 32,
// 2 x 2 MFMA tiles each), K staged through LDS in double-buffered 32-deep
// slices.  One operand may have two batches (the two layers) sharing the other.
#include <hip/hip_bf16.h>

#include "mca_internal.h"

namespace mca {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int LBM = 64, LBN = 64, LBK = 32, LTPB = 256;
constexpr int FPITCH = LBK + 4;     // FP32 LDS row pitch (floats): 16 rows hit distinct banks
constexpr int HPITCH = LBK + 8;     // BF16 LDS row pitch (bf16): 16-byte reads stay conflict-free

template <typename T>
__device__ __forceinline__ float to_f32(T v) { return (float)v; }

// Round-to-nearest-even split of an FP32 value into bfloat16 hi + lo.
__device__ __forceinline__ void split_bf16(float v, __bf16 &hi, __bf16 &lo)
{
    hi = (__bf16)v;
    lo = (__bf16)(v - (float)hi);
}

template <int MODE>
struct LdsTile;

template <>
struct LdsTile<MCA_PREC_FP32> {
    float v[LBM][FPITCH];
};

template <int MODE>
struct LdsTile {   // BF16 modes
    __bf16 hi[LBM][HPITCH];
    __bf16 lo[LBM][HPITCH];
};

template <typename T, int NBT>
struct Ptrs {
    const T *p[NBT];
};

// One operand slice (64 rows x 32 k) in registers: thread t holds row t/4,
// k = 8 (t%4) .. +7.
struct Slice {
    float v[8];
};

template <typename T>
__device__ __forceinline__ void load_slice(const T *__restrict__ base, int rows, int K, int r0,
                                           int k0, bool fast, Slice &s)
{
    const int t = threadIdx.x;
    const int r = r0 + (t >> 2), kk = k0 + (t & 3) * 8;
    if (fast) {
        const T *p = base + (size_t)r * K + kk;
#pragma unroll
        for (int e = 0; e < 8; ++e) s.v[e] = to_f32(p[e]);
    } else {
        const int rc = min(r, rows - 1);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = kk + e;
            const float x = to_f32(base[(size_t)rc * K + min(k, K - 1)]);
            s.v[e] = (r < rows && k < K) ? x : 0.0f;
        }
    }
}

template <int MODE>
__device__ __forceinline__ void stash_slice(LdsTile<MODE> &L, const Slice &s)
{
    const int t = threadIdx.x;
    const int r = t >> 2, k = (t & 3) * 8;
    if constexpr (MODE == MCA_PREC_FP32) {
#pragma unroll
        for (int e = 0; e < 8; ++e) L.v[r][k + e] = s.v[e];
    } else {
        bf8 h, l;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            __bf16 a, b;
            split_bf16(s.v[e], a, b);
            h[e] = a;
            l[e] = b;
        }
        *reinterpret_cast<bf8 *>(&L.hi[r][k]) = h;
        if constexpr (MODE == MCA_PREC_BF16X3) *reinterpret_cast<bf8 *>(&L.lo[r][k]) = l;
    }
}

// Arguments: A (M x K) and B (N x K), K contiguous; NB batches of A when
// a_batched, else of B; output O (M x N) row-major, FP32 or FP64.
struct LpArgs {
    int M, N, K;
    const void *A[2];
    const void *B[2];
    void *O[2];
    const double *lam_row, *lam_col;   // PERMODE: eigenvalues along rows (lt) / cols (lb)
    double a1, a2;
    const int *skip;
};

template <int MODE, int NB, bool A_BATCHED, typename TA, typename TB, typename TO, int EPI>
__global__ __launch_bounds__(LTPB) void k_gemm_nt_lp(LpArgs a)
{
    __shared__ LdsTile<MODE> As[2][A_BATCHED ? NB : 1];
    __shared__ LdsTile<MODE> Bs[2][A_BATCHED ? 1 : NB];
    if (a.skip && *a.skip) return;
    constexpr int NA = A_BATCHED ? NB : 1, NBB = A_BATCHED ? 1 : NB;

    const int M = a.M, N = a.N, K = a.K;
    const int tiles_n = (N + LBN - 1) / LBN;
    // XCD-aware order: every XCD owns a contiguous run of tiles
    int t = blockIdx.x;
    const int nwg = gridDim.x;
    if (nwg % 8 == 0) t = (t % 8) * (nwg / 8) + t / 8;
    const int m0 = (t / tiles_n) * LBM, n0 = (t % tiles_n) * LBN;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const bool fast_m = (m0 + LBM <= M) && (K % 8 == 0);
    const bool fast_n = (n0 + LBN <= N) && (K % 8 == 0);

    Slice sa[NA], sb[NBB];
    auto load = [&](int k0) {
        const bool kin = k0 + LBK <= K;
#pragma unroll
        for (int b = 0; b < NA; ++b)
            load_slice(static_cast<const TA *>(a.A[b]), M, K, m0, k0, fast_m && kin, sa[b]);
#pragma unroll
        for (int b = 0; b < NBB; ++b)
            load_slice(static_cast<const TB *>(a.B[b]), N, K, n0, k0, fast_n && kin, sb[b]);
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int b = 0; b < NA; ++b) stash_slice<MODE>(As[buf][b], sa[b]);
#pragma unroll
        for (int b = 0; b < NBB; ++b) stash_slice<MODE>(Bs[buf][b], sb[b]);
    };

    f4 acc[NB][2][2];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[b][i][j] = f4{0.f, 0.f, 0.f, 0.f};

    auto compute = [&](int buf) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const LdsTile<MODE> &TA_ = As[buf][A_BATCHED ? b : 0];
            const LdsTile<MODE> &TB_ = Bs[buf][A_BATCHED ? 0 : b];
            if constexpr (MODE == MCA_PREC_FP32) {
                // A fragment: row l%16, k l/16; B fragment: k l/16, column l%16
#pragma unroll
                for (int k4 = 0; k4 < LBK / 4; ++k4) {
                    const int kk = k4 * 4 + (lane >> 4);
                    float fa[2], fb[2];
#pragma unroll
                    for (int i = 0; i < 2; ++i) fa[i] = TA_.v[wm + i * 16 + (lane & 15)][kk];
#pragma unroll
                    for (int j = 0; j < 2; ++j) fb[j] = TB_.v[wn + j * 16 + (lane & 15)][kk];
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j)
                            acc[b][i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j],
                                                                                acc[b][i][j], 0, 0, 0);
                }
            } else {
                // A fragment: row l%16, k 8(l/16)..+7; B fragment: column l%16, same k
                const int kk = (lane >> 4) * 8;
                bf8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    ah[i] = *reinterpret_cast<const bf8 *>(&TA_.hi[wm + i * 16 + (lane & 15)][kk]);
                    bh[i] = *reinterpret_cast<const bf8 *>(&TB_.hi[wn + i * 16 + (lane & 15)][kk]);
                    if constexpr (MODE == MCA_PREC_BF16X3) {
                        al[i] = *reinterpret_cast<const bf8 *>(&TA_.lo[wm + i * 16 + (lane & 15)][kk]);
                        bl[i] = *reinterpret_cast<const bf8 *>(&TB_.lo[wn + i * 16 + (lane & 15)][kk]);
                    }
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        if constexpr (MODE == MCA_PREC_BF16X3) {
                            acc[b][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j],
                                                                                   acc[b][i][j], 0, 0, 0);
                            acc[b][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j],
                                                                                   acc[b][i][j], 0, 0, 0);
                        }
                        acc[b][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j],
                                                                               acc[b][i][j], 0, 0, 0);
                    }
            }
        }
    };

    const int nk = (K + LBK - 1) / LBK;
    load(0);
    stash(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load((kt + 1) * LBK);
        compute(kt & 1);
        if (kt + 1 < nk) stash((kt + 1) & 1);
        __syncthreads();
    }

    // accumulator element r of lane l: row 4 (l/16) + r, column l%16
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
                const int col = n0 + wn + j * 16 + (lane & 15);
                if (row >= M || col >= N) continue;
                const size_t o = (size_t)row * N + col;
                if constexpr (EPI == EPI_PERMODE) {
                    // mode (p, q) = (col, row): [[lt + a1, -a1], [-a2, lb + a2]] x = r
                    const double lt = a.lam_row[row], lb = a.lam_col[col];
                    const double det = lt * lb + a.a2 * lt + a.a1 * lb;
                    const double rt = acc[0][i][j][r], rb = acc[NB - 1][i][j][r];
                    static_cast<TO *>(a.O[0])[o] = (TO)(((lb + a.a2) * rt + a.a1 * rb) / det);
                    static_cast<TO *>(a.O[1])[o] = (TO)((a.a2 * rt + (lt + a.a1) * rb) / det);
                } else {
#pragma unroll
                    for (int b = 0; b < NB; ++b) static_cast<TO *>(a.O[b])[o] = (TO)acc[b][i][j][r];
                }
            }
}

template <int MODE>
hipError_t chain(const LowPrecChain &c, hipStream_t s)
{
    const int m = c.m, n = c.n;
    LpArgs g{};
    g.skip = c.skip;
    g.a1 = c.a1;
    g.a2 = c.a2;
    auto tiles = [](int M, int N) { return ((M + LBM - 1) / LBM) * ((N + LBN - 1) / LBN); };
    // 1. U^T (n x m) = Q_n^T . X^T     A = QnT (n x n), B = X (m x n), both layers of X
    g.M = n; g.N = m; g.K = n;
    g.A[0] = c.QnT; g.B[0] = c.rt; g.B[1] = c.rb; g.O[0] = c.u_t; g.O[1] = c.u_b;
    hipLaunchKernelGGL((k_gemm_nt_lp<MODE, 2, false, float, double, float, EPI_STORE>),
                       dim3(tiles(n, m)), dim3(LTPB), 0, s, g);
    // 2. W^T (n x m) = U^T . Q_m      A = U^T (n x m), B = QmT (m x m); per-mode solve
    g = LpArgs{};
    g.skip = c.skip; g.a1 = c.a1; g.a2 = c.a2;
    g.M = n; g.N = m; g.K = m;
    g.A[0] = c.u_t; g.A[1] = c.u_b; g.B[0] = c.QmT; g.O[0] = c.w_t; g.O[1] = c.w_b;
    g.lam_row = c.lt; g.lam_col = c.lb;
    hipLaunchKernelGGL((k_gemm_nt_lp<MODE, 2, true, float, float, float, EPI_PERMODE>),
                       dim3(tiles(n, m)), dim3(LTPB), 0, s, g);
    // 3. Y (m x n) = Q_m . X^hat      A = Qm (m x m), B = X^hat^T (n x m)
    g = LpArgs{};
    g.skip = c.skip;
    g.M = m; g.N = n; g.K = m;
    g.A[0] = c.Qm; g.B[0] = c.w_t; g.B[1] = c.w_b; g.O[0] = c.u_t; g.O[1] = c.u_b;
    hipLaunchKernelGGL((k_gemm_nt_lp<MODE, 2, false, float, float, float, EPI_STORE>),
                       dim3(tiles(m, n)), dim3(LTPB), 0, s, g);
    // 4. Z (m x n) = Y . Q_n^T         A = Y (m x n), B = Qn (n x n); FP64 out
    g = LpArgs{};
    g.skip = c.skip;
    g.M = m; g.N = n; g.K = n;
    g.A[0] = c.u_t; g.A[1] = c.u_b; g.B[0] = c.Qn; g.O[0] = c.zt; g.O[1] = c.zb;
    hipLaunchKernelGGL((k_gemm_nt_lp<MODE, 2, true, float, float, double, EPI_STORE>),
                       dim3(tiles(m, n)), dim3(LTPB), 0, s, g);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_precond_lowprec(int precision, const LowPrecChain &c, hipStream_t s)
{
    switch (precision) {
    case MCA_PREC_FP32: return chain<MCA_PREC_FP32>(c, s);
    case MCA_PREC_BF16: return chain<MCA_PREC_BF16>(c, s);
    case MCA_PREC_BF16X3: return chain<MCA_PREC_BF16X3>(c, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mca
