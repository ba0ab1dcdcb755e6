// gemm_lp.hip -- reduced-precision eigenbasis transforms for the mixed-precision
// preconditioner (flexible GMRES absorbs their rounding).
//
// Every transform here has the shape  O = A B^T  with both operands stored
// row-major with K contiguous (A: M x K, B: N x K).  The per-mode
// preconditioner (the block formula of eq. (block) applied per Kronecker
// eigenmode) then becomes four such products without any transpose:
//   U^T   = Q_n^T . X^T      A = Q_n^T,  B = X       (contract over j)
//   W^T   = U^T . Q_m        A = U^T,    B = Q_m^T   (contract over i), + 2x2 solve
//   Y     = Q_m . X^hat      A = Q_m,    B = X^hat^T (contract over p)
//   Z     = Y . Q_n^T        A = Y,      B = Q_n     (contract over q)
// (X is the m x n input, hats mark the eigenbasis.)
//
// Operands live in global memory in the format the MFMA consumes, so staging
// into LDS is a plain 16-byte copy: FP32 arrays for the FP32 mode
// (v_mfma_f32_16x16x4f32), or bfloat16 hi + lo planes (v = hi + lo to ~16
// bits) for the BF16 modes (v_mfma_f32_16x16x32_bf16: hi.hi for BF16,
// hi.hi + hi.lo + lo.hi for BF16X3, always accumulated in FP32).  The
// eigenbases are converted once in the plan, the FP64 input r by a split
// kernel, and every intermediate by the epilogue of the product that makes it.
//
// Tiling: 64 x 64 output tiles (four waves of 32 x 32, K slices of 64, or of
// 32 in launches with many tiles) or, where those still give 256 or more
// workgroups, 128 x 128 tiles (eight waves, K slices of 32).  K is staged
// through LDS either from registers (two slices of global loads in flight,
// double-buffered LDS) or, for interior 128 x 128 split-BF16 / BF16 tiles,
// straight from global memory into three LDS buffers in a software-pipelined
// loop whose waves read and multiply in two groups of opposite phase (see
// gemm_nt_tile).  One operand may have two batches (the two layers)
// that share the other operand.
//
// LDS layout of a staged slice (register-staged path): 16-byte chunks, in
// sub-slices of four chunks per row (32 bf16 or 16 floats of K).  Chunk c' of
// row r in 16-row group g of sub-slice h sits at index
//   h * 4 ROWS + g * 64 + c' * 16 + ((r mod 16) xor c'),
// so one MFMA fragment (16 rows of one chunk column) is one 256-byte block,
// its rows permuted by an xor of c'.  A slice is staged by lane quads that
// each load one row's 64 contiguous bytes (coalesced global loads), the four
// quads of a 16-lane group taking rows 4 apart.  Measured on gfx950
// (rocprofv3 SQ_LDS_BANK_CONFLICT, 16-byte accesses): these fragment reads
// and these stores run without bank conflicts, while rows padded to 80 bytes,
// or 64-byte rows with a chunk swizzle, take twice the LDS cycles on the
// fragment reads; lanes that each load a different row (one chunk column at a
// time) avoid the conflicts but cost more in the global loads than they save.
#include <hip/hip_bf16.h>

#include <type_traits>

#include "mca_internal.h"

namespace mca {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int LBM = 64, LBK = 64, LTPB = 256;
// Waves of a 128 x 128 tile's workgroup: eight (two per SIMD, 64 x 32 each), so
// that one wave's LDS reads and barrier waits overlap the other's MFMAs; 64 x 64
// tiles keep four waves of 32 x 32.
constexpr int kWaves128 = 8;
constexpr int kWaves64 = 4;   // 64 x 64 tiles, 64-deep slices (eight: no faster)
template <int TS, int KS>
constexpr int lp_threads()
{
    return TS == 128 ? 64 * kWaves128 : (TS == 64 && KS == 64) ? 64 * kWaves64 : LTPB;
}
template <int MODE>
struct Fmt {   // BF16 modes: two bf16 planes, 8 values per 16-byte chunk
    static constexpr int kPlanes = (MODE == MCA_PREC_BF16X3) ? 2 : 1;
    static constexpr int kPerChunk = 8;
    using elem = __bf16;
};
template <>
struct Fmt<MCA_PREC_FP32> {
    static constexpr int kPlanes = 1;
    static constexpr int kPerChunk = 4;
    using elem = float;
};

// One operand: planes[0] (hi or FP32 values) and planes[1] (lo), row stride K.
struct Operand {
    const void *p[2];
};

// One operand slice in LDS: ROWS rows (tile edge) x KS values of K, as
// 16-byte chunks in the layout described above.
template <int MODE, int ROWS, int KS>
struct Tile {
    static constexpr int kChunks = ROWS * KS / Fmt<MODE>::kPerChunk;   // per plane
    u4 c[Fmt<MODE>::kPlanes][kChunks];
};

// Chunk `id` of a staged slice: its row r and chunk column c (chunks of
// Fmt::kPerChunk values along K) for the global load, and its LDS index.
template <int ROWS>
__device__ __forceinline__ void chunk_pos(int id, int &r, int &c, int &lds)
{
    const int h = id / (4 * ROWS), v = id % (4 * ROWS);
    const int G = v >> 4, w = v & 15;
    const int g = G >> 2, j = G & 3, q = w >> 2, i = w & 3;
    r = g * 16 + q * 4 + j;
    c = h * 4 + i;
    lds = h * 4 * ROWS + g * 64 + i * 16 + ((q * 4 + j) ^ i);
}

// 16-byte chunks of one ROWS x KS operand slice per plane, per thread of NT.
template <int MODE, int ROWS, int KS, int NT>
constexpr int chunks_per_thread()
{
    static_assert(ROWS * KS / Fmt<MODE>::kPerChunk % NT == 0, "chunks per thread");
    return ROWS * KS / Fmt<MODE>::kPerChunk / NT;
}

template <int MODE, int ROWS, int KS, int NT>
struct Regs {
    u4 c[Fmt<MODE>::kPlanes][chunks_per_thread<MODE, ROWS, KS, NT>()];
};

// Operand planes are device (global) memory; loads through these pointers
// are global loads, which the wait counters track apart from LDS traffic (a
// generic pointer would give flat loads, whose waits also hold every LDS
// access behind them).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *global_ptr(const T *p)
{
    return (const __attribute__((address_space(1))) T *)p;
}

template <int MODE, int ROWS, int KS, int NT>
__device__ __forceinline__ void load_op(const Operand &op, int rows, int K, size_t ld, int koff, int r0,
                                        int k0, bool fast, Regs<MODE, ROWS, KS, NT> &g)
{
    constexpr int PC = Fmt<MODE>::kPerChunk;
    constexpr int CPT = chunks_per_thread<MODE, ROWS, KS, NT>();
    using E = typename Fmt<MODE>::elem;
#pragma unroll
    for (int pl = 0; pl < Fmt<MODE>::kPlanes; ++pl) {
        const auto *base = global_ptr(static_cast<const E *>(op.p[pl])) + koff;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            int rr, cc, li;
            chunk_pos<ROWS>(threadIdx.x + c * NT, rr, cc, li);
            const int r = r0 + rr, k = k0 + cc * PC;
            if (fast) {
                g.c[pl][c] = *reinterpret_cast<const __attribute__((address_space(1))) u4 *>(
                    base + (size_t)r * ld + k);
            } else {
                // clamped element loads; out-of-range elements become zero
                union {
                    u4 v;
                    E e[PC];
                } u;
                const size_t rc = (size_t)min(r, rows - 1);
#pragma unroll
                for (int e = 0; e < PC; ++e) {
                    const E x = base[rc * ld + min(k + e, K - 1)];
                    u.e[e] = (r < rows && k + e < K) ? x : (E)0.0f;
                }
                g.c[pl][c] = u.v;
            }
        }
    }
}

template <int MODE, int ROWS, int KS, int NT>
__device__ __forceinline__ void stash_op(Tile<MODE, ROWS, KS> &t, const Regs<MODE, ROWS, KS, NT> &g)
{
    constexpr int CPT = chunks_per_thread<MODE, ROWS, KS, NT>();
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        int r, cc, li;
        chunk_pos<ROWS>(threadIdx.x + c * NT, r, cc, li);
#pragma unroll
        for (int pl = 0; pl < Fmt<MODE>::kPlanes; ++pl) t.c[pl][li] = g.c[pl][c];
    }
}

// MFMA fragments from a staged slice.  BF16 (16x16x32): lane l holds row
// l % 16 of 16-row group g, k values 8 (l / 16) .. + 7 of k step s (sub-slice
// s).  FP32 (16x16x4): lane l holds row l % 16, k value 4 s + l / 16.
template <int MODE, int ROWS, int KS>
__device__ __forceinline__ bf8 frag_bf16(const Tile<MODE, ROWS, KS> &t, int pl, int g, int s, int lane)
{
    const int cq = lane >> 4;
    return *reinterpret_cast<const bf8 *>(&t.c[pl][s * 4 * ROWS + g * 64 + cq * 16 + ((lane & 15) ^ cq)]);
}
template <int MODE, int ROWS, int KS>
__device__ __forceinline__ float frag_f32(const Tile<MODE, ROWS, KS> &t, int g, int s, int lane)
{
    const int cq = s & 3;
    return reinterpret_cast<const float *>(
        &t.c[0][(s >> 2) * 4 * ROWS + g * 64 + cq * 16 + ((lane & 15) ^ cq)])[lane >> 4];
}

// O = A B^T.  NB batches of A (A_BATCHED) or of B, sharing the other operand.
// Output formats: OUT_F32, OUT_BF2 (hi/lo planes), OUT_BF1 (hi plane), OUT_F64.
enum { OUT_F32 = 0, OUT_BF2 = 1, OUT_F64 = 2, OUT_BF1 = 3 };

struct LpArgs {
    int M, N, K;
    Operand A[2], B[2];
    void *O[2][2];                     // [batch][plane]
    const double *lam_row, *lam_col;   // PERMODE: eigenvalues along rows (lt) / cols (lb)
    double a1, a2;
    int vec;                           // all operands 16-byte aligned with K % 8 == 0
    const int *skip;
    // Persymmetric fold (see chain below).  lda, ldb: row strides of A and B
    // (0: K).  split 1: tiles of output columns >= N / 2 read A from K on
    // (A's second half along K); split 2: tiles of output rows >= M / 2 read B
    // from K on.  ileave: output row r of the first half goes to row
    // 32 (r / 16) + r % 16, of the second half to that + 16.
    int lda, ldb, split, ileave;
    int unfold;   // as EPI_UNFOLD16, chosen at run time (grouped launches)
};

template <typename T>
__device__ __forceinline__ void put(const LpArgs &a, int b, size_t o, T v, int out)
{
    if (out == OUT_F64) {
        static_cast<double *>(a.O[b][0])[o] = (double)v;
    } else if (out == OUT_F32) {
        static_cast<float *>(a.O[b][0])[o] = (float)v;
    } else {
        const float f = (float)v;
        const __bf16 hi = (__bf16)f;
        static_cast<__bf16 *>(a.O[b][0])[o] = hi;
        if (out == OUT_BF2) static_cast<__bf16 *>(a.O[b][1])[o] = (__bf16)(f - (float)hi);
    }
}

// Four consecutive outputs from offset o (o a multiple of 4, the plane
// 16-byte aligned): one 8-, 16- or two 16-byte stores per plane.  The values
// are rounded as put() rounds them one by one.
__device__ __forceinline__ bool aligned_out(const void *p)
{
    return p == nullptr || (reinterpret_cast<uintptr_t>(p) & 15) == 0;
}
__device__ __forceinline__ void put4(const LpArgs &a, int b, size_t o, const double (&v)[4], int out)
{
    if (out == OUT_F64) {
        double2 *d = reinterpret_cast<double2 *>(static_cast<double *>(a.O[b][0]) + o);
        d[0] = double2{v[0], v[1]};
        d[1] = double2{v[2], v[3]};
    } else if (out == OUT_F32) {
        *reinterpret_cast<float4 *>(static_cast<float *>(a.O[b][0]) + o) =
            float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    } else {
        typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
        bf4 hi, lo;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float f = (float)v[r];
            hi[r] = (__bf16)f;
            lo[r] = (__bf16)(f - (float)hi[r]);
        }
        *reinterpret_cast<bf4 *>(static_cast<__bf16 *>(a.O[b][0]) + o) = hi;
        if (out == OUT_BF2) *reinterpret_cast<bf4 *>(static_cast<__bf16 *>(a.O[b][1]) + o) = lo;
    }
}

constexpr int DEPTH = 2;   // K slices in flight (deeper rings measured no faster)

// One TS x TS output tile at (m0, n0) of O = A B^T: four waves of (TS/2)^2 or
// eight waves, FI x FJ MFMA tiles of 16 x 16 each; K staged in slices of KS.
// With eight waves a wave covers half the tile along the operand that has one
// batch and a quarter along the one with two (the layers), which keeps the
// fragment reads per MFMA lowest: 16 reads for 48 split-BF16 MFMAs per k step.
template <int MODE, int NB, bool A_BATCHED, int OUT, int EPI, int TS, int KS>
__device__ __forceinline__ void gemm_nt_tile(const LpArgs &a, int m0, int n0)
{
    constexpr int NA = A_BATCHED ? NB : 1, NBB = A_BATCHED ? 1 : NB;
    constexpr int NT = lp_threads<TS, KS>(), WAVES = NT / 64;
    constexpr bool TWO_A = A_BATCHED && NB == 2;
    constexpr int WTM = (WAVES == 8) ? (TWO_A ? TS / 4 : TS / 2) : TS / 2;
    constexpr int WTN = (WAVES == 8) ? (TWO_A ? TS / 2 : TS / 4) : TS / 2;
    constexpr int FI = WTM / 16, FJ = WTN / 16;
    constexpr int PL = Fmt<MODE>::kPlanes;
    using TileT = Tile<MODE, TS, KS>;
    using RegsT = Regs<MODE, TS, KS, NT>;
    // One K slice of every operand tile (the A tiles first) per LDS buffer; the
    // buffers are distinct objects, so that the compiler's wait for the
    // direct-to-LDS loads before a fragment read covers only that buffer's.
    struct SliceBuf {
        TileT t[NA + NBB];
    };
    __shared__ SliceBuf L0, L1;
    auto As = [&](int buf, int b) -> TileT & { return buf ? L1.t[b] : L0.t[b]; };
    auto Bs = [&](int buf, int b) -> TileT & { return buf ? L1.t[NA + b] : L0.t[NA + b]; };
    const int M = a.M, N = a.N, K = a.K;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave / (TS / WTN)) * WTM, wn = (wave % (TS / WTN)) * WTN;
    const int gm = wm / 16, gn = wn / 16;   // first 16-row group of the wave's A / B rows
    const bool fast_m = a.vec && (m0 + TS <= M);
    const bool fast_n = a.vec && (n0 + TS <= N);
    const size_t lda = a.lda ? a.lda : K, ldb = a.ldb ? a.ldb : K;
    const int koa = (a.split == 1 && n0 >= N / 2) ? K : 0;
    const int kob = (a.split == 2 && m0 >= M / 2) ? K : 0;

    struct Stage {
        RegsT ra[NA], rb[NBB];
    };
    auto load = [&](Stage &st, int k0) {
        const bool kin = k0 + KS <= K;
#pragma unroll
        for (int b = 0; b < NA; ++b)
            load_op<MODE, TS, KS, NT>(a.A[b], M, K, lda, koa, m0, k0, fast_m && kin, st.ra[b]);
#pragma unroll
        for (int b = 0; b < NBB; ++b)
            load_op<MODE, TS, KS, NT>(a.B[b], N, K, ldb, kob, n0, k0, fast_n && kin, st.rb[b]);
    };
    // interior tiles with K a whole number of slices: unconditional 16-byte loads
    auto load_fast = [&](Stage &st, int k0) {
#pragma unroll
        for (int b = 0; b < NA; ++b) load_op<MODE, TS, KS, NT>(a.A[b], M, K, lda, koa, m0, k0, true, st.ra[b]);
#pragma unroll
        for (int b = 0; b < NBB; ++b) load_op<MODE, TS, KS, NT>(a.B[b], N, K, ldb, kob, n0, k0, true, st.rb[b]);
    };
    auto stash = [&](const Stage &st, int buf) {
#pragma unroll
        for (int b = 0; b < NA; ++b) stash_op<MODE, TS, KS, NT>(As(buf, b), st.ra[b]);
#pragma unroll
        for (int b = 0; b < NBB; ++b) stash_op<MODE, TS, KS, NT>(Bs(buf, b), st.rb[b]);
    };

    f4 acc[NB][FI][FJ];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < FI; ++i)
#pragma unroll
            for (int j = 0; j < FJ; ++j) acc[b][i][j] = f4{0.f, 0.f, 0.f, 0.f};

    // the MFMAs of one k step of split-BF16 / BF16 fragments: lo.hi and hi.lo
    // first, then hi.hi, each over every accumulator (no two MFMAs in a row
    // share an accumulator).  Every MFMA takes the B fragment as its first
    // operand, so it forms the transposed 16 x 16 block: lane l then holds
    // row l % 16 and the four consecutive columns 4 (l / 16) .. + 3 of the
    // output, which the epilogue stores as one vector per plane.
    auto mfma_bf16 = [&](const bf8 (&fa)[NA][PL][FI], const bf8 (&fb)[NBB][PL][FJ]) {
        if constexpr (MODE == MCA_PREC_BF16X3) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int i = 0; i < FI; ++i)
#pragma unroll
                    for (int j = 0; j < FJ; ++j)
                        acc[b][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            fb[A_BATCHED ? 0 : b][0][j], fa[A_BATCHED ? b : 0][1][i], acc[b][i][j], 0, 0, 0);
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int i = 0; i < FI; ++i)
#pragma unroll
                    for (int j = 0; j < FJ; ++j)
                        acc[b][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            fb[A_BATCHED ? 0 : b][PL - 1][j], fa[A_BATCHED ? b : 0][0][i], acc[b][i][j], 0, 0, 0);
        }
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int i = 0; i < FI; ++i)
#pragma unroll
                for (int j = 0; j < FJ; ++j)
                    acc[b][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        fb[A_BATCHED ? 0 : b][0][j], fa[A_BATCHED ? b : 0][0][i], acc[b][i][j], 0, 0, 0);
    };
    auto read_bf16 = [&](int buf, int s, bf8 (&fa)[NA][PL][FI], bf8 (&fb)[NBB][PL][FJ]) {
#pragma unroll
        for (int b = 0; b < NA; ++b)
#pragma unroll
            for (int pl = 0; pl < PL; ++pl)
#pragma unroll
                for (int i = 0; i < FI; ++i) fa[b][pl][i] = frag_bf16(As(buf, b), pl, gm + i, s, lane);
#pragma unroll
        for (int b = 0; b < NBB; ++b)
#pragma unroll
            for (int pl = 0; pl < PL; ++pl)
#pragma unroll
                for (int j = 0; j < FJ; ++j) fb[b][pl][j] = frag_bf16(Bs(buf, b), pl, gn + j, s, lane);
    };

    auto compute = [&](int buf) {
        if constexpr (MODE == MCA_PREC_FP32) {
#pragma unroll
            for (int s4 = 0; s4 < KS / 4; ++s4) {
                float fa[NA][FI], fb[NBB][FJ];
#pragma unroll
                for (int b = 0; b < NA; ++b)
#pragma unroll
                    for (int i = 0; i < FI; ++i) fa[b][i] = frag_f32(As(buf, b), gm + i, s4, lane);
#pragma unroll
                for (int b = 0; b < NBB; ++b)
#pragma unroll
                    for (int j = 0; j < FJ; ++j) fb[b][j] = frag_f32(Bs(buf, b), gn + j, s4, lane);
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int i = 0; i < FI; ++i)
#pragma unroll
                        for (int j = 0; j < FJ; ++j)
                            acc[b][i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                fb[A_BATCHED ? 0 : b][j], fa[A_BATCHED ? b : 0][i], acc[b][i][j], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int s = 0; s < KS / 32; ++s) {
                bf8 fa[NA][PL][FI], fb[NBB][PL][FJ];
                read_bf16(buf, s, fa, fb);
                mfma_bf16(fa, fb);
            }
        }
    };

    bool done = false;
    // (128 x 128 tiles, one wave per 16-row block of an operand plane; the same
    // loop on 64 x 64 tiles, four waves, two workgroups per CU instead of three,
    // measured slower: Monte-Carlo batch 41.1 vs 40.2 ms)
    if constexpr (TS == 128 && KS == 32 && MODE != MCA_PREC_FP32 && WAVES == TS / 16) {
        if (fast_m && fast_n && K % KS == 0 && K >= 3 * KS) {
            // Interior tile: every slice goes from global memory straight into
            // LDS (global_load_lds_dwordx4, 16 bytes per lane), three buffers,
            // two slices ahead of the one being read; the waves read and
            // multiply in two groups of opposite phase (below).  Layout of a
            // buffer: operand tile t, plane p, row r, 16-byte chunk c of the
            // row's 32 values at byte t sizeof(Tile) + p 64 TS + 64 r +
            // 16 (c ^ ((r >> 1) & 3)), so that each lane quad loads one row's
            // 64 contiguous bytes (the load writes LDS in lane order) and the
            // eight rows of a fragment read that one pass serves fall on
            // distinct 16-byte bank groups of a 128-byte period (rocprofv3
            // SQ_LDS_BANK_CONFLICT: half of the LDS cycles were conflicts with
            // the chunk swizzled by bits 2-3 of the row).
            __shared__ SliceBuf L2;
            constexpr int NQ = (NA + NBB) * PL;   // 1 KB loads per wave and slice
            constexpr int kPlaneBytes = TS * 64;  // one plane of a slice: TS rows of 32 values
            static_assert(sizeof(TileT) == PL * kPlaneBytes, "slice layout");
            typedef const void __attribute__((address_space(1))) *gptr;
            typedef void __attribute__((address_space(3))) *lptr;
            using I0 = std::integral_constant<int, 0>;
            using I1 = std::integral_constant<int, 1>;
            using I2 = std::integral_constant<int, 2>;
            auto bufp = [&](auto bc) -> char * {
                constexpr int B = decltype(bc)::value;
                if constexpr (B == 0) return reinterpret_cast<char *>(&L0);
                else if constexpr (B == 1) return reinterpret_cast<char *>(&L1);
                else return reinterpret_cast<char *>(&L2);
            };
            // Wave w loads row block w (16 rows) of every operand plane: its
            // instruction q takes operand tile q / PL, plane q % PL.  Each lane
            // quad loads one row's 64 bytes, chunk c of the row to chunk
            // c ^ ((row >> 1) & 3) of LDS, which for 16-row blocks is
            // c ^ ((lane >> 3) & 3).  Addresses: a wave-uniform base (scalar
            // registers) plus a per-lane byte offset, one per operand side.
            const int wv = __builtin_amdgcn_readfirstlane(wave);
            const int lc = ((lane & 3) ^ ((lane >> 3) & 3)) * 16;
            const unsigned voff_a = (unsigned)((lane >> 2) * lda * 2 + lc);
            const unsigned voff_b = (unsigned)((lane >> 2) * ldb * 2 + lc);
            const char *sbase[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int t = q / PL, pl = q % PL;
                const void *base = nullptr;
#pragma unroll
                for (int u = 0; u < NA; ++u)
                    if (t == u) base = a.A[u].p[pl];
#pragma unroll
                for (int u = 0; u < NBB; ++u)
                    if (t == NA + u) base = a.B[u].p[pl];
                const size_t row0 = (size_t)((t < NA ? m0 : n0) + wv * 16);
                sbase[q] = static_cast<const char *>(base) +
                           2 * (row0 * (t < NA ? lda : ldb) + (t < NA ? koa : kob));
            }
            const int dst_w = wv * 1024;
            auto issue = [&](auto bc, int k0) {
                char *lb = bufp(bc) + dst_w;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int t = q / PL, pl = q % PL;
                    __builtin_amdgcn_global_load_lds(
                        (gptr)(sbase[q] + 2 * (size_t)k0 + (t < NA ? voff_a : voff_b)),
                        (lptr)(lb + t * (int)sizeof(TileT) + pl * kPlaneBytes), 16, 0, 0);
                }
            };
            using FA = bf8[NA][PL][FI];
            using FB = bf8[NBB][PL][FJ];
            auto read = [&](auto bc, FA &fa, FB &fb) {
                const char *lb = bufp(bc);
                auto frag = [&](int t, int pl, int row) -> bf8 {
                    const int c = (lane >> 4) ^ ((row >> 1) & 3);
                    return *reinterpret_cast<const bf8 *>(lb + t * (int)sizeof(TileT) + pl * kPlaneBytes +
                                                          row * 64 + c * 16);
                };
#pragma unroll
                for (int b = 0; b < NA; ++b)
#pragma unroll
                    for (int pl = 0; pl < PL; ++pl)
#pragma unroll
                        for (int i = 0; i < FI; ++i) fa[b][pl][i] = frag(b, pl, wm + i * 16 + (lane & 15));
#pragma unroll
                for (int b = 0; b < NBB; ++b)
#pragma unroll
                    for (int pl = 0; pl < PL; ++pl)
#pragma unroll
                        for (int j = 0; j < FJ; ++j) fb[b][pl][j] = frag(NA + b, pl, wn + j * 16 + (lane & 15));
            };
            // s_waitcnt immediates (gfx9 encoding: vmcnt in bits 3:0 and 15:14,
            // expcnt in 6:4, lgkmcnt in 11:8): the loads of one slice may stay in
            // flight, LDS reads all done
            constexpr int kWaitOne = (NQ & 15) | ((NQ >> 4) << 14) | (7 << 4);
            constexpr int kWaitNone = 7 << 4;
            static_assert(2 * NQ < 64, "vmcnt range");
            const int nk = K / KS, last = nk - 1;
            // Two groups of four waves, one wave of each group per SIMD, work in
            // opposite phases: while one group multiplies the slice it read in
            // the previous phase, the other reads its fragments of a slice from
            // LDS and issues the next slice's loads, so that the MFMA pipe and
            // the LDS serve different waves at the same time.  Group 0 reads
            // slice j in phase 2j and multiplies it in phase 2j + 1; group 1
            // one phase later.  Phases end at a barrier; before the barrier
            // that opens an even phase (group 0 reads slice j + 1 there) every
            // wave has its part of slice j + 1 in LDS, and at every phase end
            // its own fragment reads are done, so slice j - 1's buffer is free
            // for slice j + 2 once both groups have read it.  Both groups pass
            // the same number of barriers (2 nk).
            constexpr int kWaitLgkm = 15 | (3 << 14) | (7 << 4);   // LDS reads done, loads may fly
            // (the dispatcher places waves w and w + 4 of a workgroup on one
            // SIMD, measured on gfx950 through the hardware wave id; grouping
            // w and w + 1 instead, both waves of a SIMD in one group, measured
            // 6% slower than all eight waves reading and multiplying in step)
            const int grp = wv >> 2;
            FA fa;
            FB fb;
            issue(I0{}, 0);
            issue(I1{}, KS);
            __builtin_amdgcn_s_waitcnt(kWaitOne);   // slice 0 has landed
            asm volatile("s_barrier" ::: "memory");
            auto phase_end = [&](auto vm_wait) {
                __builtin_amdgcn_sched_barrier(0);   // the wait stays at the end of the phase
                if constexpr (decltype(vm_wait)::value) __builtin_amdgcn_s_waitcnt(kWaitOne);
                else __builtin_amdgcn_s_waitcnt(kWaitLgkm);
                __builtin_amdgcn_sched_barrier(0);
                asm volatile("s_barrier" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
            };
            using ToEven = std::true_type;   // the barrier that opens an even phase
            using ToOdd = std::false_type;   // the barrier that opens an odd phase
            // read slice j (buffer BJ) and load slice min(j + 2, last) into the
            // buffer after the next (it held slice j - 1)
            auto fetch = [&](auto bj, int j) {
                constexpr int BJ = decltype(bj)::value;
                read(bj, fa, fb);
                __builtin_amdgcn_sched_barrier(0);
                issue(std::integral_constant<int, (BJ + 2) % 3>{}, min(j + 2, last) * KS);
            };
            if (grp == 0) {
                // phase 0 reads slice 0; every step then multiplies slice j and
                // reads slice j + 1 (the loop starts after the barrier whose wait
                // covers the reads' slice)
                fetch(I0{}, 0);
                auto step0 = [&](auto bn, int j) {
                    phase_end(ToOdd{});
                    mfma_bf16(fa, fb);
                    phase_end(ToEven{});
                    fetch(bn, j + 1);
                };
                int j = 0;
                for (; j + 3 < nk; j += 3) {
                    step0(I1{}, j);
                    step0(I2{}, j + 1);
                    step0(I0{}, j + 2);
                }
                // one to three steps left, the last without a read
                auto tail0 = [&](auto bn, int jj) {
                    phase_end(ToOdd{});
                    mfma_bf16(fa, fb);
                    phase_end(ToEven{});
                    if (jj + 1 < nk) fetch(bn, jj + 1);
                };
                tail0(I1{}, j);
                if (j + 1 < nk) tail0(I2{}, j + 1);
                if (j + 2 < nk) tail0(I0{}, j + 2);
            } else {
                phase_end(ToOdd{});   // phase 0: group 1 waits
                auto step1 = [&](auto bj, int j) {
                    fetch(bj, j);
                    phase_end(ToEven{});
                    mfma_bf16(fa, fb);
                    phase_end(ToOdd{});
                };
                // every step but the last ends at a barrier
                int j = 0;
                for (; j + 3 <= nk - 1; j += 3) {
                    step1(I0{}, j);
                    step1(I1{}, j + 1);
                    step1(I2{}, j + 2);
                }
                if (j < nk - 1) step1(I0{}, j);
                if (j + 1 < nk - 1) step1(I1{}, j + 1);
                auto last1 = [&](auto bj) {
                    fetch(bj, last);
                    phase_end(ToEven{});
                    mfma_bf16(fa, fb);
                };
                const int bl = last % 3;
                if (bl == 0) last1(I0{});
                else if (bl == 1) last1(I1{});
                else last1(I2{});
            }
            // no LDS DMA may outlive the workgroup (nor land in a buffer the
            // epilogue reuses)
            __builtin_amdgcn_s_waitcnt(kWaitNone);
            done = true;
        }
    }
    if (!done) {
        // DEPTH K slices in flight: a ring of register stages; the loop is unrolled
        // by DEPTH so that the stages rotate by name.  At step k the stage that
        // held slice k (already in LDS) receives slice k + DEPTH, slice k is
        // multiplied, and slice k + 1 moves from registers into the other LDS buffer.
        const int nk = (K + KS - 1) / KS;
        Stage st[DEPTH];
        int kb = 0;
        if (fast_m && fast_n && K % KS == 0 && nk >= DEPTH) {
            // the same ring with the loads' conditions lifted out of the steady
            // state, so that no branch sits between a load and the wait before
            // its LDS store and the wait covers only that stage
    #pragma unroll
            for (int u = 0; u < DEPTH; ++u) load_fast(st[u], u * KS);
            stash(st[0], 0);
            __syncthreads();
            for (; kb + 2 * DEPTH < nk + 1; kb += DEPTH) {
    #pragma unroll
                for (int u = 0; u < DEPTH; ++u) {
                    const int k = kb + u;   // k + DEPTH < nk throughout
                    load_fast(st[u], (k + DEPTH) * KS);
                    __builtin_amdgcn_sched_barrier(0);   // issue the loads before the MFMAs
                    compute(k & 1);
                    stash(st[(u + 1) % DEPTH], (k + 1) & 1);
                    __syncthreads();
                }
            }
        } else {
    #pragma unroll
            for (int u = 0; u < DEPTH; ++u)
                if (u < nk) load(st[u], u * KS);
            stash(st[0], 0);
            __syncthreads();
        }
        for (; kb < nk; kb += DEPTH) {
    #pragma unroll
            for (int u = 0; u < DEPTH; ++u) {
                const int k = kb + u;
                if (k < nk) {   // uniform
                    if (k + DEPTH < nk) load(st[u], (k + DEPTH) * KS);
                    compute(k & 1);
                    if (k + 1 < nk) stash(st[(u + 1) % DEPTH], (k + 1) & 1);
                    __syncthreads();
                }
            }
        }
    }

    // accumulator element r of lane l: row l % 16, column 4 (l / 16) + r (the
    // transposed block, see above).  Four consecutive outputs go out as one
    // vector store per plane where the row holds them and the planes allow it.
    bool ovec = (N % 4 == 0);
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int pl = 0; pl < 2; ++pl) ovec = ovec && aligned_out(a.O[b][pl]);
    if (EPI == EPI_UNFOLD16 || a.unfold) {
        // rows of A come in 16-row groups, alternately of the symmetric and the
        // antisymmetric half (the interleave of the product that made A): the
        // lane's rows in MFMA blocks 2t and 2t + 1 are row p of both halves,
        // and the output rows are p (sum) and M - 1 - p (difference)
        static_assert(FI % 2 == 0, "pairs of 16-row blocks");
#pragma unroll
        for (int t = 0; t < FI / 2; ++t)
#pragma unroll
            for (int j = 0; j < FJ; ++j) {
                const int p = (m0 + wm + 32 * t) / 2 + (lane & 15);
                const int col0 = n0 + wn + j * 16 + (lane >> 4) * 4;
                if (2 * p >= M || col0 >= N) continue;
                const size_t o0 = (size_t)p * N + col0, o1 = (size_t)(M - 1 - p) * N + col0;
                const bool whole = ovec && col0 + 4 <= N;
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    double x0[4], x1[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double sym = acc[b][2 * t][j][r], anti = acc[b][2 * t + 1][j][r];
                        x0[r] = sym + anti;
                        x1[r] = sym - anti;
                    }
                    if (whole) {
                        put4(a, b, o0, x0, OUT);
                        put4(a, b, o1, x1, OUT);
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (col0 + r < N) {
                                put(a, b, o0 + r, x0[r], OUT);
                                put(a, b, o1 + r, x1[r], OUT);
                            }
                    }
                }
            }
        return;
    }
#pragma unroll
    for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FJ; ++j) {
            const int row = m0 + wm + i * 16 + (lane & 15);
            const int col0 = n0 + wn + j * 16 + (lane >> 4) * 4;
            if (row >= M || col0 >= N) continue;
            int orow = row;
            if (a.ileave) {
                const int hh = M / 2, q = row < hh ? row : row - hh;
                orow = 32 * (q / 16) + q % 16 + (row < hh ? 0 : 16);
            }
            const size_t o = (size_t)orow * N + col0;
            const bool whole = ovec && col0 + 4 <= N;
            if constexpr (EPI == EPI_PERMODE) {
                // mode (p, q) = (col, row): [[lt + a1, -a1], [-a2, lb + a2]] x = r
                const double lt = global_ptr(a.lam_row)[row];
                double x0[4], x1[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double lb = global_ptr(a.lam_col)[min(col0 + r, N - 1)];
                    const double det = lt * lb + a.a2 * lt + a.a1 * lb;
                    const double rt = acc[0][i][j][r], rb = acc[NB - 1][i][j][r];
                    x0[r] = ((lb + a.a2) * rt + a.a1 * rb) / det;
                    x1[r] = (a.a2 * rt + (lt + a.a1) * rb) / det;
                }
                if (whole) {
                    put4(a, 0, o, x0, OUT);
                    put4(a, 1, o, x1, OUT);
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (col0 + r < N) {
                            put(a, 0, o + r, x0[r], OUT);
                            put(a, 1, o + r, x1[r], OUT);
                        }
                }
            } else {
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    if (whole) {
                        const double x[4] = {acc[b][i][j][0], acc[b][i][j][1], acc[b][i][j][2], acc[b][i][j][3]};
                        put4(a, b, o, x, OUT);
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (col0 + r < N) put(a, b, o + r, acc[b][i][j][r], OUT);
                    }
                }
            }
        }
}

// XCD-aware order: every XCD owns a contiguous run of workgroup ids.
__device__ __forceinline__ int xcd_order(int bid, int nwg)
{
    return (nwg % 8 == 0) ? (bid % 8) * (nwg / 8) + bid / 8 : bid;
}

template <int MODE, int NB, bool A_BATCHED, int OUT, int EPI, int TS, int KS>
__global__ __launch_bounds__((lp_threads<TS, KS>())) void k_gemm_nt_lp(LpArgs a)
{
    if (a.skip && *a.skip) return;
    const int t = xcd_order(blockIdx.x, gridDim.x);
    const int tiles_n = (a.N + TS - 1) / TS;
    gemm_nt_tile<MODE, NB, A_BATCHED, OUT, EPI, TS, KS>(a, (t / tiles_n) * TS, (t % tiles_n) * TS);
}

// Grouped launch over many crossbars: tile t of the table names an instance's
// product (descriptor) and the tile's origin.  The data operand and the output
// of every instance sit at an element offset from the launch's base planes;
// the eigenbasis operand is the instance's own.
template <int MODE, int NB, bool A_BATCHED, int OUT, int EPI, int TS, int KS>
__global__ __launch_bounds__((lp_threads<TS, KS>())) void k_gemm_nt_lp_grouped(GroupedLp g)
{
    const int t = xcd_order(blockIdx.x, gridDim.x);
    const int4 tile = g.tiles[t];
    const LpDesc &d = g.descs[tile.x];
    if (g.ctl && g.ctl[4 * d.inst]) return;   // this crossbar's GMRES cycle has converged
    LpArgs a{};
    a.M = d.M;
    a.N = d.N;
    a.K = d.K;
    const size_t es = g.data_elem_bytes, os = g.out_elem_bytes;
    const void *const *dbase = d.alt ? g.data_alt : g.data;
    for (int b = 0; b < 2; ++b) {
        Operand data;
        for (int pl = 0; pl < 2; ++pl)
            data.p[pl] = dbase[pl] ? static_cast<const char *>(dbase[pl]) + (d.off_data + b * d.mn) * es
                                   : nullptr;
        if (A_BATCHED) a.A[b] = data;
        else a.B[b] = data;
        for (int pl = 0; pl < 2; ++pl)
            a.O[b][pl] = g.out[pl] ? static_cast<char *>(g.out[pl]) + (d.off_out + b * d.mn) * os
                                   : nullptr;
    }
    Operand q;
    q.p[0] = d.Q[0];
    q.p[1] = d.Q[1];
    if (A_BATCHED) a.B[0] = q;
    else a.A[0] = q;
    a.lam_row = d.lam_row;
    a.lam_col = d.lam_col;
    if (g.a_inst) a.a1 = a.a2 = g.a_inst[d.inst * g.a_stride];
    a.vec = d.vec;
    a.lda = d.lda;
    a.ldb = d.ldb;
    a.split = d.split;
    a.ileave = d.ileave;
    a.unfold = d.unfold;
    gemm_nt_tile<MODE, NB, A_BATCHED, OUT, EPI, TS, KS>(a, tile.y, tile.z);
}

// FP64 -> the operand format of MODE (FP32, or bf16 hi/lo planes), two arrays.
template <int MODE>
__global__ __launch_bounds__(256) void k_split(const double *__restrict__ x0,
                                               const double *__restrict__ x1, size_t len,
                                               void *o00, void *o01, void *o10, void *o11,
                                               const int *__restrict__ skip)
{
    if (skip && *skip) return;
    const int nb = x1 ? 2 : 1;
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < len; k += (size_t)gridDim.x * 256) {
        for (int b = 0; b < nb; ++b) {
            const float f = (float)(b == 0 ? x0[k] : x1[k]);
            if constexpr (MODE == MCA_PREC_FP32) {
                static_cast<float *>(b == 0 ? o00 : o10)[k] = f;
            } else {
                const __bf16 hi = (__bf16)f;
                static_cast<__bf16 *>(b == 0 ? o00 : o10)[k] = hi;
                if constexpr (MODE == MCA_PREC_BF16X3)
                    static_cast<__bf16 *>(b == 0 ? o01 : o11)[k] = (__bf16)(f - (float)hi);
            }
        }
    }
}

// The same with the rows folded for a persymmetric G_bot (m = 2h): output row
// i < h is x_i + x_{m-1-i}, row h + i is x_i - x_{m-1-i} (in FP64, then split).
template <int MODE>
__global__ __launch_bounds__(256) void k_split_fold(const double *__restrict__ x0,
                                                    const double *__restrict__ x1, int m, int n,
                                                    void *o00, void *o01, void *o10, void *o11,
                                                    const int *__restrict__ skip)
{
    if (skip && *skip) return;
    const int h = m / 2;
    const size_t half = (size_t)h * n;
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < half; k += (size_t)gridDim.x * 256) {
        const size_t i = k / n, j = k - i * n;
        const size_t lo = i * n + j, hi = ((size_t)m - 1 - i) * n + j;
        for (int b = 0; b < 2; ++b) {
            const double *x = b == 0 ? x0 : x1;
            const double sv[2] = {x[lo] + x[hi], x[lo] - x[hi]};
            for (int q = 0; q < 2; ++q) {
                const size_t e = q == 0 ? k : half + k;
                const float f = (float)sv[q];
                if constexpr (MODE == MCA_PREC_FP32) {
                    static_cast<float *>(b == 0 ? o00 : o10)[e] = f;
                } else {
                    const __bf16 hv = (__bf16)f;
                    static_cast<__bf16 *>(b == 0 ? o00 : o10)[e] = hv;
                    if constexpr (MODE == MCA_PREC_BF16X3)
                        static_cast<__bf16 *>(b == 0 ? o01 : o11)[e] = (__bf16)(f - (float)hv);
                }
            }
        }
    }
}

// Grouped form over a batch: block b takes chunk fold_tab[b].y (kFoldChunk
// elements of the m/2 x n half) of crossbar fold_tab[b].x, whose chain is
// folded, and writes its operand-format Krylov vector x (both layers) into w
// with the rows folded as above: the planes are read back to FP32 (hi + lo),
// summed / subtracted there, and split again.
template <int MODE>
__global__ __launch_bounds__(256) void k_fold_grouped(const LpDesc *__restrict__ descs,
                                                      const int2 *__restrict__ fold_tab,
                                                      const void *x0, const void *x1, void *w0,
                                                      void *w1, const int *ctl)
{
    const int2 fb = fold_tab[blockIdx.x];
    const LpDesc &d = descs[fb.x];
    if (ctl && ctl[4 * d.inst]) return;
    const int m = d.N, n = d.M, h = m / 2;   // product 1 is n x m
    const size_t half = (size_t)h * n;
    auto get = [&](size_t e) -> float {
        if constexpr (MODE == MCA_PREC_FP32) {
            return static_cast<const float *>(x0)[e];
        } else {
            float v = (float)static_cast<const __bf16 *>(x0)[e];
            if constexpr (MODE == MCA_PREC_BF16X3) v += (float)static_cast<const __bf16 *>(x1)[e];
            return v;
        }
    };
    auto put1 = [&](size_t e, float f) {
        if constexpr (MODE == MCA_PREC_FP32) {
            static_cast<float *>(w0)[e] = f;
        } else {
            const __bf16 hv = (__bf16)f;
            static_cast<__bf16 *>(w0)[e] = hv;
            if constexpr (MODE == MCA_PREC_BF16X3) static_cast<__bf16 *>(w1)[e] = (__bf16)(f - (float)hv);
        }
    };
    const size_t k0 = (size_t)fb.y * kFoldChunk, k1 = std::min(half, k0 + kFoldChunk);
    for (size_t k = k0 + threadIdx.x; k < k1; k += 256) {
        const size_t i = k / n, j = k - i * n;
        for (int b = 0; b < 2; ++b) {
            const size_t base = d.off_data + b * d.mn;
            const float lo = get(base + i * n + j), hi = get(base + ((size_t)m - 1 - i) * n + j);
            put1(base + k, lo + hi);
            put1(base + half + k, lo - hi);
        }
    }
}

bool aligned16(const void *p) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// 128 x 128 tiles (K slices of 32) when they still give 256 or more workgroups:
// four times the operand reuse of 64 x 64 tiles; else 64 x 64 (K slices of 64).
template <int MODE, int NB, bool A_BATCHED, int OUT, int EPI>
void launch_nt(const LpArgs &g, hipStream_t s)
{
    const long big = (long)((g.M + 127) / 128) * ((g.N + 127) / 128);
    if (big >= 256)
        hipLaunchKernelGGL((k_gemm_nt_lp<MODE, NB, A_BATCHED, OUT, EPI, 128, 32>), dim3((int)big),
                           dim3(lp_threads<128, 32>()), 0, s, g);
    else
        hipLaunchKernelGGL((k_gemm_nt_lp<MODE, NB, A_BATCHED, OUT, EPI, LBM, LBK>),
                           dim3(((g.M + LBM - 1) / LBM) * ((g.N + LBM - 1) / LBM)),
                           dim3(lp_threads<LBM, LBK>()), 0, s, g);
}

template <int MODE>
hipError_t chain(const LowPrecChain &c, hipStream_t s)
{
    constexpr int OUT = (MODE == MCA_PREC_FP32) ? OUT_F32 : (MODE == MCA_PREC_BF16X3) ? OUT_BF2 : OUT_BF1;
    const int m = c.m, n = c.n;
    const size_t mn = (size_t)m * n;
    auto op = [](const LpPlanes &p) {
        Operand o;
        o.p[0] = p.p[0];
        o.p[1] = p.p[1];
        return o;
    };
    auto vec_ok = [&](const LpArgs &g) {
        bool ok = (g.K % 8 == 0) && (g.lda % 8 == 0) && (g.ldb % 8 == 0);
        for (int b = 0; b < 2; ++b)
            for (int pl = 0; pl < 2; ++pl) ok = ok && aligned16(g.A[b].p[pl]) && aligned16(g.B[b].p[pl]);
        return ok ? 1 : 0;
    };
    if (c.fold) {
        // Persymmetric G_bot (m = 2h, h a multiple of 128): its eigenvectors are
        // [u; J u] (symmetric) and [u; -J u] (antisymmetric), u from the halves
        // U_s, U_a (h x h, scaled by 1/sqrt2), so both Q_m-side products split
        // into two products of half the depth on folded data.  The modes run
        // symmetric first (eigenvalues lbp).
        const int h = m / 2;
        // 0. r -> folded rows (sums, then differences), operand format (unless
        //    the pass that made r wrote them)
        if (!c.r_split) {
            const int blocks = (int)std::min<size_t>(((size_t)h * n + 255) / 256, 4096);
            hipLaunchKernelGGL(k_split_fold<MODE>, dim3(blocks), dim3(256), 0, s, c.rt, c.rb, m, n,
                               c.x[0].p[0], c.x[0].p[1], c.x[1].p[0], c.x[1].p[1], c.skip);
        }
        LpArgs g{};
        // 1. U'^T (n x m) = Q_n^T . X'^T: columns i < h from the sums, h + i from the differences
        g.skip = c.skip;
        g.M = n; g.N = m; g.K = n;
        g.A[0] = op(c.QnT); g.B[0] = op(c.x[0]); g.B[1] = op(c.x[1]);
        for (int b = 0; b < 2; ++b) { g.O[b][0] = c.u[b].p[0]; g.O[b][1] = c.u[b].p[1]; }
        g.vec = vec_ok(g);
        launch_nt<MODE, 2, false, OUT, EPI_STORE>(g, s);
        // 2. W'^T (n x m): symmetric modes = U'^T[:, :h] . U_s, antisymmetric =
        //    U'^T[:, h:] . U_a (B = [U_s^T; U_a^T], m x h); per-mode solve
        g = LpArgs{};
        g.skip = c.skip; g.a1 = c.a1; g.a2 = c.a2;
        g.M = n; g.N = m; g.K = h; g.lda = m; g.split = 1;
        g.A[0] = op(c.u[0]); g.A[1] = op(c.u[1]); g.B[0] = op(c.QmTf);
        for (int b = 0; b < 2; ++b) { g.O[b][0] = c.w[b].p[0]; g.O[b][1] = c.w[b].p[1]; }
        g.lam_row = c.lt; g.lam_col = c.lbp;
        g.vec = vec_ok(g);
        launch_nt<MODE, 2, true, OUT, EPI_PERMODE>(g, s);
        // 3. Y' (m x n) = [U_s . X^hat_s; U_a . X^hat_a] (A = [U_s; U_a], m x h; B
        //    from K = h on for the antisymmetric rows), rows interleaved in groups of 16
        g = LpArgs{};
        g.skip = c.skip;
        g.M = m; g.N = n; g.K = h; g.ldb = m; g.split = 2; g.ileave = 1;
        g.A[0] = op(c.Qmf); g.B[0] = op(c.w[0]); g.B[1] = op(c.w[1]);
        for (int b = 0; b < 2; ++b) { g.O[b][0] = c.u[b].p[0]; g.O[b][1] = c.u[b].p[1]; }
        g.vec = vec_ok(g);
        launch_nt<MODE, 2, false, OUT, EPI_STORE>(g, s);
        // 4. Z = unfold(Y' . Q_n^T): row p of both halves gives rows p and m-1-p
        g = LpArgs{};
        g.skip = c.skip;
        g.M = m; g.N = n; g.K = n;
        g.A[0] = op(c.u[0]); g.A[1] = op(c.u[1]); g.B[0] = op(c.Qn);
        g.O[0][0] = c.zt; g.O[1][0] = c.zb;
        g.vec = vec_ok(g);
        launch_nt<MODE, 2, true, OUT_F64, EPI_UNFOLD16>(g, s);
        return hipGetLastError();
    }
    // 0. r (FP64) -> operand format
    if (!c.r_split) {
        const int blocks = (int)std::min<size_t>((mn + 255) / 256, 4096);
        hipLaunchKernelGGL(k_split<MODE>, dim3(blocks), dim3(256), 0, s, c.rt, c.rb, mn,
                           c.x[0].p[0], c.x[0].p[1], c.x[1].p[0], c.x[1].p[1], c.skip);
    }
    LpArgs g{};
    // 1. U^T (n x m) = Q_n^T . X^T     A = QnT (n x n), B = X (m x n), both layers of X
    g.skip = c.skip;
    g.M = n; g.N = m; g.K = n;
    g.A[0] = op(c.QnT); g.B[0] = op(c.x[0]); g.B[1] = op(c.x[1]);
    for (int b = 0; b < 2; ++b) { g.O[b][0] = c.u[b].p[0]; g.O[b][1] = c.u[b].p[1]; }
    g.vec = vec_ok(g);
    launch_nt<MODE, 2, false, OUT, EPI_STORE>(g, s);
    // 2. W^T (n x m) = U^T . Q_m      A = U^T (n x m), B = QmT (m x m); per-mode solve
    g = LpArgs{};
    g.skip = c.skip; g.a1 = c.a1; g.a2 = c.a2;
    g.M = n; g.N = m; g.K = m;
    g.A[0] = op(c.u[0]); g.A[1] = op(c.u[1]); g.B[0] = op(c.QmT);
    for (int b = 0; b < 2; ++b) { g.O[b][0] = c.w[b].p[0]; g.O[b][1] = c.w[b].p[1]; }
    g.lam_row = c.lt; g.lam_col = c.lb;
    g.vec = vec_ok(g);
    launch_nt<MODE, 2, true, OUT, EPI_PERMODE>(g, s);
    // 3. Y (m x n) = Q_m . X^hat      A = Qm (m x m), B = X^hat^T (n x m)
    g = LpArgs{};
    g.skip = c.skip;
    g.M = m; g.N = n; g.K = m;
    g.A[0] = op(c.Qm); g.B[0] = op(c.w[0]); g.B[1] = op(c.w[1]);
    for (int b = 0; b < 2; ++b) { g.O[b][0] = c.u[b].p[0]; g.O[b][1] = c.u[b].p[1]; }
    g.vec = vec_ok(g);
    launch_nt<MODE, 2, false, OUT, EPI_STORE>(g, s);
    // 4. Z (m x n) = Y . Q_n^T         A = Y (m x n), B = Qn (n x n); FP64 out
    g = LpArgs{};
    g.skip = c.skip;
    g.M = m; g.N = n; g.K = n;
    g.A[0] = op(c.u[0]); g.A[1] = op(c.u[1]); g.B[0] = op(c.Qn);
    g.O[0][0] = c.zt; g.O[1][0] = c.zb;
    g.vec = vec_ok(g);
    launch_nt<MODE, 2, true, OUT_F64, EPI_STORE>(g, s);
    return hipGetLastError();
}

// Tile edge 128 (K slices of 32); 64 with K slices of 64, or of 32 when the
// launch has at least two tiles per CU: the shallower slices halve the LDS
// and the registers of a workgroup, so that two share a CU.
constexpr int kSlice32Tiles = 512;

template <int MODE, int NB, bool A_BATCHED, int OUT, int EPI>
void launch_grouped(const GroupedLp &g, int ntiles, int tile, hipStream_t s)
{
    if (tile == 64 && ntiles >= kSlice32Tiles)
        hipLaunchKernelGGL((k_gemm_nt_lp_grouped<MODE, NB, A_BATCHED, OUT, EPI, 64, 32>),
                           dim3(ntiles), dim3(lp_threads<64, 32>()), 0, s, g);
    else if (tile == 128)
        hipLaunchKernelGGL((k_gemm_nt_lp_grouped<MODE, NB, A_BATCHED, OUT, EPI, 128, 32>),
                           dim3(ntiles), dim3(lp_threads<128, 32>()), 0, s, g);
    else
        hipLaunchKernelGGL((k_gemm_nt_lp_grouped<MODE, NB, A_BATCHED, OUT, EPI, LBM, LBK>),
                           dim3(ntiles), dim3(lp_threads<LBM, LBK>()), 0, s, g);
}

template <int MODE>
hipError_t chain_grouped(const GroupedChain &c, hipStream_t s)
{
    constexpr int OUT = (MODE == MCA_PREC_FP32) ? OUT_F32 : (MODE == MCA_PREC_BF16X3) ? OUT_BF2 : OUT_BF1;
    const size_t es = (MODE == MCA_PREC_FP32) ? 4 : 2;
    if (!c.r_split) {
        const int blocks = (int)std::min<size_t>((c.len + 255) / 256, 8192);
        hipLaunchKernelGGL(k_split<MODE>, dim3(blocks), dim3(256), 0, s, c.r, nullptr, c.len,
                           c.x.p[0], c.x.p[1], nullptr, nullptr, nullptr);
    }
    GroupedLp g{};
    g.a_inst = c.a_inst;
    g.a_stride = c.a_stride;
    g.ctl = c.ctl;
    g.data_elem_bytes = es;
    g.out_elem_bytes = es;
    auto set = [&](int step, const LpPlanes &in, const LpPlanes &out) {
        g.descs = c.descs[step];
        g.tiles = c.tiles[step];
        g.data[0] = in.p[0];
        g.data[1] = in.p[1];
        g.out[0] = out.p[0];
        g.out[1] = out.p[1];
        g.data_alt[0] = g.data_alt[1] = nullptr;
    };
    // folded crossbars: x -> w with the rows folded (unless the pass that
    // converted r did so); product 1 reads w
    if (c.fold_blocks > 0 && !(c.r_split && c.r_folded))
        hipLaunchKernelGGL(k_fold_grouped<MODE>, dim3(c.fold_blocks), dim3(256), 0, s, c.descs[0],
                           c.fold_tab, c.x.p[0], c.x.p[1], c.w.p[0], c.w.p[1], c.ctl);
    set(0, c.x, c.u);
    g.data_alt[0] = c.w.p[0];
    g.data_alt[1] = c.w.p[1];
    if (c.ev[0]) {
        const hipError_t e = hipEventRecord(c.ev[0], s);
        if (e != hipSuccess) return e;
    }
    launch_grouped<MODE, 2, false, OUT, EPI_STORE>(g, c.ntiles[0], c.tile, s);
    set(1, c.u, c.w);
    launch_grouped<MODE, 2, true, OUT, EPI_PERMODE>(g, c.ntiles[1], c.tile, s);
    set(2, c.w, c.u);
    launch_grouped<MODE, 2, false, OUT, EPI_STORE>(g, c.ntiles[2], c.tile, s);
    LpPlanes z;
    z.p[0] = c.z;
    z.p[1] = nullptr;
    set(3, c.u, z);
    g.out_elem_bytes = 4;
    launch_grouped<MODE, 2, true, OUT_F32, EPI_STORE>(g, c.ntiles[3], c.tile, s);
    if (c.ev[1]) {
        const hipError_t e = hipEventRecord(c.ev[1], s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_precond_lowprec_grouped(int precision, const GroupedChain &c, hipStream_t s)
{
    switch (precision) {
    case MCA_PREC_FP32: return chain_grouped<MCA_PREC_FP32>(c, s);
    case MCA_PREC_BF16: return chain_grouped<MCA_PREC_BF16>(c, s);
    case MCA_PREC_BF16X3: return chain_grouped<MCA_PREC_BF16X3>(c, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_precond_lowprec(int precision, const LowPrecChain &c, hipStream_t s)
{
    switch (precision) {
    case MCA_PREC_FP32: return chain<MCA_PREC_FP32>(c, s);
    case MCA_PREC_BF16: return chain<MCA_PREC_BF16>(c, s);
    case MCA_PREC_BF16X3: return chain<MCA_PREC_BF16X3>(c, s);
    default: return hipErrorInvalidValue;
    }
}

// FP64 eigenbasis -> FP32 values or bf16 hi/lo (host, at plan upload).
void split_host(const double *src, size_t count, int precision, void *p0, void *p1)
{
    for (size_t k = 0; k < count; ++k) {
        const float f = (float)src[k];
        if (precision == MCA_PREC_FP32) {
            static_cast<float *>(p0)[k] = f;
        } else {
            const __bf16 hi = (__bf16)f;
            static_cast<__bf16 *>(p0)[k] = hi;
            static_cast<__bf16 *>(p1)[k] = (__bf16)(f - (float)hi);
        }
    }
}

}  // namespace mca
