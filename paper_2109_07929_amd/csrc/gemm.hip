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
// Tiling: 64 x 64 output tile per 512-thread workgroup, eight waves of 32 x 16
// (two waves per SIMD), each wave a 2 x 1 grid of v_mfma_f64_16x16x4
// accumulators; K is staged through LDS in double-buffered 32-deep slices
// with two slices of global loads in flight.  A second batch (the bottom
// layer) may share the same R tile: the per-mode 2x2 solve of the block
// formula (eq. (block)) then runs in the epilogue on both accumulators.
// Launches of at most one whole tile per CU take the direct-to-LDS variant
// (k_gemm_tn_f64_dma), which can also fuse the persymmetric unfold.
#include "mca_internal.h"

namespace mca {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, PAD = 0;

// LDS column of element (k, c) of a staged slice: odd K rows swap their
// 16-double halves, so the four K rows that one MFMA fragment read touches
// (16 lanes each) fall on distinct banks in every 32-lane pass (rows are 64
// doubles = 128 dwords, a multiple of the 64 banks).
__device__ __forceinline__ int swz(int k, int c) { return c ^ ((k & 1) << 4); }
constexpr int kXcds = 8;      // MI355X: 8 XCDs, workgroups dispatched round-robin
constexpr int kGroupM = 4;    // tile rows per group of the tile order

// Tile of workgroup `bid`.  Consecutive workgroup ids land on different XCDs
// (each with its own L2), so ids are first regrouped so that every XCD owns a
// contiguous run of tile ids, and runs are ordered in groups of kGroupM tile
// rows: the 32 tiles one XCD holds at a time then share 4 row panels of L and
// 8 column panels of R instead of 16 + 2.
__device__ __forceinline__ void tile_of(int bid, int nwg, int tiles_m, int tiles_n, int &tm,
                                        int &tn)
{
    int t = bid;
    if (nwg % kXcds == 0) t = (bid % kXcds) * (nwg / kXcds) + bid / kXcds;
    const int per_group = kGroupM * tiles_n;
    const int g = t / per_group;
    const int first = g * kGroupM;
    const int gsize = min(tiles_m - first, kGroupM);
    const int r = t - g * per_group;
    tm = first + r % gsize;
    tn = r / gsize;
}

// One K slice of L (NB batches) and R in registers: rows lr + RP h of the
// slice (RP = threads / 16 rows per pass), 4 consecutive columns each.
template <int NB, int H>
struct Stage {
    double2 l[NB][H][2];
    double2 r[H][2];
};

// Epilogue: accumulator element r of lane l is row l/16 + 4r, column l%16 of
// its 16 x 16 tile (the f64 16x16x4 layout, checked on gfx950).
template <int NB, int EPI, int WJ>
__device__ __forceinline__ void store_tile(const GemmArgs &a, const d4 (&acc)[NB][2][WJ], int m0,
                                           int n0, int wm, int wn, int lane)
{
    const int M = a.M, N = a.N;
    // the shift a1 = a2 from the device when the launch carries it there
    const double a1 = (EPI != EPI_STORE && a.shift) ? a.shift[0] : a.a1;
    const double a2 = (EPI != EPI_STORE && a.shift) ? a.shift[0] : a.a2;
    const double inv_a1 = (EPI != EPI_STORE) ? (a.shift ? a.shift[1] : 1.0 / a1) : 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < WJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + i * 16 + (lane >> 4) + 4 * r;
                const int col = n0 + wn + j * 16 + (lane & 15);
                if (row >= M || col >= N) continue;
                const size_t ldo = a.ldo ? (size_t)a.ldo : (size_t)N;
                const size_t o = (size_t)row * ldo + col;
                if constexpr (EPI == EPI_STORE) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) (b == 0 ? a.O0 : a.O1)[o] = acc[b][i][j][r];
                } else if constexpr (EPI == EPI_DIV_MU) {
                    // eigenvalue of M (eq. (M)) for mode (row, col), summed without cancellation
                    const double lb = a.lb[row], lt = a.lt[col];
                    const double mu = lb * lt * inv_a1 + lb + a2 * inv_a1 * lt;
                    a.O0[o] = acc[0][i][j][r] / mu;
                } else {
                    // per-mode block solve [[lt + a1, -a1], [-a2, lb + a2]] x = r
                    const double lb = a.lb[row], lt = a.lt[col];
                    const double det = lt * lb + a2 * lt + a1 * lb;
                    const double rt = acc[0][i][j][r], rb = acc[NB - 1][i][j][r];
                    a.O0[o] = ((lb + a2) * rt + a1 * rb) / det;
                    a.O1[o] = (a2 * rt + (lt + a1) * rb) / det;
                }
            }
}

// WAVES = 4: 2 x 2 waves of 32 x 32 (2 x 2 MFMA tiles each), one wave per SIMD.
// WAVES = 8: 2 x 4 waves of 32 x 16 (2 x 1 MFMA tiles each), two waves per
// SIMD, so that one wave's LDS reads overlap the other's MFMAs.
// UPFRONT: read every MFMA fragment of a K slice from LDS before its MFMAs.
template <int NB, int EPI, int BK, int WAVES, bool UPFRONT>
__global__ __launch_bounds__(64 * WAVES) void k_gemm_tn_f64(GemmArgs a)
{
    // a pair launch: the second half of the grid computes the second product
    int bid = blockIdx.x, nwg = gridDim.x;
    if (NB == 1 && a.pair) {
        nwg >>= 1;
        if (bid >= nwg) {
            bid -= nwg;
            a.L0 = a.L1;
            a.R = a.R1;
            a.O0 = a.O1;
        }
    }
    constexpr int NT = 64 * WAVES;
    constexpr int RP = NT / 16;          // slice rows staged per pass
    constexpr int H = BK / RP;           // passes per slice
    constexpr int WJ = (WAVES == 4) ? 2 : 1;    // 16-column MFMA tiles per wave
    constexpr int WCOLS = 16 * WJ;
    static_assert(H >= 1 && BK % RP == 0, "slice depth");
    __shared__ double Ls[2][NB][BK][BM + PAD];
    __shared__ double Rs[2][BK][BN + PAD];
    if (a.skip && *a.skip) return;   // uniform: a converged GMRES cycle

    // EPI_UNFOLD (whole tiles only): 32 rows of A = Y_s^T R over the same rows
    // of B = Y_a^T R, as in the direct-to-LDS kernel
    constexpr bool UNF = EPI == EPI_UNFOLD;
    static_assert(!UNF || NB == 1, "one batch");
    const int M = a.M, N = a.N, K = a.K;
    const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
    int tm, tn;
    tile_of(bid, nwg, tiles_m, tiles_n, tm, tn);
    const int m0 = tm * (UNF ? BM / 2 : BM), n0 = tn * BN;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave / (BN / WCOLS)) * 32, wn = (wave % (BN / WCOLS)) * WCOLS;
    const double *Lb[2] = {a.L0, NB > 1 ? a.L1 : a.L0};

    // Interior tiles with 16-byte aligned rows (a.vec) use unconditional
    // 16-byte loads; edge tiles clamp every address into the array and zero
    // the out-of-range values, so no load is ever out of bounds.
    const int lr = tid >> 4, lc = (tid & 15) * 4;
    const bool inside = a.vec && (m0 + BM <= M) && (n0 + BN <= N);

    auto load = [&](Stage<NB, H> &st, int k0) {
        if (inside && k0 + BK <= K) {
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const size_t gk = (size_t)(k0 + lr + RP * h);
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const double2 *p = reinterpret_cast<const double2 *>(
                        UNF ? (lc < 32 ? a.L0 : a.L1) + gk * (M / 2) + m0 + (lc & 31)
                            : Lb[b] + gk * M + m0 + lc);
                    st.l[b][h][0] = p[0];
                    st.l[b][h][1] = p[1];
                }
                const double2 *q = reinterpret_cast<const double2 *>(a.R + gk * N + n0 + lc);
                st.r[h][0] = q[0];
                st.r[h][1] = q[1];
            }
        } else {
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const int gk = k0 + lr + RP * h;
                const bool krow = gk < K;
                const size_t kc = (size_t)min(gk, K - 1);
                double v[4];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int gm = m0 + lc + e;
                        const double x = Lb[b][kc * M + min(gm, M - 1)];
                        v[e] = (krow && gm < M) ? x : 0.0;
                    }
                    st.l[b][h][0] = double2{v[0], v[1]};
                    st.l[b][h][1] = double2{v[2], v[3]};
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int gn = n0 + lc + e;
                    const double x = a.R[kc * N + min(gn, N - 1)];
                    v[e] = (krow && gn < N) ? x : 0.0;
                }
                st.r[h][0] = double2{v[0], v[1]};
                st.r[h][1] = double2{v[2], v[3]};
            }
        }
    };
    auto stash = [&](const Stage<NB, H> &st, int buf) {
#pragma unroll
        for (int h = 0; h < H; ++h) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int row = lr + RP * h;
                double2 *d = reinterpret_cast<double2 *>(&Ls[buf][b][row][swz(row, lc)]);
                d[0] = st.l[b][h][0];
                d[1] = st.l[b][h][1];
            }
            const int row = lr + RP * h;
            double2 *d = reinterpret_cast<double2 *>(&Rs[buf][row][swz(row, lc)]);
            d[0] = st.r[h][0];
            d[1] = st.r[h][1];
        }
    };

    d4 acc[NB][2][WJ];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < WJ; ++j) acc[b][i][j] = d4{0.0, 0.0, 0.0, 0.0};

    // MFMA operands: A (16 x 4) lane l holds row l%16, k l/16; B (4 x 16) lane l
    // holds k l/16, column l%16.
    constexpr int NS = UPFRONT ? BK / 4 : 2;
    double af[NS][NB][2], bf[NS][WJ];
    auto frag = [&](int buf, int k4, int slot) {
        const int kr = k4 * 4 + (lane >> 4);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int b = 0; b < NB; ++b)
                af[slot][b][i] = Ls[buf][b][kr][swz(kr, wm + i * 16 + (lane & 15))];
#pragma unroll
        for (int j = 0; j < WJ; ++j) bf[slot][j] = Rs[buf][kr][swz(kr, wn + j * 16 + (lane & 15))];
    };
    auto mfmas = [&](int slot) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < WJ; ++j)
                    acc[b][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[slot][b][i], bf[slot][j],
                                                                         acc[b][i][j], 0, 0, 0);
    };
    auto compute = [&](int buf) {
        // sched_barrier fences keep the compiler from sinking the LDS reads
        // next to their first use, which would expose their latency
        if constexpr (UPFRONT) {
#pragma unroll
            for (int k4 = 0; k4 < BK / 4; ++k4) frag(buf, k4, k4);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k4 = 0; k4 < BK / 4; ++k4) mfmas(k4);
        } else {
            frag(buf, 0, 0);
#pragma unroll
            for (int k4 = 0; k4 < BK / 4; ++k4) {
                if (k4 + 1 < BK / 4) frag(buf, k4 + 1, (k4 + 1) & 1);
                __builtin_amdgcn_sched_barrier(0);
                mfmas(k4 & 1);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };

    // Two K slices in flight: the registers of slice kt+1 were loaded one step
    // earlier and slice kt+2 is issued now (two register sets; the loop is
    // unrolled by two so that the sets swap by name).
    const int nk = (K + BK - 1) / BK;
    Stage<NB, H> s0, s1;
    load(s0, 0);
    stash(s0, 0);
    if (nk > 1) load(s1, BK);
    __syncthreads();
    int kt = 0;
    for (; kt + 1 < nk; kt += 2) {
        if (kt + 2 < nk) load(s0, (kt + 2) * BK);
        compute(kt & 1);
        stash(s1, (kt + 1) & 1);
        __syncthreads();
        if (kt + 3 < nk) load(s1, (kt + 3) * BK);
        compute((kt + 1) & 1);
        if (kt + 2 < nk) stash(s0, (kt + 2) & 1);
        __syncthreads();
    }
    if (kt < nk) compute(kt & 1);

    if constexpr (UNF) {
        // B passes through the first L buffer once every wave is done with it
        __syncthreads();
        double(*X)[BM + PAD] = Ls[0][0];
        if (wm == 32) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < WJ; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        X[i * 16 + (lane >> 4) + 4 * r][wn + j * 16 + (lane & 15)] = acc[0][i][j][r];
        }
        __syncthreads();
        if (wm == 0) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < WJ; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int p = m0 + i * 16 + (lane >> 4) + 4 * r;
                        const int c = wn + j * 16 + (lane & 15);
                        const double A = acc[0][i][j][r], Bv = X[p - m0][c];
                        a.O0[(size_t)p * N + n0 + c] = A + Bv;
                        a.O0[(size_t)(M - 1 - p) * N + n0 + c] = A - Bv;
                    }
        }
    } else {
        store_tile<NB, EPI, WJ>(a, acc, m0, n0, wm, wn, lane);
    }
}

// Direct-to-LDS variant for whole tiles (M, N multiples of 64, K a multiple of
// BK * ST, 16-byte aligned rows, one batch): every BK-deep K slice moves from
// global memory into LDS by global_load_lds_dwordx4 (16 bytes per lane, 1 KB
// per wave instruction, no register staging), ST slices deep in ST LDS
// buffers.  A wave's instruction fills two consecutive slice rows in LDS
// order; each lane picks the global columns that land in the swizzled layout
// of swz().  One barrier per slice: after it, the buffer computed one slice
// earlier is free and takes the slice ST - 1 ahead.
// EPI_UNFOLD: the tile is 32 rows p of A = Y_s^T R (LDS columns 0..31 of the L
// slice, from Y_s) over the same 32 rows of B = Y_a^T R (columns 32..63, from
// Y_a); the waves holding B pass it through LDS to the waves holding A, which
// store A + B to row p and A - B to row M-1-p.
template <int BK>
struct DmaSlice {
    double l[BK][64];
    double r[BK][64];
};

template <int EPI, int BK, int ST, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_gemm_tn_f64_dma(GemmArgs a)
{
    static_assert(BK % (2 * WAVES) == 0 && BK >= 32 && (ST == 2 || ST == 4), "slice shape");
    static_assert(WAVES == 4 || WAVES == 8, "2 x 2 waves of 32 x 32 or 2 x 4 of 32 x 16");
    int bid = blockIdx.x, nwg = gridDim.x;
    if (a.pair) {
        nwg >>= 1;
        if (bid >= nwg) {
            bid -= nwg;
            a.L0 = a.L1;
            a.R = a.R1;
            a.O0 = a.O1;
        }
    }
    // distinct objects, so that the compiler's wait for LDS DMA before a read
    // of one buffer does not count the loads still filling the others (the
    // buffers past ST are never referenced and take no LDS)
    __shared__ DmaSlice<BK> S0, S1, S2, S3;
    if (a.skip && *a.skip) return;   // uniform: a converged GMRES cycle

    constexpr bool UNF = EPI == EPI_UNFOLD;
    constexpr int T = BK / (2 * WAVES);   // row pairs per wave and operand in a slice
    constexpr int WJ = (WAVES == 4) ? 2 : 1, WCOLS = 16 * WJ;
    const int M = a.M, N = a.N, K = a.K;
    int tm, tn;
    tile_of(bid, nwg, M / BM, N / BN, tm, tn);   // (UNF: M/2 rows in tiles of 32)
    const int m0 = tm * (UNF ? BM / 2 : BM), n0 = tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave / (BN / WCOLS)) * 32, wn = (wave % (BN / WCOLS)) * WCOLS;
    const size_t ldl = UNF ? (size_t)(M / 2) : (size_t)M;

    // wave w fills slice rows 2T w .. 2T w + 2T - 1, two per instruction
    const int prow = 2 * T * wave;
    const double *lsrc[T], *rsrc[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int row = prow + 2 * t + (lane >> 5);
        const int col = (2 * (lane & 31)) ^ ((row & 1) << 4);   // swz() is an involution
        if (UNF)
            lsrc[t] = (col < 32 ? a.L0 : a.L1) + (size_t)row * ldl + m0 + (col & 31);
        else
            lsrc[t] = a.L0 + (size_t)row * ldl + m0 + col;
        rsrc[t] = a.R + (size_t)row * N + n0 + col;
    }
    const size_t lstep = BK * ldl, rstep = (size_t)BK * N;
    typedef const void __attribute__((address_space(1))) *gptr;
    typedef void __attribute__((address_space(3))) *lptr;
    auto issue = [&](DmaSlice<BK> &S, int kt) {
#pragma unroll
        for (int t = 0; t < T; ++t) {
            __builtin_amdgcn_global_load_lds((gptr)(lsrc[t] + kt * lstep),
                                             (lptr)&S.l[prow + 2 * t][0], 16, 0, 0);
            __builtin_amdgcn_global_load_lds((gptr)(rsrc[t] + kt * rstep),
                                             (lptr)&S.r[prow + 2 * t][0], 16, 0, 0);
        }
    };

    d4 acc[1][2][WJ];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < WJ; ++j) acc[0][i][j] = d4{0.0, 0.0, 0.0, 0.0};
    double af[2][2], bf[2][WJ];
    auto frag = [&](const DmaSlice<BK> &S, int k4, int slot) {
        const int kr = k4 * 4 + (lane >> 4);
#pragma unroll
        for (int i = 0; i < 2; ++i) af[slot][i] = S.l[kr][swz(kr, wm + i * 16 + (lane & 15))];
#pragma unroll
        for (int j = 0; j < WJ; ++j) bf[slot][j] = S.r[kr][swz(kr, wn + j * 16 + (lane & 15))];
    };
    auto compute = [&](const DmaSlice<BK> &S) {
        frag(S, 0, 0);
#pragma unroll
        for (int k4 = 0; k4 < BK / 4; ++k4) {
            if (k4 + 1 < BK / 4) frag(S, k4 + 1, (k4 + 1) & 1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < WJ; ++j)
                    acc[0][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[k4 & 1][i], bf[k4 & 1][j],
                                                                        acc[0][i][j], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    // s_waitcnt immediates (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt
    // and lgkmcnt left at their maxima)
    constexpr int kYounger = (ST - 2) * 2 * T;   // loads of the slices issued after the oldest
    static_assert(kYounger < 64, "vmcnt range");
    constexpr int kWaitVm = 0xF70 | (kYounger & 15) | ((kYounger >> 4) << 14), kWaitVm0 = 0xF70;
    const int nk = K / BK;
    const int last = nk - 1;
    auto step = [&](const DmaSlice<BK> &cur, DmaSlice<BK> &nxt, int kt) {
        // slice kt is this wave's oldest DMA, ST - 2 younger slices may still
        // be in flight; the barrier then publishes every wave's part
        __builtin_amdgcn_s_waitcnt(kWaitVm);
        asm volatile("s_barrier" ::: "memory");
        // past the end the last slice is loaded again (in bounds, never read),
        // which keeps the count of loads in flight the same at every step
        issue(nxt, min(kt + ST - 1, last));
        compute(cur);
    };
    if constexpr (ST == 4) {
        issue(S0, 0);
        issue(S1, 1);
        issue(S2, 2);
        for (int kt = 0; kt < nk; kt += 4) {
            step(S0, S3, kt);
            step(S1, S0, kt + 1);
            step(S2, S1, kt + 2);
            step(S3, S2, kt + 3);
        }
    } else {
        issue(S0, 0);
        for (int kt = 0; kt < nk; kt += 2) {
            step(S0, S1, kt);
            step(S1, S0, kt + 1);
        }
    }
    // no LDS DMA may outlive the workgroup
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    if constexpr (UNF) {
        // every wave's DMA has landed (S0 is free); B goes through S0.l
        asm volatile("s_barrier" ::: "memory");
        if (wm == 32) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < WJ; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        S0.l[i * 16 + (lane >> 4) + 4 * r][wn + j * 16 + (lane & 15)] = acc[0][i][j][r];
        }
        asm volatile("s_barrier" ::: "memory");
        if (wm == 0) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < WJ; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int p = m0 + i * 16 + (lane >> 4) + 4 * r;
                        const int c = wn + j * 16 + (lane & 15);
                        const double A = acc[0][i][j][r], Bv = S0.l[p - m0][c];
                        a.O0[(size_t)p * N + n0 + c] = A + Bv;
                        a.O0[(size_t)(M - 1 - p) * N + n0 + c] = A - Bv;
                    }
        }
    } else {
        store_tile<1, EPI, WJ>(a, acc, m0, n0, wm, wn, lane);
    }
}

}  // namespace

// 8 waves (two per SIMD), 32-deep K slices, fragments double-buffered: the
// fastest of the measured shapes (4 waves of 32 x 32; fragments read up front;
// 64-deep slices) at 1024^3 and 2048^3.
template <int NB, int EPI>
static void launch_variant(const GemmArgs &a, int tiles, hipStream_t s)
{
    hipLaunchKernelGGL((k_gemm_tn_f64<NB, EPI, 32, 8, false>), dim3(tiles), dim3(512), 0, s, a);
}

// direct-to-LDS launches: 32-deep slices in two buffers (64 KB of LDS), eight
// waves.  Measured at 1024^2 (application of the persymmetric literal form):
// 126.8 us with two 32-deep buffers, 126.6 us with two 64-deep, 129 us with
// four 32-deep; four waves of 32 x 32: 134.9 us (32-deep), 139 us (64-deep).
constexpr int kDmaBk = 32, kDmaSt = 2, kDmaKStep = kDmaBk * kDmaSt, kDmaWaves = 8;

bool gemm_unfold_fits(int M, int N, int K)
{
    // whole tiles (M/2 rows in 32-row tiles) and whole K slices of either kernel
    return M > 0 && N > 0 && M % BM == 0 && N % BN == 0 && K % kDmaKStep == 0 && K > 0;
}

hipError_t launch_gemm_f64(const GemmArgs &in, int epi, hipStream_t s)
{
    GemmArgs a = in;
    auto al16 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    a.vec = (a.M % 2 == 0) && (a.N % 2 == 0) && al16(a.L0) && al16(a.R) &&
            (a.L1 == nullptr || al16(a.L1)) && (!a.pair || al16(a.R1)) &&
            (a.ldo == 0 || a.ldo % 2 == 0);
    int tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
    const bool dual = a.L1 != nullptr && !a.pair;
    if (a.pair) {
        if (!a.L1 || !a.R1 || !a.O1 || epi != EPI_STORE) return hipErrorInvalidValue;
        tiles *= 2;
    }
    if (epi == EPI_PERMODE && !dual) return hipErrorInvalidValue;
    if (epi == EPI_UNFOLD) {
        if (!gemm_unfold_fits(a.M, a.N, a.K) || !a.vec || !a.L1 || a.pair || a.ldo)
            return hipErrorInvalidValue;
        if (tiles <= 256)
            hipLaunchKernelGGL((k_gemm_tn_f64_dma<EPI_UNFOLD, kDmaBk, kDmaSt, kDmaWaves>), dim3(tiles),
                               dim3(64 * kDmaWaves), 0, s, a);
        else
            hipLaunchKernelGGL((k_gemm_tn_f64<1, EPI_UNFOLD, 32, 8, false>), dim3(tiles), dim3(512), 0, s, a);
        return hipGetLastError();
    }
    // whole tiles, at most one tile per CU: the direct-to-LDS kernel (with
    // more tiles the register-staged kernel is as fast or faster: 2048^2
    // transforms at 80% of the FP64 matrix peak with it, 79% with two 32-deep
    // DMA buffers, 72% with four)
    const bool dma = !dual && a.vec && a.M % BM == 0 && a.N % BN == 0 && a.K % kDmaKStep == 0 &&
                     a.K > 0 && epi != EPI_PERMODE && tiles <= 256;
    if (dma) {
        if (epi == EPI_DIV_MU)
            hipLaunchKernelGGL((k_gemm_tn_f64_dma<EPI_DIV_MU, kDmaBk, kDmaSt, kDmaWaves>), dim3(tiles), dim3(64 * kDmaWaves), 0, s, a);
        else
            hipLaunchKernelGGL((k_gemm_tn_f64_dma<EPI_STORE, kDmaBk, kDmaSt, kDmaWaves>), dim3(tiles), dim3(64 * kDmaWaves), 0, s, a);
        return hipGetLastError();
    }
    if (dual) {
        if (epi == EPI_PERMODE) launch_variant<2, EPI_PERMODE>(a, tiles, s);
        else if (epi == EPI_STORE) launch_variant<2, EPI_STORE>(a, tiles, s);
        else return hipErrorInvalidValue;
    } else {
        if (epi == EPI_DIV_MU) launch_variant<1, EPI_DIV_MU>(a, tiles, s);
        else if (epi == EPI_STORE) launch_variant<1, EPI_STORE>(a, tiles, s);

        else return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mca
