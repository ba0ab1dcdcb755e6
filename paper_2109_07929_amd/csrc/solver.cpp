// solver.cpp -- C ABI, plan set-up and the Newton / flexible-GMRES control loop.
//
// The control flow is host code; every arithmetic step runs in the HIP kernels
// of kernels.hip and gemm.hip, including the Givens rotations and the small
// triangular solve of GMRES.  Within a GMRES cycle the host never stalls the
// GPU: it enqueues Arnoldi step j, then waits for the convergence flag of step
// j-1 (already computed on the device) while step j runs.  Once the flag is
// set, the kernels of the one step enqueued beyond it return immediately.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "mca_internal.h"

namespace mca {

namespace {
thread_local std::string g_last_error;

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Carves typed sub-buffers out of one caller-owned block (base may be null to
// only measure the size).
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count)
    {
        off = align_up(off);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t size() const { return align_up(off); }
};

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

mca_status validate_geometry(const mca_geometry *g)
{
    if (!g) return MCA_ERR_INVALID_ARG;
    if (g->m < 1 || g->n < 1 || g->reserved != 0) return MCA_ERR_INVALID_ARG;
    if ((size_t)g->m * (size_t)g->n > (size_t)1 << 30) return MCA_ERR_INVALID_ARG;
    if (g->device_model != MCA_DEVICE_SINH && g->device_model != MCA_DEVICE_LINEAR)
        return MCA_ERR_INVALID_ARG;
    const double c[] = {g->g_top, g->g_bot, g->g_src, g->g_top_end, g->g_bot_end0, g->g_bot_end1};
    for (double x : c)
        if (!finite_nonneg(x)) return MCA_ERR_INVALID_ARG;
    if (!(g->g_top > 0.0) || !(g->g_bot > 0.0)) return MCA_ERR_INVALID_ARG;
    if (!(g->g_src + g->g_top_end > 0.0) || !(g->g_bot_end0 + g->g_bot_end1 > 0.0))
        return MCA_ERR_INVALID_ARG;
    if (g->device_model == MCA_DEVICE_SINH && !(std::isfinite(g->v0) && g->v0 > 0.0))
        return MCA_ERR_INVALID_ARG;
    return MCA_OK;
}

mca_status validate_options(const mca_options *o)
{
    if (!(o->newton_tol >= 0.0) || !(o->gmres_tol > 0.0) || !(o->gmres_tol < 1.0))
        return MCA_ERR_INVALID_ARG;
    if (o->restart < 1 || o->restart > MCA_MAX_RESTART) return MCA_ERR_INVALID_ARG;
    if (o->max_newton < 1 || o->max_newton > MCA_MAX_NEWTON) return MCA_ERR_INVALID_ARG;
    if (o->max_krylov < 1) return MCA_ERR_INVALID_ARG;
    if (o->precision != MCA_PREC_FP64 && o->precision != MCA_PREC_FP32 &&
        o->precision != MCA_PREC_BF16X3 && o->precision != MCA_PREC_BF16)
        return MCA_ERR_INVALID_ARG;
    if (o->precond < MCA_PRECOND_LITERAL || o->precond > MCA_PRECOND_JACOBI)
        return MCA_ERR_INVALID_ARG;
    // reduced precision applies to the eigenbasis transforms of the per-mode form only
    if (o->precision != MCA_PREC_FP64 && o->precond != MCA_PRECOND_PERMODE &&
        o->precond != MCA_PRECOND_NONE)
        return MCA_ERR_INVALID_ARG;
    if (o->flags & ~(MCA_FLAG_INITIAL_GUESS | MCA_FLAG_TIMING | MCA_FLAG_GUESS_FALLBACK |
                     MCA_FLAG_SWEEP_START | MCA_FLAG_MGS_PASSES | MCA_FLAG_TIMING_SAMPLED))
        return MCA_ERR_INVALID_ARG;
    if ((o->flags & MCA_FLAG_INITIAL_GUESS) && (o->flags & MCA_FLAG_SWEEP_START))
        return MCA_ERR_INVALID_ARG;
    return MCA_OK;
}

// The approximate form holds whole wires in LDS.
bool approx_fits(const mca_plan *P) { return P->geom.m <= kTridiagMaxLen && P->geom.n <= kTridiagMaxLen; }

// The reduced-precision chain folds the Q_m-side products (half their depth)
// when G_bot is persymmetric and each half is a whole number of 128-row tiles.
bool lp_fold(const mca_plan *P) { return P->persym && (P->geom.m / 2) % 128 == 0; }

// Wire matrix of eq. (G) with the two end terminations (see mca.h).
Wire make_wire(int len, double g, double end0, double end1) { return Wire{g, end0, end1, len}; }

void wire_tridiag(const Wire &w, std::vector<double> &diag, std::vector<double> &off)
{
    diag.assign(w.len, 0.0);
    off.assign(w.len > 1 ? w.len - 1 : 0, 0.0);
    for (int k = 0; k + 1 < w.len; ++k) {
        diag[k] += w.g;
        diag[k + 1] += w.g;
        off[k] = -w.g;
    }
    diag[0] += w.end0;
    diag[w.len - 1] += w.end1;
}

// Layout of the plan's device block.
struct PlanLayout {
    double *Qm, *QmT, *Qn, *QnT, *lb, *lt;
    float *Qm32, *QmT32, *Qn32, *QnT32;
    uint16_t *QmH, *QmL, *QmTH, *QmTL, *QnH, *QnL, *QnTH, *QnTL;   // bfloat16 planes
    double *Us, *UsT, *Ua, *UaT, *lbp;                               // persymmetric halves
    // the folded reduced-precision chain's halves: [U_s^T; U_a^T], [U_s; U_a] (m x h)
    float *QmTf32, *Qmf32;
    uint16_t *QmTfH, *QmTfL, *QmfH, *QmfL;
    size_t bytes;
};

PlanLayout plan_layout(const mca_plan *P, void *base)
{
    const size_t m = P->geom.m, n = P->geom.n;
    Carver c(base);
    PlanLayout L;
    L.Qm = c.take<double>(m * m);
    L.QmT = c.take<double>(m * m);
    L.Qn = c.take<double>(n * n);
    L.QnT = c.take<double>(n * n);
    L.lb = c.take<double>(m);
    L.lt = c.take<double>(n);
    L.Qm32 = c.take<float>(m * m);
    L.QmT32 = c.take<float>(m * m);
    L.Qn32 = c.take<float>(n * n);
    L.QnT32 = c.take<float>(n * n);
    L.QmH = c.take<uint16_t>(m * m);
    L.QmL = c.take<uint16_t>(m * m);
    L.QmTH = c.take<uint16_t>(m * m);
    L.QmTL = c.take<uint16_t>(m * m);
    L.QnH = c.take<uint16_t>(n * n);
    L.QnL = c.take<uint16_t>(n * n);
    L.QnTH = c.take<uint16_t>(n * n);
    L.QnTL = c.take<uint16_t>(n * n);
    L.Us = L.UsT = L.Ua = L.UaT = L.lbp = nullptr;
    L.QmTf32 = L.Qmf32 = nullptr;
    L.QmTfH = L.QmTfL = L.QmfH = L.QmfL = nullptr;
    if (P->persym) {
        const size_t h = m / 2;
        L.Us = c.take<double>(h * h);
        L.UsT = c.take<double>(h * h);
        L.Ua = c.take<double>(h * h);
        L.UaT = c.take<double>(h * h);
        L.lbp = c.take<double>(m);
        L.QmTf32 = c.take<float>(m * h);
        L.Qmf32 = c.take<float>(m * h);
        L.QmTfH = c.take<uint16_t>(m * h);
        L.QmTfL = c.take<uint16_t>(m * h);
        L.QmfH = c.take<uint16_t>(m * h);
        L.QmfL = c.take<uint16_t>(m * h);
    }
    L.bytes = c.size();
    return L;
}

// Workspace of the preconditioner: up to four m x n FP64 buffers, or six
// m x n operands of 4 bytes per value (FP32, or two bfloat16 planes) in the
// reduced-precision modes.
struct PrecondWs {
    double *b0t, *b0b, *b1t, *b1b;
    LpPlanes lp[6];
    TridiagTables g1, g2;   // approximate form: G_top + a1 I (len n), G_bot + a2 I (len m)
};

PrecondWs precond_layout(const mca_plan *P, Carver &c, int form, int precision = MCA_PREC_FP64)
{
    const size_t mn = (size_t)P->geom.m * P->geom.n;
    PrecondWs w{};
    if (form == MCA_PRECOND_NONE || form == MCA_PRECOND_JACOBI) return w;
    if (form == MCA_PRECOND_LITERAL && precision == MCA_PREC_FP64 && P->persym) {
        w.b0t = c.take<double>(mn);
        w.b1t = c.take<double>(mn);
        w.b0b = c.take<double>(mn);   // the symmetric half of the inverse Q_m transform
        return w;
    }
    if (form == MCA_PRECOND_APPROX) {
        w.g1 = tridiag_carve(c.take<double>(tridiag_table_doubles(P->geom.n)), P->geom.n, P->top.g);
        w.g2 = tridiag_carve(c.take<double>(tridiag_table_doubles(P->geom.m)), P->geom.m, P->bot.g);
        return w;
    }
    if (precision != MCA_PREC_FP64) {
        for (auto &op : w.lp) {
            if (precision == MCA_PREC_FP32) {
                op.p[0] = c.take<float>(mn);
                op.p[1] = nullptr;
            } else {
                op.p[0] = c.take<uint16_t>(mn);
                op.p[1] = c.take<uint16_t>(mn);
            }
        }
        return w;
    }
    w.b0t = c.take<double>(mn);
    w.b1t = c.take<double>(mn);
    if (form == MCA_PRECOND_PERMODE) {
        w.b0b = c.take<double>(mn);
        w.b1b = c.take<double>(mn);
    }
    return w;
}

// Workspace of a solve.
struct SolveWs {
    double *V;        // (restart+1) Krylov vectors of length 2mn
    double *Z;        // restart preconditioned vectors
    double *X;        // Newton correction
    double *Vc, *Vn;  // current and trial iterate
    double *F, *Fn;   // residual at Vc / Vn
    double *D, *Dn;   // device slopes at Vc / Vn
    double *tmp;      // J X for restarts
    double *pa, *pb;  // per-block partial sums (ping-pong)
    double *pg1, *pg2;  // two-pass Gram-Schmidt partials (projections; update pass)
    double *Lg;       // strictly lower V^T V, row-major, ld = restart + 1
    double *sig;      // basis scales sig_q = 1 / ||u_q|| (two-pass form)
    double *H;        // Hessenberg, column-major, ld = restart + 1
    double *coef;     // least-squares solution y
    double *scal;     // reduced scalars
    double *nsc;      // Newton scalars on the device (launch_newton_next)
    double *g, *cs, *sn, *resid;   // Givens state of the current cycle
    int *ctl;         // cycle control block (stop flag, steps done, reason)
    PrecondWs pw;
    size_t bytes;
};

SolveWs solve_layout(const mca_plan *P, const mca_options *o, void *base)
{
    const size_t mn = (size_t)P->geom.m * P->geom.n, len = 2 * mn;
    const size_t R = o->restart;
    Carver c(base);
    SolveWs w;
    w.V = c.take<double>((R + 1) * len);
    w.Z = c.take<double>(R * len);
    w.X = c.take<double>(len);
    w.Vc = c.take<double>(len);
    w.Vn = c.take<double>(len);
    w.F = c.take<double>(len);
    w.Fn = c.take<double>(len);
    w.D = c.take<double>(mn);
    w.Dn = c.take<double>(mn);
    w.tmp = c.take<double>(len);
    w.pa = c.take<double>(4 * 1024);
    w.pb = c.take<double>(4 * 1024);
    w.pg1 = c.take<double>((size_t)kGsMaxV * kGsBlocks);
    w.pg2 = c.take<double>((size_t)(kGsMaxV + 1) * kGsBlocks);
    w.Lg = c.take<double>((R + 1) * (R + 1));
    w.sig = c.take<double>(R + 1);
    w.H = c.take<double>((R + 1) * R);
    w.coef = c.take<double>(R);
    w.scal = c.take<double>(8);
    w.nsc = c.take<double>(8);
    w.g = c.take<double>(R + 1);
    w.cs = c.take<double>(R);
    w.sn = c.take<double>(R);
    w.resid = c.take<double>(R);
    w.ctl = c.take<int>(4);
    w.pw = precond_layout(P, c, o->precond, o->precision);
    w.bytes = c.size();
    return w;
}

// Small pinned host staging area for the scalars read back per iteration, one
// per host thread, released when the thread ends.
struct PinnedScratch {
    double *buf = nullptr;
    double *dev = nullptr;   // the same words as the device addresses them
    ~PinnedScratch()
    {
        if (buf) (void)hipHostFree(buf);
    }
};

PinnedScratch *pinned()
{
    thread_local PinnedScratch ps;
    if (!ps.buf) {
        void *p = nullptr, *d = nullptr;
        if (hipHostMalloc(&p, 4096 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess)
            return nullptr;
        if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) {
            (void)hipHostFree(p);
            return nullptr;
        }
        ps.buf = static_cast<double *>(p);
        ps.dev = static_cast<double *>(d);
    }
    return &ps;
}

double *pinned_scratch()
{
    PinnedScratch *ps = pinned();
    return ps ? ps->buf : nullptr;
}

// device address of a pointer into the pinned scratch block
template <class T>
T *pinned_dev(T *host_ptr)
{
    PinnedScratch *ps = pinned();
    return reinterpret_cast<T *>(reinterpret_cast<char *>(ps->dev) +
                                 (reinterpret_cast<char *>(host_ptr) - reinterpret_cast<char *>(ps->buf)));
}

#define MCA_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) {                         \
            set_hip_error(#expr, e_);                   \
            return MCA_ERR_HIP;                         \
        }                                               \
    } while (0)

bool plan_ready(const mca_plan *P) { return P && P->dev_buf != nullptr; }

// Markers in pinned host memory: a kernel publishes data for the host (a
// snapshot, a reduced norm) and then stores a fresh marker value with release
// order at system scope; the host spins on the marker with acquire order.
// Unlike an event recorded between two kernels, this leaves no gap between
// them on the GPU.  Values come from a per-thread counter, so a marker left
// by an earlier wait never matches.
int next_epoch()
{
    thread_local unsigned counter = 0;
    ++counter;
    if ((int)counter == 0) ++counter;
    return (int)counter;
}

mca_status wait_marker(const int *mark, int epoch, hipStream_t s)
{
    // Only the marker is read for the first 20 ms: a stream query enqueues
    // work of its own, which delays the next kernel of the stream by a few
    // microseconds.  After that, every millisecond, the stream is asked
    // whether it still has work.
    using clock = std::chrono::steady_clock;
    const auto t0 = clock::now();
    auto next_check = t0 + std::chrono::milliseconds(20);
    for (unsigned spin = 1;; ++spin) {
        if (__atomic_load_n(mark, __ATOMIC_ACQUIRE) == epoch) return MCA_OK;
        __builtin_ia32_pause();
        if ((spin & 1023) == 0 && clock::now() >= next_check) {
            next_check = clock::now() + std::chrono::milliseconds(1);
            // a stream with no work left and no marker: the publishing kernel failed
            const hipError_t q = hipStreamQuery(s);
            if (q == hipSuccess) {
                if (__atomic_load_n(mark, __ATOMIC_ACQUIRE) == epoch) return MCA_OK;
                set_hip_error("marker wait: the stream drained without the marker",
                              hipErrorLaunchFailure);
                return MCA_ERR_HIP;
            }
            if (q != hipErrorNotReady) {
                set_hip_error("hipStreamQuery", q);
                return MCA_ERR_HIP;
            }
        }
    }
}

// GPU time per kernel class, from HIP events recorded around each group of
// launches.  Two slots alternate between consecutive Arnoldi steps (the host
// runs one step ahead); a slot is collected once its step has completed, and
// counted only if the step ran (a step skipped after convergence is not).
// Sampled mode: only the preconditioner class, every kSampleStride-th group.
struct Timing {
    static constexpr int kSlots = 2;
    static constexpr int kSampleStride = 4;
    bool on = false, sampled = false;
    unsigned gemm_groups = 0;
    hipEvent_t ev[kSlots][MCA_NUM_KCLASS][2] = {};
    bool active[kSlots][MCA_NUM_KCLASS] = {};
    int pending[kSlots][MCA_NUM_KCLASS] = {};
    double ms[MCA_NUM_KCLASS] = {};
    int launches[MCA_NUM_KCLASS] = {};

    hipError_t init(bool sample = false)
    {
        on = true;
        sampled = sample;
        for (auto &sl : ev)
            for (auto &c : sl)
                for (auto &e : c) {
                    hipError_t r = hipEventCreate(&e);
                    if (r != hipSuccess) return r;
                }
        return hipSuccess;
    }
    ~Timing()
    {
        for (auto &sl : ev)
            for (auto &c : sl)
                for (auto &e : c)
                    if (e) (void)hipEventDestroy(e);
    }
    hipError_t begin(int c, hipStream_t s, int slot = 0)
    {
        if (!on) return hipSuccess;
        bool take = true;
        if (sampled)
            take = c == MCA_KCLASS_GEMM && gemm_groups++ % kSampleStride == 0;
        active[slot][c] = take;
        return take ? hipEventRecord(ev[slot][c][0], s) : hipSuccess;
    }
    hipError_t end(int c, hipStream_t s, int nlaunch, int slot = 0)
    {
        if (!on || !active[slot][c]) return hipSuccess;
        active[slot][c] = false;
        pending[slot][c] = nlaunch;
        return hipEventRecord(ev[slot][c][1], s);
    }
    // after the events of `slot` have completed (only class `only` if >= 0)
    hipError_t collect(int slot = 0, bool count = true, int only = -1)
    {
        if (!on) return hipSuccess;
        for (int c = 0; c < MCA_NUM_KCLASS; ++c) {
            if (!pending[slot][c] || (only >= 0 && c != only)) continue;
            if (count) {
                float t = 0.f;
                hipError_t r = hipEventElapsedTime(&t, ev[slot][c][0], ev[slot][c][1]);
                if (r == hipErrorNotReady) {   // (seen through a marker, not yet by the runtime)
                    r = hipEventSynchronize(ev[slot][c][1]);
                    if (r == hipSuccess) r = hipEventElapsedTime(&t, ev[slot][c][0], ev[slot][c][1]);
                }
                if (r != hipSuccess) return r;
                ms[c] += t;
                launches[c] += pending[slot][c];
            }
            pending[slot][c] = 0;
        }
        return hipSuccess;
    }
};

// z = P^{-1} r (eq. (P)) in the chosen evaluation form.
// Per-shift set-up of the approximate form (the factorisations of
// G_top + a1 I and G_bot + a2 I); nothing for the other forms.
mca_status precond_setup(const mca_plan *P, int form, double a1, double a2, const PrecondWs &w,
                         hipStream_t s)
{
    if (form != MCA_PRECOND_APPROX) return MCA_OK;
    MCA_TRY(launch_tridiag_setup2(P->top, a1, w.g1, P->bot, a2, w.g2, s));
    return MCA_OK;
}

mca_status precond_run(const mca_plan *P, int form, int precision, double a1, double a2,
                       const double *rt, const double *rb, double *zt, double *zb,
                       const PrecondWs &w, hipStream_t s, Timing *tm = nullptr, int slot = 0,
                       const int *skip = nullptr, const double *D = nullptr, bool r_split = false,
                       bool defer_post = false, const GsStep *fin = nullptr,
                       hipEvent_t fin_done = nullptr, const double *shift = nullptr)
{
    // shift (persymmetric literal FP64 form only): a1 = a2 = shift[0] and
    // 1 / a1 = shift[1] are read on the device instead of a1, a2
    Timing off;
    if (!tm) tm = &off;
    // fin: the previous Arnoldi step's finish, launched with this application's
    // first kernel where that is the persymmetric fold, else on its own first;
    // fin_done is recorded right after it
    if (fin && !(form == MCA_PRECOND_LITERAL && precision == MCA_PREC_FP64 && P->persym)) {
        MCA_TRY(launch_gs_step(*fin, 2, s));
        if (fin_done) MCA_TRY(hipEventRecord(fin_done, s));
        fin = nullptr;
    }
    if (form == MCA_PRECOND_APPROX) {
        // the paper's M ~ Mhat (eqs. (Mhat)-(2matrix4)) as a block back-substitution:
        // z_b = (G_b + a2 I)^{-1} r_b down the columns, then
        // z_t = (G_t + a1 I)^{-1} (r_t + a1 z_b) along the rows
        const int m = P->geom.m, n = P->geom.n;
        MCA_TRY(tm->begin(MCA_KCLASS_GEMM, s, slot));
        MCA_TRY(launch_tridiag_solve(w.g2, n, false, 1, (size_t)n, rb, nullptr, 0.0, zb, skip, s));
        MCA_TRY(launch_tridiag_solve(w.g1, m, true, (size_t)n, 1, rt, zb, a1, zt, skip, s));
        MCA_TRY(tm->end(MCA_KCLASS_GEMM, s, 2, slot));
        return MCA_OK;
    }
    if (form == MCA_PRECOND_JACOBI) {
        MCA_TRY(tm->begin(MCA_KCLASS_GEMM, s, slot));
        MCA_TRY(launch_jacobi(P, D, rt, rb, zt, zb, skip, s));
        MCA_TRY(tm->end(MCA_KCLASS_GEMM, s, 1, slot));
        return MCA_OK;
    }
    if (form != MCA_PRECOND_NONE && precision != MCA_PREC_FP64) {
        const DevPlan &d = P->dev;
        LowPrecChain c{};
        c.m = P->geom.m;
        c.n = P->geom.n;
        c.a1 = a1;
        c.a2 = a2;
        c.skip = skip;
        auto planes = [](const void *a, const void *b) {
            LpPlanes p;
            p.p[0] = const_cast<void *>(a);
            p.p[1] = const_cast<void *>(b);
            return p;
        };
        if (precision == MCA_PREC_FP32) {
            c.QnT = planes(d.QnT32, nullptr); c.QmT = planes(d.QmT32, nullptr);
            c.Qm = planes(d.Qm32, nullptr); c.Qn = planes(d.Qn32, nullptr);
        } else {
            c.QnT = planes(d.QnTH, d.QnTL); c.QmT = planes(d.QmTH, d.QmTL);
            c.Qm = planes(d.QmH, d.QmL); c.Qn = planes(d.QnH, d.QnL);
        }
        c.lt = d.lt; c.lb = d.lb;
        c.fold = lp_fold(P) ? 1 : 0;
        if (c.fold) {
            if (precision == MCA_PREC_FP32) {
                c.QmTf = planes(d.QmTf32, nullptr); c.Qmf = planes(d.Qmf32, nullptr);
            } else {
                c.QmTf = planes(d.QmTfH, d.QmTfL); c.Qmf = planes(d.QmfH, d.QmfL);
            }
            c.lbp = d.lbp;
        }
        c.rt = rt; c.rb = rb;
        c.r_split = r_split ? 1 : 0;
        for (int b = 0; b < 2; ++b) {
            c.x[b] = w.lp[b];
            c.u[b] = w.lp[2 + b];
            c.w[b] = w.lp[4 + b];
        }
        c.zt = zt; c.zb = zb;
        MCA_TRY(tm->begin(MCA_KCLASS_GEMM, s, slot));
        MCA_TRY(launch_precond_lowprec(precision, c, s));
        MCA_TRY(tm->end(MCA_KCLASS_GEMM, s, r_split ? 4 : 5, slot));   // operand split + 4 products
        return MCA_OK;
    }
    const int m = P->geom.m, n = P->geom.n;
    const size_t mn = (size_t)m * n;
    const DevPlan &d = P->dev;
    if (form == MCA_PRECOND_NONE) {
        MCA_TRY(hipMemcpyAsync(zt, rt, mn * sizeof(double), hipMemcpyDeviceToDevice, s));
        MCA_TRY(hipMemcpyAsync(zb, rb, mn * sizeof(double), hipMemcpyDeviceToDevice, s));
        return MCA_OK;
    }
    GemmArgs g{};
    g.lb = d.lb;
    g.lt = d.lt;
    g.a1 = a1;
    g.a2 = a2;
    g.skip = skip;
    if (form == MCA_PRECOND_LITERAL && P->persym) {
        // G_bot persymmetric (m = 2h): every Q_m transform splits into a symmetric and
        // an antisymmetric half of h modes each, half the work of the full transform.
        const int h = m / 2;
        const size_t hn = (size_t)h * n;
        // P = w_top + J w_bot, Q = w_top - J w_bot with w = r_b + (G_b + a2 I) r_t / a1
        if (fin) {
            MCA_TRY(launch_finish_fold(*fin, P, a1, a2, rt, rb, w.b0t, s, skip, shift));
            if (fin_done) MCA_TRY(hipEventRecord(fin_done, s));
        } else if (shift) {
            MCA_TRY(launch_precond_pre_fold_dev(P, shift, rt, rb, w.b0t, s, skip));
        } else {
            MCA_TRY(launch_precond_pre_fold(P, a1, a2, rt, rb, w.b0t, s, skip));
        }
        g.shift = shift;
        MCA_TRY(tm->begin(MCA_KCLASS_GEMM, s, slot));
        // W_hat^T = [P^T U_s | Q^T U_a]   (n x m, modes: symmetric, antisymmetric; one launch)
        g.M = n; g.N = h; g.K = h; g.ldo = m; g.pair = 1;
        g.L0 = w.b0t; g.R = d.Us; g.O0 = w.b1t;
        g.L1 = w.b0t + hn; g.R1 = d.Ua; g.O1 = w.b1t + h;
        MCA_TRY(launch_gemm_f64(g, EPI_STORE, s));
        g.pair = 0; g.ldo = 0; g.L1 = nullptr; g.R1 = nullptr; g.O1 = nullptr;
        // X_hat = (W_hat Q_n) ./ mu        (m x n, rows in that mode order)
        g.M = m; g.N = n; g.K = n; g.lb = d.lbp;
        g.L0 = w.b1t; g.R = d.Qn; g.O0 = w.b0t;
        MCA_TRY(launch_gemm_f64(g, EPI_DIV_MU, s));
        g.lb = d.lb;
        // Y_s = X_hat_s^T U_s^T, Y_a = X_hat_a^T U_a^T   (n x h each; one launch)
        g.M = n; g.N = h; g.K = h; g.pair = 1;
        g.L0 = w.b0t; g.R = d.UsT; g.O0 = w.b0b;
        g.L1 = w.b0t + hn; g.R1 = d.UaT; g.O1 = w.b0b + hn;
        MCA_TRY(launch_gemm_f64(g, EPI_STORE, s));
        g.pair = 0; g.L1 = nullptr; g.R1 = nullptr; g.O1 = nullptr;
        int nl = 4;
        if (gemm_unfold_fits(m, n, n)) {
            // z_t = X Q_n^T with X^T = [Y_s + Y_a | mirrored (Y_s - Y_a)] formed
            // inside the product: rows i and m-1-i from the same tile
            g.M = m; g.N = n; g.K = n; g.L0 = w.b0b; g.L1 = w.b0b + hn; g.R = d.QnT; g.O0 = zt;
            MCA_TRY(launch_gemm_f64(g, EPI_UNFOLD, s));
            g.L1 = nullptr;
        } else {
            // X^T = [Y_s + Y_a | mirrored (Y_s - Y_a)]        (n x m)
            MCA_TRY(launch_unfold(w.b0b, w.b0b + hn, n, h, w.b1t, s, skip));
            // z_t = X Q_n^T                                   (m x n)
            g.M = m; g.N = n; g.K = n; g.L0 = w.b1t; g.R = d.QnT; g.O0 = zt;
            MCA_TRY(launch_gemm_f64(g, EPI_STORE, s));
            nl = 5;
        }
        MCA_TRY(tm->end(MCA_KCLASS_GEMM, s, nl, slot));
        // (deferred: the caller's Jacobian pass forms z_b)
        if (!defer_post) {
            if (shift) return MCA_ERR_INVALID_ARG;   // (not a combination the solver makes)
            MCA_TRY(launch_precond_post(P, a1, zt, rt, zb, s, skip));
        }
        return MCA_OK;
    }
    if (form == MCA_PRECOND_LITERAL) {
        // w = r_b + (G_b + a2 I) r_t / a1
        MCA_TRY(launch_precond_pre(P, a1, a2, rt, rb, w.b0t, s, skip));
        // (Q_m^T W)^T = W^T Q_m                      (n x m)
        MCA_TRY(tm->begin(MCA_KCLASS_GEMM, s, slot));
        g.M = n; g.N = m; g.K = m; g.L0 = w.b0t; g.L1 = nullptr; g.R = d.Qm; g.O0 = w.b1t;
        MCA_TRY(launch_gemm_f64(g, EPI_STORE, s));
        // W_hat = Q_m^T W Q_n, then ./ mu             (m x n)
        g.M = m; g.N = n; g.K = n; g.L0 = w.b1t; g.R = d.Qn; g.O0 = w.b0t;
        MCA_TRY(launch_gemm_f64(g, EPI_DIV_MU, s));
        // (Q_m X_hat)^T                               (n x m)
        g.M = n; g.N = m; g.K = m; g.L0 = w.b0t; g.R = d.QmT; g.O0 = w.b1t;
        MCA_TRY(launch_gemm_f64(g, EPI_STORE, s));
        // z_t = Q_m X_hat Q_n^T                       (m x n)
        g.M = m; g.N = n; g.K = n; g.L0 = w.b1t; g.R = d.QnT; g.O0 = zt;
        MCA_TRY(launch_gemm_f64(g, EPI_STORE, s));
        MCA_TRY(tm->end(MCA_KCLASS_GEMM, s, 4, slot));
        // z_b = ((G_t + a1 I) z_t - r_t) / a1 (deferred: the caller's Jacobian pass forms it)
        if (!defer_post) MCA_TRY(launch_precond_post(P, a1, zt, rt, zb, s, skip));
        return MCA_OK;
    }
    // per-mode: transform both layers, solve each mode's 2x2 block, transform back
    MCA_TRY(tm->begin(MCA_KCLASS_GEMM, s, slot));
    g.M = n; g.N = m; g.K = m; g.L0 = rt; g.L1 = rb; g.R = d.Qm; g.O0 = w.b1t; g.O1 = w.b1b;
    MCA_TRY(launch_gemm_f64(g, EPI_STORE, s));
    g.M = m; g.N = n; g.K = n; g.L0 = w.b1t; g.L1 = w.b1b; g.R = d.Qn; g.O0 = w.b0t; g.O1 = w.b0b;
    MCA_TRY(launch_gemm_f64(g, EPI_PERMODE, s));
    g.M = n; g.N = m; g.K = m; g.L0 = w.b0t; g.L1 = w.b0b; g.R = d.QmT; g.O0 = w.b1t; g.O1 = w.b1b;
    MCA_TRY(launch_gemm_f64(g, EPI_STORE, s));
    g.M = m; g.N = n; g.K = n; g.L0 = w.b1t; g.L1 = w.b1b; g.R = d.QnT; g.O0 = zt; g.O1 = zb;
    MCA_TRY(launch_gemm_f64(g, EPI_STORE, s));
    MCA_TRY(tm->end(MCA_KCLASS_GEMM, s, 4, slot));
    return MCA_OK;
}

// Flexible GMRES(restart) with modified Gram-Schmidt for J X = -F, right
// preconditioned by P(a, a), for one Newton step.  On return X holds the
// correction.  Gram-Schmidt runs in two passes per Arnoldi step (compact WY
// form) when restart <= 32 and MCA_FLAG_MGS_PASSES is not set, else in one
// pass per basis vector.
//
// start() enqueues the Newton scalars of F (launch_newton_next: the shift a,
// ||F||, the GMRES stop) and v_0 = -F / ||F||; step(j) enqueues Arnoldi step
// j; run() enqueues the rest and drives the cycles.  The two calls before
// run() may come before the host knows F's norm: the Newton loop enqueues
// them behind a trial point's residual, gated on the device by the trial's
// acceptance, so the GPU goes on into the next Newton step while the host
// reads the trial's norm.  In the persymmetric literal FP64 form the kernels
// take the shift and the stop from the device scalars (the form in which the
// start is enqueued ahead); the other forms take the host's values.
struct Fgmres {
    const mca_plan *P;
    const mca_options *o;
    SolveWs w;
    hipStream_t s;
    Timing *tm;
    size_t mn, len;
    int R, ldh;
    bool two_pass, lp_fused, post_fused, merge_fin;
    static constexpr int kSnapInts = 8;   // ints per step's snapshot slot (marker at [4])
    double *host = nullptr;
    int *snap = nullptr, *snap_dev = nullptr;
    int epoch[MCA_MAX_RESTART] = {};
    GsStep gs{}, fin{};
    bool fin_pending = false;
    double a = 0.0;          // host shift (forms without the device shift)
    double fnorm_host = 0.0; // ||F|| as the host has it (set by run)
    int enqueued = 0;        // Arnoldi steps of the first cycle already enqueued

    Fgmres(const mca_plan *P_, const mca_options *o_, const SolveWs &w_, hipStream_t s_, Timing *tm_)
        : P(P_), o(o_), w(w_), s(s_), tm(tm_)
    {
        mn = (size_t)P->geom.m * P->geom.n;
        len = 2 * mn;
        R = o->restart;
        ldh = R + 1;
        two_pass = !(o->flags & MCA_FLAG_MGS_PASSES) && R <= kGsMaxV;
        // the reduced-precision per-mode chain: the update pass converts the new
        // vector into the chain's operand planes itself (for the folded chain,
        // with its rows i and m - 1 - i folded)
        lp_fused = two_pass && o->precond == MCA_PRECOND_PERMODE && o->precision != MCA_PREC_FP64;
        // the literal form's last step (z_b from z_t) runs inside the Jacobian pass
        post_fused = two_pass && o->precond == MCA_PRECOND_LITERAL && o->precision == MCA_PREC_FP64;
        // persymmetric literal form: step j's finish shares a launch with step j + 1's
        // first stencil (the finish of the cycle's last enqueued step runs alone)
        merge_fin = post_fused && P->persym;
        host = pinned_scratch();
        if (host) {
            snap = reinterpret_cast<int *>(host + 256);
            snap_dev = pinned_dev(snap);
        }
        gs.m = P->geom.m;
        gs.n = P->geom.n;
        gs.top = P->top;
        gs.bot = P->bot;
        gs.d = w.D;
        gs.V = w.V;
        gs.ldv = len;
        gs.sig = w.sig;
        gs.L = w.Lg;
        gs.ldl = R + 1;
        gs.H = w.H;
        gs.ldh = ldh;
        gs.p1 = w.pg1;
        gs.p2 = w.pg2;
        gs.g = w.g;
        gs.cs = w.cs;
        gs.sn = w.sn;
        gs.resid = w.resid;
        gs.ctl = w.ctl;
        gs.tol = w.nsc + 4;
        if (lp_fused) {
            for (int b = 0; b < 2; ++b)
                for (int pl = 0; pl < 2; ++pl) gs.xp[b][pl] = w.pw.lp[b].p[pl];
            gs.prec = o->precision;
            gs.fold_h = lp_fold(P) ? P->geom.m / 2 : 0;
        }
        if (merge_fin) gs.shift = w.nsc;
    }

    // whether the kernels of this form read the shift from the device
    bool device_shift() const { return merge_fin; }

    // Newton scalars of F from its reduced sums (device address; ||F||^2,
    // sum D), the first cycle's start (gated by accept2 / conv2, see
    // launch_newton_next) and v_0 = -F / ||F||.
    mca_status start(const double *sums_dev, double accept2, double conv2)
    {
        if (!host) {
            set_hip_error("hipHostMalloc", hipErrorOutOfMemory);
            return MCA_ERR_HIP;
        }
        MCA_TRY(launch_newton_next(sums_dev, (double)mn, o->gmres_tol, accept2, conv2, w.nsc, w.ctl,
                                   w.g, R, two_pass ? w.sig : nullptr, s));
        MCA_TRY(launch_scale_dev(w.F, w.nsc + 3, w.V, len, s));
        return MCA_OK;
    }

    // Arnoldi step j of the current cycle
    mca_status step(int j)
    {
        const int slot = j & 1;
        double *vj = w.V + (size_t)j * len, *zj = w.Z + (size_t)j * len;
        double *wv = w.V + (size_t)(j + 1) * len;
        const int *skip = w.ctl;
        // (the previous step's update pass left v_j in operand format)
        mca_status st = precond_run(P, o->precond, o->precision, a, a, vj, vj + mn, zj, zj + mn,
                                    w.pw, s, tm, slot, skip, w.D, lp_fused && j > 0, post_fused,
                                    fin_pending ? &fin : nullptr, nullptr,
                                    device_shift() ? w.nsc : nullptr);
        fin_pending = false;
        if (st != MCA_OK) return st;
        double *hcol = w.H + (size_t)j * ldh;
        if (two_pass) {
            // w = sig_j J z~_j fused with the projections on the basis and
            // MGS's coefficients, then w -= V h with the Givens update
            gs.j = j;
            gs.zt = zj;
            gs.zb = zj + mn;
            if (post_fused) {
                gs.post_rt = vj;
                gs.zb_store = zj + mn;
                gs.post_a1 = a;
                gs.post_inv_a1 = device_shift() ? 0.0 : 1.0 / a;
            }
            gs.w = wv;
            gs.hcol = hcol;
            gs.snap = snap_dev + kSnapInts * j;
            gs.epoch = epoch[j] = next_epoch();
            MCA_TRY(tm->begin(MCA_KCLASS_JACOBIAN, s, slot));
            MCA_TRY(launch_gs_step(gs, 0, s));
            MCA_TRY(tm->end(MCA_KCLASS_JACOBIAN, s, 1, slot));
            MCA_TRY(tm->begin(MCA_KCLASS_ORTHO, s, slot));
            MCA_TRY(launch_gs_step(gs, 1, s));
            MCA_TRY(tm->end(MCA_KCLASS_ORTHO, s, j + 1 <= kGsFusedMaxV ? 1 : 2, slot));
            if (merge_fin) {
                fin = gs;
                fin_pending = true;
            } else {
                MCA_TRY(launch_gs_step(gs, 2, s));
            }
        } else {
            // w = J z_j, fused with the partial sums of <w, v_0>
            MCA_TRY(tm->begin(MCA_KCLASS_JACOBIAN, s, slot));
            MCA_TRY(launch_jacobian(P, w.D, zj, zj + mn, wv, wv + mn, s, w.V, w.pa, skip));
            MCA_TRY(tm->end(MCA_KCLASS_JACOBIAN, s, 1, slot));
            // modified Gram-Schmidt, one pass per basis vector:
            // h_ij = <w, v_i>, w -= h_ij v_i, i = 0..j
            MCA_TRY(tm->begin(MCA_KCLASS_ORTHO, s, slot));
            double *pin = w.pa, *pout = w.pb;
            for (int i = 0; i <= j; ++i) {
                const double *vnext = (i < j) ? w.V + (size_t)(i + 1) * len : nullptr;
                MCA_TRY(launch_mgs_step(wv, w.V + (size_t)i * len, vnext, len, pin, pout, hcol + i,
                                        s, skip));
                std::swap(pin, pout);
            }
            MCA_TRY(launch_normalize(wv, len, pin, hcol + j + 1, s, skip));
            MCA_TRY(tm->end(MCA_KCLASS_ORTHO, s, j + 2, slot));
            epoch[j] = next_epoch();
            MCA_TRY(launch_givens(w.H, ldh, j, w.g, w.cs, w.sn, o->gmres_tol * fnorm_host, w.ctl,
                                  w.resid, snap_dev + kSnapInts * j, epoch[j], s));
        }
        return MCA_OK;
    }

    // a first step enqueued ahead that the host does not take: its timing slot
    // is dropped (its kernels return at once on the gated stop flag)
    mca_status abandon()
    {
        if (enqueued > 0) MCA_TRY(tm->collect(0, false));
        enqueued = 0;
        fin_pending = false;
        return MCA_OK;
    }

    // step 0 enqueued ahead of run()
    mca_status prelaunch_first_step()
    {
        const mca_status st = step(0);
        if (st == MCA_OK) enqueued = 1;
        return st;
    }

    // The GMRES solve from F with ||F|| = fnorm and shift a (host values),
    // after start() (and possibly step(0)) were enqueued.
    mca_status run(double fnorm, double a_host, int *its_out, int *restarts_out, bool *conv_out)
    {
        a = a_host;
        fnorm_host = fnorm;
        double beta = fnorm;
        const double abs_tol = o->gmres_tol * fnorm;
        if (!device_shift()) {
            const mca_status st = precond_setup(P, o->precond, a, a, w.pw, s);
            if (st != MCA_OK) return st;
        }
        int its = 0, restarts = 0;
        bool converged = false, first = true, cycle_started = true;
        for (;;) {
            if (!cycle_started)
                MCA_TRY(launch_cycle_init(w.ctl, w.g, R, beta, s, two_pass ? w.sig : nullptr));
            cycle_started = false;
            const int jmax = std::min(R, o->max_krylov - its);
            const int j0 = std::min(enqueued, jmax);
            enqueued = 0;
            int last = j0 - 1, stopped_at = -1;
            for (int j = j0; j < jmax; ++j) {
                const mca_status st = step(j);
                if (st != MCA_OK) return st;
                last = j;
                if (j > 0) {
                    // step j runs on the GPU while the host reads step j-1's outcome
                    // (step j-1's snapshot is written by its finish, which with the
                    // finish merged runs in step j's first launch)
                    const int *c = snap + kSnapInts * (j - 1);
                    const mca_status ws = wait_marker(c + 4, epoch[j - 1], s);
                    if (ws != MCA_OK) return ws;
                    MCA_TRY(tm->collect((j - 1) & 1, c[1] == j));
                    if (c[0]) {
                        // the cycle stopped at step j - 1: step j, already enqueued,
                        // returns at once (its timing slot is dropped); the update
                        // below needs no further wait
                        stopped_at = j - 1;
                        break;
                    }
                }
            }
            if (fin_pending) {   // the last enqueued step's finish, alone
                MCA_TRY(launch_gs_step(fin, 2, s));
                fin_pending = false;
            }
            const int *c = nullptr;
            if (stopped_at >= 0) {
                c = snap + kSnapInts * stopped_at;
                MCA_TRY(tm->collect(last & 1, false));
            } else if (last >= 0) {
                c = snap + kSnapInts * last;
                const mca_status ws = wait_marker(c + 4, epoch[last], s);
                if (ws != MCA_OK) return ws;
                MCA_TRY(tm->collect(last & 1, c[1] == last + 1));
            }
            const int k = c ? c[1] : 0;
            const int reason = c ? c[2] : CYCLE_RUNNING;
            if (reason == CYCLE_NONFINITE) return MCA_ERR_NONFINITE;
            its += k;
            if (k > 0) {
                MCA_TRY(launch_backsolve(w.H, ldh, w.g, w.ctl, w.coef, s, two_pass ? w.sig : nullptr));
                // the number of completed steps is ctl[1]
                MCA_TRY(launch_update(w.Z, len, w.coef, 0, w.ctl + 1, len, w.X, first ? 0 : 1, s));
                first = false;
            } else if (first) {
                MCA_TRY(launch_fill(w.X, 0.0, len, s));
                first = false;
            }
            converged = reason == CYCLE_CONVERGED;
            if (converged || its >= o->max_krylov || reason == CYCLE_BREAKDOWN || k == 0) break;
            // restart from the true residual  r = -F - J X
            ++restarts;
            MCA_TRY(tm->begin(MCA_KCLASS_JACOBIAN, s));
            MCA_TRY(launch_jacobian(P, w.D, w.X, w.X + mn, w.tmp, w.tmp + mn, s));
            MCA_TRY(tm->end(MCA_KCLASS_JACOBIAN, s, 1));
            MCA_TRY(launch_neg_sum(w.F, w.tmp, w.V, len, s));
            MCA_TRY(launch_dot_partials(w.V, w.V, len, w.pa, s));
            MCA_TRY(launch_reduce(w.pa, reduce_blocks(len), 1, w.scal, s));
            MCA_TRY(hipMemcpyAsync(host, w.scal, sizeof(double), hipMemcpyDeviceToHost, s));
            MCA_TRY(hipStreamSynchronize(s));
            MCA_TRY(tm->collect());
            beta = std::sqrt(host[0]);
            if (!std::isfinite(beta)) return MCA_ERR_NONFINITE;
            if (beta <= abs_tol) {
                converged = true;
                break;
            }
            MCA_TRY(launch_scale(w.V, 1.0 / beta, w.V, len, s));
        }
        *its_out = its;
        *restarts_out = restarts;
        *conv_out = converged;
        return MCA_OK;
    }
};

// Residual at (vt, vb) into F/D: residual_enqueue launches it and its reduction
// into host words 0 and 1 (||F||^2, sum D) with a marker (host word 4 as ints);
// residual_wait returns ||F||, ||F||^2 and sum D on the host once they are there.
mca_status residual_enqueue(const mca_plan *P, const double *g_dev, const double *v_in,
                            const double *vt, const double *vb, double *F, double *D,
                            const SolveWs &w, hipStream_t s, Timing *tm, int *epoch)
{
    const size_t mn = (size_t)P->geom.m * P->geom.n;
    double *host = pinned_scratch();
    if (!host) {
        set_hip_error("hipHostMalloc", hipErrorOutOfMemory);
        return MCA_ERR_HIP;
    }
    double *host_dev = pinned_dev(host);   // the same pinned words, as the device sees them
    MCA_TRY(tm->begin(MCA_KCLASS_RESIDUAL, s));
    MCA_TRY(launch_residual(P, g_dev, v_in, vt, vb, F, F + mn, D, w.pa, s));
    MCA_TRY(tm->end(MCA_KCLASS_RESIDUAL, s, 1));
    *epoch = next_epoch();
    MCA_TRY(launch_reduce(w.pa, reduce_blocks(mn), 2, host_dev, s,
                          reinterpret_cast<int *>(host_dev + 4), *epoch));
    return MCA_OK;
}

mca_status residual_wait(int epoch, hipStream_t s, Timing *tm, double *fnorm, double *fnorm2,
                         double *dsum)
{
    double *host = pinned_scratch();
    const mca_status ws = wait_marker(reinterpret_cast<int *>(host + 4), epoch, s);
    if (ws != MCA_OK) return ws;
    MCA_TRY(tm->collect(0, true, MCA_KCLASS_RESIDUAL));
    *fnorm2 = host[0];
    *fnorm = std::sqrt(host[0]);
    *dsum = host[1];
    if (!std::isfinite(*fnorm) || !std::isfinite(*dsum)) return MCA_ERR_NONFINITE;
    return MCA_OK;
}

mca_status residual_norms(const mca_plan *P, const double *g_dev, const double *v_in,
                          const double *vt, const double *vb, double *F, double *D,
                          const SolveWs &w, hipStream_t s, Timing *tm, double *fnorm,
                          double *fnorm2, double *dsum)
{
    int e = 0;
    const mca_status st = residual_enqueue(P, g_dev, v_in, vt, vb, F, D, w, s, tm, &e);
    if (st != MCA_OK) return st;
    return residual_wait(e, s, tm, fnorm, fnorm2, dsum);
}

// Workspace of mca_precond_apply_noalloc: one array per GPU, held by the code
// object for the life of the process.  Host code never passes `scratch` itself
// to a kernel (its host-side name is not the device address): the address
// comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoAllocBytes = (size_t)MCA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's scratch array (looked up on first use).
mca_status noalloc_scratch(void **out)
{
    int dev = -1;
    MCA_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return MCA_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        MCA_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return MCA_ERR_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MCA_OK;
}

}  // namespace

void set_hip_error(const char *what, hipError_t e)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
}

mca_status wait_flag64(const long long *slot, hipStream_t s, int *value)
{
    // as wait_marker: the stream is queried only after 20 ms without the flag
    using clock = std::chrono::steady_clock;
    auto next_check = clock::now() + std::chrono::milliseconds(20);
    for (unsigned spin = 1;; ++spin) {
        const long long v = __atomic_load_n(slot, __ATOMIC_ACQUIRE);
        if ((v >> 32) == 1) {
            *value = (int)(v & 0xffffffffLL);
            return MCA_OK;
        }
        __builtin_ia32_pause();
        if ((spin & 1023) == 0 && clock::now() >= next_check) {
            next_check = clock::now() + std::chrono::milliseconds(1);
            const hipError_t q = hipStreamQuery(s);
            if (q == hipSuccess) {
                const long long w = __atomic_load_n(slot, __ATOMIC_ACQUIRE);
                if ((w >> 32) == 1) {
                    *value = (int)(w & 0xffffffffLL);
                    return MCA_OK;
                }
                set_hip_error("flag wait: the stream drained without the flag", hipErrorLaunchFailure);
                return MCA_ERR_HIP;
            }
            if (q != hipErrorNotReady) {
                set_hip_error("hipStreamQuery", q);
                return MCA_ERR_HIP;
            }
        }
    }
}

}  // namespace mca

using namespace mca;

extern "C" {

void mca_options_default(mca_options *o)
{
    if (!o) return;
    o->newton_tol = 1e-10;
    o->gmres_tol = 1e-8;
    o->restart = 30;
    o->max_newton = 50;
    o->max_krylov = 600;
    o->precision = MCA_PREC_FP64;
    o->precond = MCA_PRECOND_LITERAL;
    o->flags = 0;
}

const char *mca_status_string(mca_status s)
{
    switch (s) {
    case MCA_OK: return "ok";
    case MCA_ERR_INVALID_ARG: return "invalid argument";
    case MCA_ERR_NONFINITE: return "non-finite value";
    case MCA_ERR_WORKSPACE: return "workspace too small or plan not uploaded";
    case MCA_ERR_NOT_CONVERGED: return "not converged";
    case MCA_ERR_BREAKDOWN: return "GMRES breakdown";
    case MCA_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

const char *mca_last_error(void) { return g_last_error.c_str(); }

size_t mca_abi_struct_size(int32_t which)
{
    switch (which) {
    case 0: return sizeof(mca_geometry);
    case 1: return sizeof(mca_options);
    case 2: return sizeof(mca_stats);
    default: return 0;
    }
}

mca_status mca_plan_create(const mca_geometry *geom, mca_plan **out)
{
    if (!out) return MCA_ERR_INVALID_ARG;
    *out = nullptr;
    mca_status st = validate_geometry(geom);
    if (st != MCA_OK) return st;
    mca_plan *P = new (std::nothrow) mca_plan();
    if (!P) return MCA_ERR_INVALID_ARG;
    P->geom = *geom;
    P->top = make_wire(geom->n, geom->g_top, geom->g_src, geom->g_top_end);
    P->bot = make_wire(geom->m, geom->g_bot, geom->g_bot_end0, geom->g_bot_end1);
    const int m = geom->m, n = geom->n;
    // the top wire's problem on a thread of its own, beside the bottom wire's
    P->lt.resize(n);
    P->Qn.resize((size_t)n * n);
    auto top_job = [P, n] {
        std::vector<double> d, o;
        wire_tridiag(P->top, d, o);
        tridiag_eigen(n, d.data(), o.data(), P->lt.data(), P->Qn.data());
    };
    std::thread top_th;
    try {
        top_th = std::thread(top_job);
    } catch (...) {   // no thread to be had: run it here
        top_job();
    }
    std::vector<double> diag, off;
    P->lb.resize(m);
    P->Qm.resize((size_t)m * m);
    wire_tridiag(P->bot, diag, off);
    // persymmetric G_bot: the symmetric / antisymmetric eigenvectors [u; +-J u]/sqrt2
    // come from two h x h problems, the last diagonal entry shifted by -+ the
    // coupling of the two middle nodes; the full basis Q_m is assembled from
    // them (eigenvalues merged in ascending order)
    P->persym = (m >= 2) && (m % 2 == 0) && (geom->g_bot_end0 == geom->g_bot_end1);
    if (P->persym) {
        const int h = m / 2;
        std::vector<double> dh(diag.begin(), diag.begin() + h), oh(off.begin(), off.begin() + (h - 1));
        const double cpl = off[h - 1];
        const double r2 = 1.0 / std::sqrt(2.0);
        for (int sign = 0; sign < 2; ++sign) {
            std::vector<double> dd = dh, lam(h), Q((size_t)h * h);
            dd[h - 1] += (sign == 0) ? cpl : -cpl;
            tridiag_eigen(h, dd.data(), oh.data(), lam.data(), Q.data());
            for (double &x : Q) x *= r2;
            (sign == 0 ? P->Us : P->Ua) = Q;
            (sign == 0 ? P->ls : P->la) = lam;
        }
        int is = 0, ia = 0;
        for (int col = 0; col < m; ++col) {
            const bool sym = ia >= h || (is < h && P->ls[is] <= P->la[ia]);
            const std::vector<double> &Q = sym ? P->Us : P->Ua;
            const int s = sym ? is++ : ia++;
            P->lb[col] = sym ? P->ls[s] : P->la[s];
            for (int i = 0; i < h; ++i) {
                const double v = Q[(size_t)i * h + s];
                P->Qm[(size_t)i * m + col] = v;
                P->Qm[(size_t)(m - 1 - i) * m + col] = sym ? v : -v;
            }
        }
    } else {
        tridiag_eigen(m, diag.data(), off.data(), P->lb.data(), P->Qm.data());
    }
    if (top_th.joinable()) top_th.join();
    P->dev_bytes = plan_layout(P, nullptr).bytes;
    *out = P;
    return MCA_OK;
}

void mca_plan_destroy(mca_plan *P) { delete P; }

size_t mca_plan_device_bytes(const mca_plan *P) { return P ? P->dev_bytes : 0; }

mca_status mca_plan_host_eigen(const mca_plan *P, int32_t layer, double *lambda, double *q)
{
    if (!P || (layer != 0 && layer != 1)) return MCA_ERR_INVALID_ARG;
    const std::vector<double> &lam = layer == 0 ? P->lt : P->lb;
    const std::vector<double> &Q = layer == 0 ? P->Qn : P->Qm;
    if (lambda) std::memcpy(lambda, lam.data(), lam.size() * sizeof(double));
    if (q) std::memcpy(q, Q.data(), Q.size() * sizeof(double));
    return MCA_OK;
}

mca_status mca_plan_upload(mca_plan *P, void *dev_buf, size_t bytes, void *stream)
{
    if (!P || !dev_buf) return MCA_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(dev_buf) % kAlign) return MCA_ERR_INVALID_ARG;
    if (bytes < P->dev_bytes) return MCA_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t m = P->geom.m, n = P->geom.n;
    // host image of the whole block (same offsets), then one copy
    std::vector<char> img(P->dev_bytes);
    PlanLayout H = plan_layout(P, img.data());
    for (size_t i = 0; i < m; ++i)
        for (size_t p = 0; p < m; ++p) {
            H.Qm[i * m + p] = P->Qm[i * m + p];
            H.QmT[p * m + i] = P->Qm[i * m + p];
        }
    for (size_t j = 0; j < n; ++j)
        for (size_t q = 0; q < n; ++q) {
            H.Qn[j * n + q] = P->Qn[j * n + q];
            H.QnT[q * n + j] = P->Qn[j * n + q];
        }
    std::memcpy(H.lb, P->lb.data(), m * sizeof(double));
    std::memcpy(H.lt, P->lt.data(), n * sizeof(double));
    split_host(H.Qm, m * m, MCA_PREC_FP32, H.Qm32, nullptr);
    split_host(H.QmT, m * m, MCA_PREC_FP32, H.QmT32, nullptr);
    split_host(H.Qn, n * n, MCA_PREC_FP32, H.Qn32, nullptr);
    split_host(H.QnT, n * n, MCA_PREC_FP32, H.QnT32, nullptr);
    split_host(H.Qm, m * m, MCA_PREC_BF16X3, H.QmH, H.QmL);
    split_host(H.QmT, m * m, MCA_PREC_BF16X3, H.QmTH, H.QmTL);
    split_host(H.Qn, n * n, MCA_PREC_BF16X3, H.QnH, H.QnL);
    split_host(H.QnT, n * n, MCA_PREC_BF16X3, H.QnTH, H.QnTL);
    if (P->persym) {
        const size_t h = m / 2;
        for (size_t i = 0; i < h; ++i)
            for (size_t k = 0; k < h; ++k) {
                H.Us[i * h + k] = P->Us[i * h + k];
                H.UsT[k * h + i] = P->Us[i * h + k];
                H.Ua[i * h + k] = P->Ua[i * h + k];
                H.UaT[k * h + i] = P->Ua[i * h + k];
            }
        std::memcpy(H.lbp, P->ls.data(), h * sizeof(double));
        std::memcpy(H.lbp + h, P->la.data(), h * sizeof(double));
        std::vector<double> qtf(m * h), qf(m * h);
        std::memcpy(qtf.data(), H.UsT, h * h * sizeof(double));
        std::memcpy(qtf.data() + h * h, H.UaT, h * h * sizeof(double));
        std::memcpy(qf.data(), H.Us, h * h * sizeof(double));
        std::memcpy(qf.data() + h * h, H.Ua, h * h * sizeof(double));
        split_host(qtf.data(), m * h, MCA_PREC_FP32, H.QmTf32, nullptr);
        split_host(qf.data(), m * h, MCA_PREC_FP32, H.Qmf32, nullptr);
        split_host(qtf.data(), m * h, MCA_PREC_BF16X3, H.QmTfH, H.QmTfL);
        split_host(qf.data(), m * h, MCA_PREC_BF16X3, H.QmfH, H.QmfL);
    }
    MCA_TRY(hipMemcpyAsync(dev_buf, img.data(), P->dev_bytes, hipMemcpyHostToDevice, s));
    MCA_TRY(hipStreamSynchronize(s));
    PlanLayout L = plan_layout(P, dev_buf);
    P->dev_buf = dev_buf;
    P->dev = DevPlan{};
    P->dev.Qm = L.Qm;
    P->dev.QmT = L.QmT;
    P->dev.Qn = L.Qn;
    P->dev.QnT = L.QnT;
    P->dev.lb = L.lb;
    P->dev.lt = L.lt;
    P->dev.Qm32 = L.Qm32;
    P->dev.QmT32 = L.QmT32;
    P->dev.Qn32 = L.Qn32;
    P->dev.QnT32 = L.QnT32;
    P->dev.QmH = L.QmH; P->dev.QmL = L.QmL; P->dev.QmTH = L.QmTH; P->dev.QmTL = L.QmTL;
    P->dev.QnH = L.QnH; P->dev.QnL = L.QnL; P->dev.QnTH = L.QnTH; P->dev.QnTL = L.QnTL;
    P->dev.Us = L.Us; P->dev.UsT = L.UsT; P->dev.Ua = L.Ua; P->dev.UaT = L.UaT;
    P->dev.lbp = L.lbp;
    P->dev.QmTf32 = L.QmTf32; P->dev.Qmf32 = L.Qmf32;
    P->dev.QmTfH = L.QmTfH; P->dev.QmTfL = L.QmTfL; P->dev.QmfH = L.QmfH; P->dev.QmfL = L.QmfL;
    return MCA_OK;
}

size_t mca_workspace_bytes(const mca_plan *P, const mca_options *opts)
{
    if (!P) return 0;
    mca_options o;
    if (opts) o = *opts;
    else mca_options_default(&o);
    if (validate_options(&o) != MCA_OK) return 0;
    if (o.precond == MCA_PRECOND_APPROX && !approx_fits(P)) return 0;
    return solve_layout(P, &o, nullptr).bytes;
}

size_t mca_precond_workspace_bytes(const mca_plan *P, int32_t form, int32_t precision)
{
    if (!P) return 0;
    Carver c(nullptr);
    precond_layout(P, c, form, precision);
    return c.size() > 0 ? c.size() : kAlign;
}

mca_status mca_residual(const mca_plan *P, const double *g_dev, const double *v_in,
                        const double *v_t, const double *v_b, double *f_t, double *f_b,
                        double *d, void *stream)
{
    if (!P || !g_dev || !v_in || !v_t || !v_b || !f_t || !f_b) return MCA_ERR_INVALID_ARG;
    if (!plan_ready(P)) return MCA_ERR_WORKSPACE;
    MCA_TRY(launch_residual(P, g_dev, v_in, v_t, v_b, f_t, f_b, d, nullptr,
                            static_cast<hipStream_t>(stream)));
    return MCA_OK;
}

mca_status mca_jacobian_apply(const mca_plan *P, const double *d, const double *x_t,
                              const double *x_b, double *y_t, double *y_b, void *stream)
{
    if (!P || !d || !x_t || !x_b || !y_t || !y_b) return MCA_ERR_INVALID_ARG;
    if (!plan_ready(P)) return MCA_ERR_WORKSPACE;
    MCA_TRY(launch_jacobian(P, d, x_t, x_b, y_t, y_b, static_cast<hipStream_t>(stream)));
    return MCA_OK;
}

mca_status mca_precond_apply(const mca_plan *P, int32_t form, int32_t precision, double a1,
                             double a2, const double *r_t, const double *r_b, double *z_t,
                             double *z_b, void *ws, size_t ws_bytes, void *stream)
{
    if (!P || !r_t || !r_b || !z_t || !z_b) return MCA_ERR_INVALID_ARG;
    if (form != MCA_PRECOND_LITERAL && form != MCA_PRECOND_PERMODE && form != MCA_PRECOND_NONE &&
        form != MCA_PRECOND_APPROX)
        return MCA_ERR_INVALID_ARG;
    if (precision != MCA_PREC_FP64 && precision != MCA_PREC_FP32 &&
        precision != MCA_PREC_BF16X3 && precision != MCA_PREC_BF16)
        return MCA_ERR_INVALID_ARG;
    if (precision != MCA_PREC_FP64 && form != MCA_PRECOND_PERMODE && form != MCA_PRECOND_NONE)
        return MCA_ERR_INVALID_ARG;
    if (form == MCA_PRECOND_APPROX && !approx_fits(P)) return MCA_ERR_INVALID_ARG;
    if (!(std::isfinite(a1) && a1 > 0.0 && std::isfinite(a2) && a2 > 0.0))
        return MCA_ERR_INVALID_ARG;
    if (!plan_ready(P)) return MCA_ERR_WORKSPACE;
    if (form != MCA_PRECOND_NONE && (!ws || ws_bytes < mca_precond_workspace_bytes(P, form, precision)))
        return MCA_ERR_WORKSPACE;
    Carver c(ws);
    PrecondWs w = precond_layout(P, c, form, precision);
    const mca_status st = precond_setup(P, form, a1, a2, w, static_cast<hipStream_t>(stream));
    if (st != MCA_OK) return st;
    return precond_run(P, form, precision, a1, a2, r_t, r_b, z_t, z_b, w,
                       static_cast<hipStream_t>(stream));
}

mca_status mca_precond_apply_noalloc(const mca_plan *P, int32_t form, int32_t precision,
                                     double a1, double a2, const double *r_t, const double *r_b,
                                     double *z_t, double *z_b, void *stream)
{
    if (!P) return MCA_ERR_INVALID_ARG;
    if (mca_precond_workspace_bytes(P, form, precision) > kNoAllocBytes) return MCA_ERR_WORKSPACE;
    void *ws = nullptr;
    const mca_status st = noalloc_scratch(&ws);
    if (st != MCA_OK) return st;
    return mca_precond_apply(P, form, precision, a1, a2, r_t, r_b, z_t, z_b, ws, kNoAllocBytes,
                             stream);
}

mca_status mca_solve(const mca_plan *P, const double *g_dev, const double *v_in, double *v_t,
                     double *v_b, const mca_options *opts, void *ws, size_t ws_bytes,
                     mca_stats *stats, void *stream)
{
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (!P || !g_dev || !v_in || !v_t || !v_b) return MCA_ERR_INVALID_ARG;
    mca_options o;
    if (opts) o = *opts;
    else mca_options_default(&o);
    mca_status st = validate_options(&o);
    if (st != MCA_OK) return st;
    if (o.precond == MCA_PRECOND_APPROX && !approx_fits(P)) return MCA_ERR_INVALID_ARG;
    if ((o.flags & MCA_FLAG_SWEEP_START) &&
        (P->geom.m > kSweepMaxLen || P->geom.n > kSweepMaxLen))
        return MCA_ERR_INVALID_ARG;
    if (!plan_ready(P)) return MCA_ERR_WORKSPACE;
    SolveWs w = solve_layout(P, &o, ws);
    if (!ws || ws_bytes < w.bytes) return MCA_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t mn = (size_t)P->geom.m * P->geom.n, len = 2 * mn;
    double *host = pinned_scratch();
    if (!host) {
        set_hip_error("hipHostMalloc", hipErrorOutOfMemory);
        return MCA_ERR_HIP;
    }

    // ||Y|| = g_src ||v_in||
    double *host_dev = pinned_dev(host);
    // (into host word 2, its marker at host word 6; read after the first
    // residual, which is enqueued behind it without a wait in between)
    MCA_TRY(launch_dot_partials(v_in, v_in, P->geom.m, w.pa, s));
    const int e_y = next_epoch();
    MCA_TRY(launch_reduce(w.pa, reduce_blocks(P->geom.m), 1, host_dev + 2, s,
                          reinterpret_cast<int *>(host_dev + 6), e_y));
    double *Vc = w.Vc, *Vn = w.Vn, *F = w.F, *Fn = w.Fn, *D = w.D, *Dn = w.Dn;
    if (o.flags & MCA_FLAG_INITIAL_GUESS) {
        MCA_TRY(hipMemcpyAsync(Vc, v_t, mn * sizeof(double), hipMemcpyDeviceToDevice, s));
        MCA_TRY(hipMemcpyAsync(Vc + mn, v_b, mn * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else if (o.flags & MCA_FLAG_SWEEP_START) {
        MCA_TRY(launch_sweep_guess(P->top, P->bot, P->geom.m, P->geom.n, P->geom.g_src, g_dev,
                                   v_in, Vc, Vc + mn, s));
    } else {
        MCA_TRY(launch_fill(Vc, 0.0, len, s));
    }
    Timing tm;
    if (o.flags & (MCA_FLAG_TIMING | MCA_FLAG_TIMING_SAMPLED))
        MCA_TRY(tm.init(!(o.flags & MCA_FLAG_TIMING)));
    double fnorm = 0.0, fn2 = 0.0, dsum = 0.0;
    SolveWs wk = w;
    st = residual_norms(P, g_dev, v_in, Vc, Vc + mn, F, D, wk, s, &tm, &fnorm, &fn2, &dsum);
    if (st == MCA_ERR_HIP) return st;
    {
        const mca_status ws = wait_marker(reinterpret_cast<int *>(host + 6), e_y, s);
        if (ws != MCA_OK) return ws;
    }
    const double ynorm = P->geom.g_src * std::sqrt(host[2]);
    if (!std::isfinite(ynorm)) return MCA_ERR_NONFINITE;
    if (ynorm == 0.0) {
        // no drive: V = 0 solves F = 0 exactly
        MCA_TRY(launch_fill(v_t, 0.0, mn, s));
        MCA_TRY(launch_fill(v_b, 0.0, mn, s));
        MCA_TRY(hipStreamSynchronize(s));
        return MCA_OK;
    }
    int from_guess = (o.flags & (MCA_FLAG_INITIAL_GUESS | MCA_FLAG_SWEEP_START)) ? 1 : 0;
    if (from_guess && (o.flags & MCA_FLAG_GUESS_FALLBACK) && !(st == MCA_OK && fnorm < ynorm)) {
        // the guess is no better than V = 0, whose residual is ||Y||: start from 0
        MCA_TRY(launch_fill(Vc, 0.0, len, s));
        st = residual_norms(P, g_dev, v_in, Vc, Vc + mn, F, D, wk, s, &tm, &fnorm, &fn2, &dsum);
        if (st == MCA_ERR_HIP) return st;
        from_guess = 0;
    }

    mca_status result = (st == MCA_OK) ? MCA_ERR_NOT_CONVERGED : st;
    int k = 0, total_its = 0, backtracks = 0, restarts = 0;
    double a = 0.0;
    // Tests on squared norms, so that the host and a gated start enqueued ahead
    // (launch_newton_next) decide alike on the same reduced sum.
    const double conv = o.newton_tol * ynorm, conv2 = conv * conv;
    const double *sums_dev = pinned_dev(host);   // the last residual's ||F||^2, sum D
    // the next Newton step's GMRES, its start and first Arnoldi step enqueued
    // behind the full-step trial point before the host has read that point's norm
    std::unique_ptr<Fgmres> ahead;
    const bool look_ahead = Fgmres(P, &o, wk, s, &tm).device_shift();
    for (; st == MCA_OK; ++k) {
        if (stats) stats->residual_history[k] = fnorm / ynorm;
        if (fn2 <= conv2) {
            result = MCA_OK;
            break;
        }
        if (k >= o.max_newton) break;
        a = dsum / (double)mn;   // a1 = a2 = mean device slope (Section III-A)
        wk.F = F;
        wk.D = D;
        std::unique_ptr<Fgmres> fg = std::move(ahead);
        if (!fg) {
            fg.reset(new Fgmres(P, &o, wk, s, &tm));
            st = fg->start(sums_dev, INFINITY, -1.0);
            if (st != MCA_OK) return st;
        }
        int its = 0, rs = 0;
        bool cv = false;
        st = fg->run(fnorm, a, &its, &rs, &cv);
        fg.reset();
        if (st != MCA_OK) {
            result = st;
            break;
        }
        total_its += its;
        restarts += rs;
        if (stats) stats->krylov_history[k] = its;
        // damped update: halve s while ||F(V + s X)|| > (1 - 1e-4 s) ||F(V)||
        double step = 1.0, fn_new = 0.0, fn2_new = 0.0, ds_new = 0.0;
        int halvings = 0;
        for (;;) {
            MCA_TRY(launch_axpby(Vc, step, w.X, Vn, len, s));
            int e = 0;
            st = residual_enqueue(P, g_dev, v_in, Vn, Vn + mn, Fn, Dn, wk, s, &tm, &e);
            if (st != MCA_OK) return st;
            const double thr = (1.0 - 1e-4 * step) * fnorm, accept2 = thr * thr;
            if (look_ahead && step == 1.0 && k + 1 < o.max_newton) {
                SolveWs wn = wk;
                wn.F = Fn;
                wn.D = Dn;
                ahead.reset(new Fgmres(P, &o, wn, s, &tm));
                st = ahead->start(sums_dev, accept2, conv2);
                if (st == MCA_OK) st = ahead->prelaunch_first_step();
                if (st != MCA_OK) return st;
            }
            st = residual_wait(e, s, &tm, &fn_new, &fn2_new, &ds_new);
            if (st != MCA_OK && st != MCA_ERR_NONFINITE) return st;
            if (st == MCA_OK && fn2_new <= accept2) break;
            if (ahead) {   // (its kernels return at once: the device saw the rejection too)
                if ((st = ahead->abandon()) != MCA_OK) return st;
                ahead.reset();
            }
            if (halvings >= 30) break;
            step *= 0.5;
            ++halvings;
        }
        backtracks += halvings;
        if (!(std::isfinite(fn_new) && fn_new < fnorm)) {
            // no decrease: the rounding floor (accepted below 1e-12 ||Y||) or a failure
            result = (fnorm <= 1e-12 * ynorm) ? MCA_OK : MCA_ERR_NOT_CONVERGED;
            break;
        }
        std::swap(Vc, Vn);
        std::swap(F, Fn);
        std::swap(D, Dn);
        fnorm = fn_new;
        fn2 = fn2_new;
        dsum = ds_new;
    }
    if (ahead) {   // converged (the device saw it too) or out of steps: nothing to take
        const mca_status sa = ahead->abandon();
        if (sa != MCA_OK) return sa;
        ahead.reset();
    }
    MCA_TRY(hipMemcpyAsync(v_t, Vc, mn * sizeof(double), hipMemcpyDeviceToDevice, s));
    MCA_TRY(hipMemcpyAsync(v_b, Vc + mn, mn * sizeof(double), hipMemcpyDeviceToDevice, s));
    MCA_TRY(hipStreamSynchronize(s));
    if (stats) {
        stats->newton_iters = k;
        stats->krylov_iters = total_its;
        stats->backtracks = backtracks;
        stats->restarts = restarts;
        stats->rel_residual = fnorm / ynorm;
        stats->a_last = a;
        stats->start = from_guess;
        stats->err_bound = fnorm / std::min(P->lt[0], P->lb[0]);
        for (int c = 0; c < MCA_NUM_KCLASS; ++c) {
            stats->kernel_ms[c] = tm.ms[c];
            stats->kernel_launches[c] = tm.launches[c];
        }
    }
    return result;
}

}  // extern "C"
