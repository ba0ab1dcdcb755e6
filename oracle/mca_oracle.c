/*
 * mca_oracle.c -- plain, slow FP64 CPU reference for the steady-state
 * memristor-crossbar (MCA) solver of "A Fast Method for Steady-State Memristor
 * Crossbar Array Circuit Simulation" (Xie et al.).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline of the benchmark may load this library. The HIP solver never
 * calls, links or includes anything from here, and this file includes nothing
 * from the HIP side: the two share no code, header or table.
 *
 * What it computes (every routine follows the paper's definitions literally):
 *   - the wire conductance matrix of one uniform wire (Section II, eq. (G)),
 *     with the end rows carrying the terminations described below;
 *   - the MNA residual F (eqs. (MNA) and (F)) and the device derivative D;
 *   - the Jacobian product J x (eq. (J)) with the four diagonal device blocks
 *     that the perpendicular natural indexing gives (Section III-A);
 *   - the preconditioner solve z = P^{-1} r with P from eq. (P), by a direct
 *     method on the assembled P (dense LU, or band Cholesky of a symmetrised P);
 *   - the paper's approximate preconditioner (M ~ Mhat, eqs. (Mhat) to
 *     (2matrix4)) in the paper's order with tridiagonal solves, and the
 *     point-Jacobi preconditioner as a baseline;
 *   - the steady state F(V) = 0 by Newton's method (eq. (Newton3)) whose
 *     linear steps are direct band-Cholesky solves of J (oracle A), or
 *     preconditioned CG with exact wire-line block solves (oracle B, for sizes
 *     whose band does not fit in memory).
 *
 * Readings where the paper is silent (the same ones the HIP side documents):
 *   - Drive: an ideal source V_in[i] behind conductance g_src into top node
 *     (i,0); so Y_t[i,0] = g_src * V_in[i], Y_b = 0.
 *   - Terminations: top node (i,n-1) to ground through g_top_end; bottom nodes
 *     (0,j) and (m-1,j) to ground through g_bot_end0 / g_bot_end1.  Each wire
 *     end adds its termination to the diagonal; with every termination equal
 *     to g the matrix is the paper's eq. (G) (2g on the whole diagonal).
 *   - Device: I = g v0 sinh(u/v0) with u = V_t - V_b (or the linear I = g u);
 *     D = dI/du.  I leaves the top node and enters the bottom node.
 *   - Indexing: both layers m x n row-major, k = i*n + j (top wires are rows,
 *     bottom wires are columns), so G_t = I_m (x) G_top, G_b = G_bot (x) I_n.
 *
 * Parity pins: see the tests.  Every routine here is pinned by at least one
 * independent check (netlist stamping, dense LU, finite differences, closed
 * forms, Kirchhoff balance, exactness of P for uniform linear devices).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int m, n;
    int device;            /* 0: sinh device, 1: linear device */
    int pad_;
    double g_top, g_bot, g_src, g_top_end, g_bot_end0, g_bot_end1, v0;
} orc_geom;

/* ------------------------------------------------------------------------ */
/* Wire conductance matrix of one uniform wire of `len` nodes (eq. (G)).
 * Stamped element by element: each segment of conductance g between nodes k
 * and k+1 adds g to both diagonal entries and -g to the coupling; the wire's
 * first node has end0 to its far side, the last node end1.
 * diag has len entries, off has len-1 (off[k] couples k and k+1).           */
void orc_wire_matrix(int len, double g, double end0, double end1,
                     double *diag, double *off)
{
    for (int k = 0; k < len; ++k) diag[k] = 0.0;
    for (int k = 0; k + 1 < len; ++k) {
        diag[k] += g;
        diag[k + 1] += g;
        off[k] = -g;
    }
    diag[0] += end0;
    diag[len - 1] += end1;
}

static void top_wire(const orc_geom *G, double *diag, double *off)
{
    orc_wire_matrix(G->n, G->g_top, G->g_src, G->g_top_end, diag, off);
}

static void bot_wire(const orc_geom *G, double *diag, double *off)
{
    orc_wire_matrix(G->m, G->g_bot, G->g_bot_end0, G->g_bot_end1, diag, off);
}

/* Device current and its derivative (the device model of the crossbar). */
static double dev_current(const orc_geom *G, double g, double u)
{
    if (G->device == 1) return g * u;
    return g * G->v0 * sinh(u / G->v0);
}

static double dev_slope(const orc_geom *G, double g, double u)
{
    if (G->device == 1) return g;
    return g * cosh(u / G->v0);
}

/* ------------------------------------------------------------------------ */
/* y_t = (I_m (x) G_top) x_t  and  y_b = (G_bot (x) I_n) x_b   (eqs. (Gt), (Gb)).
 * Written as the Kronecker definitions: G_top acts on each row i of x_t,
 * G_bot on each column j of x_b.                                            */
static void apply_layers(const orc_geom *G, const double *xt, const double *xb,
                         double *yt, double *yb)
{
    int m = G->m, n = G->n;
    double *td = malloc(sizeof(double) * n), *to = malloc(sizeof(double) * (n + 1));
    double *bd = malloc(sizeof(double) * m), *bo = malloc(sizeof(double) * (m + 1));
    top_wire(G, td, to);
    bot_wire(G, bd, bo);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            double s = td[j] * xt[i * n + j];
            if (j > 0) s += to[j - 1] * xt[i * n + j - 1];
            if (j + 1 < n) s += to[j] * xt[i * n + j + 1];
            yt[i * n + j] = s;
        }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            double s = bd[i] * xb[i * n + j];
            if (i > 0) s += bo[i - 1] * xb[(i - 1) * n + j];
            if (i + 1 < m) s += bo[i] * xb[(i + 1) * n + j];
            yb[i * n + j] = s;
        }
    free(td); free(to); free(bd); free(bo);
}

/* MNA residual, eqs. (MNA)/(F):
 *   F_t = G_t V_t + I(V_t - V_b) - Y_t,   F_b = G_b V_b - I(V_t - V_b) - Y_b,
 * plus D = dI/du at every crosspoint (the diagonal of each device block of
 * eq. (J)).  Any of f_t, f_b, d may be NULL.                                 */
void orc_residual(const orc_geom *G, const double *g_dev, const double *v_in,
                  const double *vt, const double *vb,
                  double *f_t, double *f_b, double *d)
{
    int m = G->m, n = G->n;
    size_t mn = (size_t)m * n;
    double *yt = malloc(sizeof(double) * mn), *yb = malloc(sizeof(double) * mn);
    apply_layers(G, vt, vb, yt, yb);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            size_t k = (size_t)i * n + j;
            double u = vt[k] - vb[k];
            double cur = dev_current(G, g_dev[k], u);
            double src = (j == 0) ? G->g_src * v_in[i] : 0.0;   /* Y_t */
            if (f_t) f_t[k] = yt[k] + cur - src;
            if (f_b) f_b[k] = yb[k] - cur;                       /* Y_b = 0 */
            if (d) d[k] = dev_slope(G, g_dev[k], u);
        }
    free(yt); free(yb);
}

/* ||Y||_2: the norm of the boundary-source vector. */
double orc_source_norm(const orc_geom *G, const double *v_in)
{
    double s = 0.0;
    for (int i = 0; i < G->m; ++i) s += (G->g_src * v_in[i]) * (G->g_src * v_in[i]);
    return sqrt(s);
}

/* Jacobian product, eq. (J): the layer block diagonal plus the device blocks
 *   [[ D, -D], [-D, D]]  (dI_t/dV_t = D = -dI_t/dV_b, Section III-A).      */
void orc_jacobian_apply(const orc_geom *G, const double *d,
                        const double *xt, const double *xb,
                        double *yt, double *yb)
{
    size_t mn = (size_t)G->m * G->n;
    apply_layers(G, xt, xb, yt, yb);
    for (size_t k = 0; k < mn; ++k) {
        double c = d[k] * (xt[k] - xb[k]);
        yt[k] += c;
        yb[k] -= c;
    }
}

/* ------------------------------------------------------------------------ */
/* Dense assembly.  Unknown order: top layer k = i*n+j first (0..mn-1), then
 * the bottom layer (mn..2mn-1), the paper's stacking [V_t; V_b].  Row-major
 * N x N with N = 2mn.                                                        */
static void dense_layers(const orc_geom *G, double *A)
{
    int m = G->m, n = G->n;
    size_t N = 2 * (size_t)m * n, mn = (size_t)m * n;
    double *td = malloc(sizeof(double) * n), *to = malloc(sizeof(double) * (n + 1));
    double *bd = malloc(sizeof(double) * m), *bo = malloc(sizeof(double) * (m + 1));
    top_wire(G, td, to);
    bot_wire(G, bd, bo);
    memset(A, 0, sizeof(double) * N * N);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            size_t k = (size_t)i * n + j;
            A[k * N + k] = td[j];
            if (j > 0) A[k * N + (k - 1)] = to[j - 1];
            if (j + 1 < n) A[k * N + (k + 1)] = to[j];
            size_t kb = mn + k;
            A[kb * N + kb] = bd[i];
            if (i > 0) A[kb * N + (kb - n)] = bo[i - 1];
            if (i + 1 < m) A[kb * N + (kb + n)] = bo[i];
        }
    free(td); free(to); free(bd); free(bo);
}

/* Dense J (eq. (J)) for a device-derivative array d. */
void orc_dense_jacobian(const orc_geom *G, const double *d, double *A)
{
    size_t mn = (size_t)G->m * G->n, N = 2 * mn;
    dense_layers(G, A);
    for (size_t k = 0; k < mn; ++k) {
        A[k * N + k] += d[k];
        A[k * N + mn + k] -= d[k];
        A[(mn + k) * N + k] -= d[k];
        A[(mn + k) * N + mn + k] += d[k];
    }
}

/* Dense P (eq. (P)): [[G_t + a1 I, -a1 I], [-a2 I, G_b + a2 I]]. */
void orc_dense_precond(const orc_geom *G, double a1, double a2, double *A)
{
    size_t mn = (size_t)G->m * G->n, N = 2 * mn;
    dense_layers(G, A);
    for (size_t k = 0; k < mn; ++k) {
        A[k * N + k] += a1;
        A[k * N + mn + k] -= a1;
        A[(mn + k) * N + k] -= a2;
        A[(mn + k) * N + mn + k] += a2;
    }
}

/* Gaussian elimination with partial pivoting; solves A x = b in place
 * (A is destroyed, b becomes x).  Returns 0, or -1 for a zero pivot.       */
int orc_dense_solve(int N, double *A, double *b)
{
    for (int c = 0; c < N; ++c) {
        int p = c;
        for (int r = c + 1; r < N; ++r)
            if (fabs(A[(size_t)r * N + c]) > fabs(A[(size_t)p * N + c])) p = r;
        if (A[(size_t)p * N + c] == 0.0) return -1;
        if (p != c) {
            for (int k = 0; k < N; ++k) {
                double t = A[(size_t)c * N + k];
                A[(size_t)c * N + k] = A[(size_t)p * N + k];
                A[(size_t)p * N + k] = t;
            }
            double t = b[c]; b[c] = b[p]; b[p] = t;
        }
        for (int r = c + 1; r < N; ++r) {
            double f = A[(size_t)r * N + c] / A[(size_t)c * N + c];
            if (f == 0.0) continue;
            for (int k = c; k < N; ++k) A[(size_t)r * N + k] -= f * A[(size_t)c * N + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = N - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < N; ++k) s -= A[(size_t)r * N + k] * b[k];
        b[r] = s / A[(size_t)r * N + r];
    }
    return 0;
}

/* z = P^{-1} r by dense LU of the assembled P (tiny sizes only). */
int orc_precond_apply_dense(const orc_geom *G, double a1, double a2,
                            const double *rt, const double *rb,
                            double *zt, double *zb)
{
    size_t mn = (size_t)G->m * G->n, N = 2 * mn;
    double *A = malloc(sizeof(double) * N * N), *x = malloc(sizeof(double) * N);
    if (!A || !x) { free(A); free(x); return -2; }
    orc_dense_precond(G, a1, a2, A);
    memcpy(x, rt, sizeof(double) * mn);
    memcpy(x + mn, rb, sizeof(double) * mn);
    int rc = orc_dense_solve((int)N, A, x);
    memcpy(zt, x, sizeof(double) * mn);
    memcpy(zb, x + mn, sizeof(double) * mn);
    free(A); free(x);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Band storage of a symmetric positive definite matrix in the interleaved
 * order: unknown 2c is the top node of crosspoint c, 2c+1 its bottom node,
 * with c = i*n + j when n <= m and c = j*m + i otherwise, so that the
 * half bandwidth is p = 2 min(m, n).  L[r*(p+1) + (r - col)] holds entry
 * (r, col) of the lower triangle for r - p <= col <= r.                      */
typedef struct {
    size_t N;
    int p;
    double *L;
} band_t;

static size_t cross_index(const orc_geom *G, int i, int j)
{
    return (G->n <= G->m) ? (size_t)i * G->n + j : (size_t)j * G->m + i;
}

static void band_set(band_t *B, size_t r, size_t c, double v)
{
    if (c > r) { size_t t = r; r = c; c = t; }
    B->L[r * (B->p + 1) + (r - c)] += v;
}

/* Assemble  [[G_t + Dt, -Dc], [-Dc, s*G_b + Db]]  (Dt, Dc, Db per crosspoint)
 * in band storage.  J is Dt = Dc = Db = d, s = 1; the symmetrised P is
 * Dt = Dc = Db = a1 with s = a1/a2 (rows of the bottom block scaled).       */
static int band_assemble(const orc_geom *G, double dcoef_scalar,
                         const double *dvec, double bot_scale, band_t *B)
{
    int m = G->m, n = G->n;
    B->N = 2 * (size_t)m * n;
    B->p = 2 * (m < n ? m : n);
    B->L = calloc(B->N * (size_t)(B->p + 1), sizeof(double));
    if (!B->L) return -2;
    double *td = malloc(sizeof(double) * n), *to = malloc(sizeof(double) * (n + 1));
    double *bd = malloc(sizeof(double) * m), *bo = malloc(sizeof(double) * (m + 1));
    top_wire(G, td, to);
    bot_wire(G, bd, bo);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            size_t c = cross_index(G, i, j);
            size_t t = 2 * c, b = 2 * c + 1;
            size_t k = (size_t)i * n + j;
            double dk = dvec ? dvec[k] : dcoef_scalar;
            band_set(B, t, t, td[j] + dk);
            if (j + 1 < n) band_set(B, t, 2 * cross_index(G, i, j + 1), to[j]);
            band_set(B, b, b, bot_scale * bd[i] + dk);
            if (i + 1 < m) band_set(B, b, 2 * cross_index(G, i + 1, j) + 1, bot_scale * bo[i]);
            band_set(B, t, b, -dk);
        }
    free(td); free(to); free(bd); free(bo);
    return 0;
}

/* Band Cholesky A = L L^T, in place, row by row. Returns 0 or -1 (not SPD). */
static int band_cholesky(band_t *B)
{
    size_t N = B->N;
    int p = B->p;
    double *L = B->L;
    for (size_t r = 0; r < N; ++r) {
        size_t c0 = r > (size_t)p ? r - p : 0;
        for (size_t c = c0; c <= r; ++c) {
            /* entry (r, c) minus sum_{k} L(r,k) L(c,k) over shared columns */
            size_t k0 = c > (size_t)p ? c - p : 0;
            if (k0 < c0) k0 = c0;
            double s = L[r * (p + 1) + (r - c)];
            for (size_t k = k0; k < c; ++k)
                s -= L[r * (p + 1) + (r - k)] * L[c * (p + 1) + (c - k)];
            if (c == r) {
                if (!(s > 0.0)) return -1;
                L[r * (p + 1)] = sqrt(s);
            } else {
                L[r * (p + 1) + (r - c)] = s / L[c * (p + 1)];
            }
        }
    }
    return 0;
}

/* Solve L L^T x = b in place. */
static void band_solve(const band_t *B, double *x)
{
    size_t N = B->N;
    int p = B->p;
    const double *L = B->L;
    for (size_t r = 0; r < N; ++r) {
        size_t c0 = r > (size_t)p ? r - p : 0;
        double s = x[r];
        for (size_t c = c0; c < r; ++c) s -= L[r * (p + 1) + (r - c)] * x[c];
        x[r] = s / L[r * (p + 1)];
    }
    for (size_t r = N; r-- > 0;) {
        size_t c1 = r + p < N - 1 ? r + p : N - 1;
        double s = x[r];
        for (size_t c = r + 1; c <= c1; ++c) s -= L[c * (p + 1) + (c - r)] * x[c];
        x[r] = s / L[r * (p + 1)];
    }
}

static void to_interleaved(const orc_geom *G, const double *xt, const double *xb, double *x)
{
    for (int i = 0; i < G->m; ++i)
        for (int j = 0; j < G->n; ++j) {
            size_t c = cross_index(G, i, j), k = (size_t)i * G->n + j;
            x[2 * c] = xt[k];
            x[2 * c + 1] = xb[k];
        }
}

static void from_interleaved(const orc_geom *G, const double *x, double *xt, double *xb)
{
    for (int i = 0; i < G->m; ++i)
        for (int j = 0; j < G->n; ++j) {
            size_t c = cross_index(G, i, j), k = (size_t)i * G->n + j;
            xt[k] = x[2 * c];
            xb[k] = x[2 * c + 1];
        }
}

/* z = P^{-1} r for P of eq. (P), any a1, a2 > 0.  Scaling P's bottom block row
 * by a1/a2 gives [[G_t + a1 I, -a1 I], [-a1 I, (a1/a2) G_b + a1 I]], which is
 * symmetric positive definite; solve that by band Cholesky.                  */
int orc_precond_apply_band(const orc_geom *G, double a1, double a2,
                           const double *rt, const double *rb,
                           double *zt, double *zb)
{
    if (!(a1 > 0.0) || !(a2 > 0.0)) return -3;
    band_t B;
    double s = a1 / a2;
    if (band_assemble(G, a1, NULL, s, &B)) return -2;
    if (band_cholesky(&B)) { free(B.L); return -1; }
    size_t mn = (size_t)G->m * G->n;
    double *x = malloc(sizeof(double) * 2 * mn), *rbs = malloc(sizeof(double) * mn);
    for (size_t k = 0; k < mn; ++k) rbs[k] = s * rb[k];
    to_interleaved(G, rt, rbs, x);
    band_solve(&B, x);
    from_interleaved(G, x, zt, zb);
    free(x); free(rbs); free(B.L);
    return 0;
}

/* Solve J x = b for J of eq. (J) at device derivative d, by band Cholesky. */
int orc_jacobian_solve_band(const orc_geom *G, const double *d,
                            const double *bt, const double *bb,
                            double *xt, double *xb)
{
    band_t B;
    if (band_assemble(G, 0.0, d, 1.0, &B)) return -2;
    if (band_cholesky(&B)) { free(B.L); return -1; }
    size_t mn = (size_t)G->m * G->n;
    double *x = malloc(sizeof(double) * 2 * mn);
    to_interleaved(G, bt, bb, x);
    band_solve(&B, x);
    from_interleaved(G, x, xt, xb);
    free(x); free(B.L);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Oracle B's linear solver: CG on J (symmetric positive definite) with the
 * block-diagonal preconditioner made of every top row wire
 * (G_top + diag D[i,:]) and every bottom column wire (G_bot + diag D[:,j]),
 * each solved exactly by the Thomas algorithm.                               */
static void thomas(int len, const double *diag, const double *off, double *x, double *wk)
{
    /* solve tridiag(off, diag, off) y = x in place; wk has len entries */
    double c = diag[0];
    x[0] /= c;
    for (int k = 1; k < len; ++k) {
        wk[k] = off[k - 1] / c;
        c = diag[k] - off[k - 1] * wk[k];
        x[k] = (x[k] - off[k - 1] * x[k - 1]) / c;
    }
    for (int k = len - 2; k >= 0; --k) x[k] -= wk[k + 1] * x[k + 1];
}

static void line_jacobi(const orc_geom *G, const double *d,
                        const double *rt, const double *rb, double *zt, double *zb)
{
    int m = G->m, n = G->n;
    int L = m > n ? m : n;
    double *td = malloc(sizeof(double) * n), *to = malloc(sizeof(double) * (n + 1));
    double *bd = malloc(sizeof(double) * m), *bo = malloc(sizeof(double) * (m + 1));
    double *dg = malloc(sizeof(double) * L), *x = malloc(sizeof(double) * L),
           *wk = malloc(sizeof(double) * L);
    top_wire(G, td, to);
    bot_wire(G, bd, bo);
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < n; ++j) {
            dg[j] = td[j] + d[(size_t)i * n + j];
            x[j] = rt[(size_t)i * n + j];
        }
        thomas(n, dg, to, x, wk);
        for (int j = 0; j < n; ++j) zt[(size_t)i * n + j] = x[j];
    }
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < m; ++i) {
            dg[i] = bd[i] + d[(size_t)i * n + j];
            x[i] = rb[(size_t)i * n + j];
        }
        thomas(m, dg, bo, x, wk);
        for (int i = 0; i < m; ++i) zb[(size_t)i * n + j] = x[i];
    }
    free(td); free(to); free(bd); free(bo); free(dg); free(x); free(wk);
}

static double dot2(size_t mn, const double *at, const double *ab,
                   const double *bt, const double *bb)
{
    double s = 0.0;
    for (size_t k = 0; k < mn; ++k) s += at[k] * bt[k] + ab[k] * bb[k];
    return s;
}

/* Returns the number of CG iterations, or -1 if rel_tol was not reached. */
int orc_jacobian_solve_cg(const orc_geom *G, const double *d,
                          const double *bt, const double *bb,
                          double *xt, double *xb, double rel_tol, int max_it)
{
    size_t mn = (size_t)G->m * G->n;
    double *r = malloc(sizeof(double) * 2 * mn), *z = malloc(sizeof(double) * 2 * mn),
           *p = malloc(sizeof(double) * 2 * mn), *q = malloc(sizeof(double) * 2 * mn);
    double *rt = r, *rb = r + mn, *zt = z, *zb = z + mn, *pt = p, *pb = p + mn,
           *qt = q, *qb = q + mn;
    memset(xt, 0, sizeof(double) * mn);
    memset(xb, 0, sizeof(double) * mn);
    memcpy(rt, bt, sizeof(double) * mn);
    memcpy(rb, bb, sizeof(double) * mn);
    double bnorm = sqrt(dot2(mn, bt, bb, bt, bb));
    int it = 0, ok = (bnorm == 0.0);
    if (!ok) {
        line_jacobi(G, d, rt, rb, zt, zb);
        memcpy(p, z, sizeof(double) * 2 * mn);
        double rz = dot2(mn, rt, rb, zt, zb);
        for (it = 1; it <= max_it; ++it) {
            orc_jacobian_apply(G, d, pt, pb, qt, qb);
            double alpha = rz / dot2(mn, pt, pb, qt, qb);
            for (size_t k = 0; k < mn; ++k) {
                xt[k] += alpha * pt[k];
                xb[k] += alpha * pb[k];
            }
            for (size_t k = 0; k < 2 * mn; ++k) r[k] -= alpha * q[k];
            if (sqrt(dot2(mn, rt, rb, rt, rb)) <= rel_tol * bnorm) { ok = 1; break; }
            line_jacobi(G, d, rt, rb, zt, zb);
            double rz_new = dot2(mn, rt, rb, zt, zb);
            double beta = rz_new / rz;
            rz = rz_new;
            for (size_t k = 0; k < 2 * mn; ++k) p[k] = z[k] + beta * p[k];
        }
    }
    free(r); free(z); free(p); free(q);
    return ok ? it : -1;
}

/* ------------------------------------------------------------------------ */
/* Newton's method for F(V) = 0 (eq. (Newton3)), starting from the given V
 * (zero unless the caller passes a guess).  Each step solves J(V) dV = -F(V)
 * directly (linear = 0: band Cholesky) or by CG to 1e-13 (linear = 1), then
 * backtracks: halve s while ||F(V + s dV)|| > (1 - 1e-4 s) ||F(V)||.
 * Stops when ||F|| <= tol ||Y||, or at the rounding floor (no decrease once
 * ||F|| <= 1e-12 ||Y||), or after max_it steps.  hist (may be NULL) receives
 * ||F||/||Y|| before each step, max_it + 1 entries.
 * Returns the number of Newton steps taken, or -1 if it did not converge.   */
int orc_solve(const orc_geom *G, const double *g_dev, const double *v_in,
              double *vt, double *vb, double tol, int max_it, int linear,
              double *hist)
{
    size_t mn = (size_t)G->m * G->n;
    double ynorm = orc_source_norm(G, v_in);
    if (ynorm == 0.0) {
        memset(vt, 0, sizeof(double) * mn);
        memset(vb, 0, sizeof(double) * mn);
        if (hist) hist[0] = 0.0;
        return 0;
    }
    double *f = malloc(sizeof(double) * 2 * mn), *d = malloc(sizeof(double) * mn),
           *dv = malloc(sizeof(double) * 2 * mn), *nt = malloc(sizeof(double) * 2 * mn),
           *nf = malloc(sizeof(double) * 2 * mn), *nd = malloc(sizeof(double) * mn);
    orc_residual(G, g_dev, v_in, vt, vb, f, f + mn, d);
    double fn = sqrt(dot2(mn, f, f + mn, f, f + mn));
    int k = 0, rc = -1;
    for (; k <= max_it; ++k) {
        if (hist) hist[k] = fn / ynorm;
        if (fn <= tol * ynorm) { rc = k; break; }
        if (k == max_it) break;
        for (size_t q = 0; q < 2 * mn; ++q) f[q] = -f[q];
        int lrc = linear ? (orc_jacobian_solve_cg(G, d, f, f + mn, dv, dv + mn, 1e-13, 20000) < 0)
                         : orc_jacobian_solve_band(G, d, f, f + mn, dv, dv + mn);
        if (lrc) break;
        double s = 1.0, nfn = 0.0;
        int halvings = 0;
        for (;;) {
            for (size_t q = 0; q < mn; ++q) {
                nt[q] = vt[q] + s * dv[q];
                nt[mn + q] = vb[q] + s * dv[mn + q];
            }
            orc_residual(G, g_dev, v_in, nt, nt + mn, nf, nf + mn, nd);
            nfn = sqrt(dot2(mn, nf, nf + mn, nf, nf + mn));
            if (nfn <= (1.0 - 1e-4 * s) * fn || halvings >= 30) break;
            s *= 0.5;
            ++halvings;
        }
        if (!(nfn < fn)) {
            /* no decrease: the rounding floor is reached, keep V */
            if (fn <= 1e-12 * ynorm) rc = k;
            break;
        }
        memcpy(vt, nt, sizeof(double) * mn);
        memcpy(vb, nt + mn, sizeof(double) * mn);
        memcpy(f, nf, sizeof(double) * 2 * mn);
        memcpy(d, nd, sizeof(double) * mn);
        fn = nfn;
    }
    free(f); free(d); free(dv); free(nt); free(nf); free(nd);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* The paper's approximate preconditioner (Section III-B, eqs. (diagM) to
 * (2matrix4)).  The Schur complement M of eq. (M) is -a2 I + (G2 (x) G1)/a1
 * with G1 = G_top + a1 I (eq. (G1), n x n) and G2 = G_bot + a2 I (eq. (G2),
 * m x m).  Dropping the -a2 I term (small against the wire conductance,
 * eq. (condition)) gives M ~ Mhat = G2hat (x) G1 with G2hat = G2 / a1
 * (eq. (Mhat); the off-diagonal of eq. (G2hat) is read as -g/a1), whose
 * inverse is G2hat^{-1} (x) G1^{-1} (eq. (M-1hat)).  With the row-major
 * vec of an m x n array, (A (x) B) vec(X) = vec(A X B^T), so eq. (2matrix4)
 * reads  Mhat^{-1} w  <->  G2hat^{-1} W G1^{-1}: one tridiagonal solve with
 * G2hat down every column of W and one with G1 along every row.            */

/* Tridiagonal solve T x = b by Gaussian elimination without pivoting (the
 * Thomas algorithm; T is diagonally dominant here).  diag has len entries,
 * off len-1 (symmetric T).  x and b may alias; `stride` steps between the
 * entries of b / x.                                                         */
static void tridiag_solve(int len, const double *diag, const double *off,
                          const double *b, double *x, size_t stride)
{
    double *cp = malloc(sizeof(double) * len), *dp = malloc(sizeof(double) * len);
    cp[0] = (len > 1) ? off[0] / diag[0] : 0.0;
    dp[0] = b[0] / diag[0];
    for (int k = 1; k < len; ++k) {
        double den = diag[k] - off[k - 1] * cp[k - 1];
        cp[k] = (k + 1 < len) ? off[k] / den : 0.0;
        dp[k] = (b[k * stride] - off[k - 1] * dp[k - 1]) / den;
    }
    x[(size_t)(len - 1) * stride] = dp[len - 1];
    for (int k = len - 2; k >= 0; --k)
        x[k * stride] = dp[k] - cp[k] * x[(size_t)(k + 1) * stride];
    free(cp); free(dp);
}

/* out = Mhat^{-1} w (eqs. (M-1hat), (2matrix4)); w, out m x n row-major. */
void orc_mhat_inverse_apply(const orc_geom *G, double a1, double a2,
                            const double *w, double *out)
{
    int m = G->m, n = G->n;
    double *g1d = malloc(sizeof(double) * n), *g1o = malloc(sizeof(double) * (n + 1));
    double *g2d = malloc(sizeof(double) * m), *g2o = malloc(sizeof(double) * (m + 1));
    /* G1 = G_top + a1 I (eq. (G1)); G2hat = (G_bot + a2 I) / a1 (eqs. (G2), (G2hat)) */
    top_wire(G, g1d, g1o);
    for (int j = 0; j < n; ++j) g1d[j] += a1;
    bot_wire(G, g2d, g2o);
    for (int i = 0; i < m; ++i) g2d[i] = (g2d[i] + a2) / a1;
    for (int i = 0; i + 1 < m; ++i) g2o[i] /= a1;
    memcpy(out, w, sizeof(double) * (size_t)m * n);
    /* G2hat^{-1} W: one solve down each column j */
    for (int j = 0; j < n; ++j) tridiag_solve(m, g2d, g2o, out + j, out + j, (size_t)n);
    /* (G2hat^{-1} W) G1^{-1}: one solve along each row i (G1 symmetric) */
    for (int i = 0; i < m; ++i)
        tridiag_solve(n, g1d, g1o, out + (size_t)i * n, out + (size_t)i * n, 1);
    free(g1d); free(g1o); free(g2d); free(g2o);
}

/* z = Phat^{-1} r: the block-inversion formula of eq. (block) with M replaced
 * by Mhat, in the paper's order:
 *   w   = r_b + (G_b + a2 I) r_t / a1       (-D B^{-1} r_t + r_b, B = -a1 I)
 *   z_t = Mhat^{-1} w
 *   z_b = ((G_t + a1 I) z_t - r_t) / a1     (B^{-1} (r_t - A z_t))          */
void orc_precond_apply_approx(const orc_geom *G, double a1, double a2,
                              const double *rt, const double *rb,
                              double *zt, double *zb)
{
    size_t mn = (size_t)G->m * G->n;
    double *gt = malloc(sizeof(double) * mn), *gb = malloc(sizeof(double) * mn);
    double *w = malloc(sizeof(double) * mn);
    apply_layers(G, rt, rt, gt, gb);   /* gb = G_b r_t (gt unused) */
    for (size_t q = 0; q < mn; ++q) w[q] = rb[q] + (gb[q] + a2 * rt[q]) / a1;
    orc_mhat_inverse_apply(G, a1, a2, w, zt);
    apply_layers(G, zt, zt, gt, gb);   /* gt = G_t z_t */
    for (size_t q = 0; q < mn; ++q) zb[q] = (gt[q] + a1 * zt[q] - rt[q]) / a1;
    free(gt); free(gb); free(w);
}

/* Jacobi (point-diagonal) preconditioner of J, a baseline: z = r ./ diag(J)
 * with diag(J) = diag(G_t) + D on the top layer, diag(G_b) + D below.      */
void orc_jacobi_apply(const orc_geom *G, const double *d, const double *rt,
                      const double *rb, double *zt, double *zb)
{
    int m = G->m, n = G->n;
    double *td = malloc(sizeof(double) * n), *to = malloc(sizeof(double) * (n + 1));
    double *bd = malloc(sizeof(double) * m), *bo = malloc(sizeof(double) * (m + 1));
    top_wire(G, td, to);
    bot_wire(G, bd, bo);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            size_t q = (size_t)i * n + j;
            zt[q] = rt[q] / (td[j] + d[q]);
            zb[q] = rb[q] / (bd[i] + d[q]);
        }
    free(td); free(to); free(bd); free(bo);
}

/* ------------------------------------------------------------------------ */
/* One block Gauss-Seidel sweep on the linearisation at V = 0, a cheap start
 * for Newton's method: J(0) = [[G_t + D, -D], [-D, G_b + D]] with D = g_dev
 * (the device slope at u = 0 for both device models), right-hand side Y.
 *   V_t = (G_t + D)^{-1} Y_t              (one tridiagonal solve per row)
 *   V_b = (G_b + D)^{-1} (D V_t)          (one per column; Y_b = 0)
 * Written as the Thomas algorithm per wire with the device conductances on
 * the diagonal.                                                              */
static void tridiag_solve_var(int len, const double *diag, const double *off,
                              const double *b, double *x, size_t stride)
{
    double *cp = malloc(sizeof(double) * len), *dp = malloc(sizeof(double) * len);
    cp[0] = (len > 1) ? off[0] / diag[0] : 0.0;
    dp[0] = b[0] / diag[0];
    for (int k = 1; k < len; ++k) {
        double den = diag[k * stride] - off[k - 1] * cp[k - 1];
        cp[k] = (k + 1 < len) ? off[k] / den : 0.0;
        dp[k] = (b[k * stride] - off[k - 1] * dp[k - 1]) / den;
    }
    x[(size_t)(len - 1) * stride] = dp[len - 1];
    for (int k = len - 2; k >= 0; --k)
        x[k * stride] = dp[k] - cp[k] * x[(size_t)(k + 1) * stride];
    free(cp); free(dp);
}

void orc_sweep_guess(const orc_geom *G, const double *g_dev, const double *v_in,
                     double *vt, double *vb)
{
    int m = G->m, n = G->n;
    size_t mn = (size_t)m * n;
    double *td = malloc(sizeof(double) * n), *to = malloc(sizeof(double) * (n + 1));
    double *bd = malloc(sizeof(double) * m), *bo = malloc(sizeof(double) * (m + 1));
    double *dg = malloc(sizeof(double) * mn), *rhs = malloc(sizeof(double) * mn);
    top_wire(G, td, to);
    bot_wire(G, bd, bo);
    /* rows: (G_top + diag(g_dev[i, :])) v = Y_t[i, :] */
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < n; ++j) {
            size_t q = (size_t)i * n + j;
            dg[q] = td[j] + g_dev[q];
            rhs[q] = (j == 0) ? G->g_src * v_in[i] : 0.0;
        }
        tridiag_solve_var(n, dg + (size_t)i * n, to, rhs + (size_t)i * n, vt + (size_t)i * n, 1);
    }
    /* columns: (G_bot + diag(g_dev[:, j])) v = g_dev[:, j] * V_t[:, j] */
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            size_t q = (size_t)i * n + j;
            dg[q] = bd[i] + g_dev[q];
            rhs[q] = g_dev[q] * vt[q];
        }
    for (int j = 0; j < n; ++j) tridiag_solve_var(m, dg + j, bo, rhs + j, vb + j, (size_t)n);
    free(td); free(to); free(bd); free(bo); free(dg); free(rhs);
}
