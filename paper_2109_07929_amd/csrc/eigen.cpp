// eigen.cpp -- host eigen-decomposition of a symmetric tridiagonal wire matrix.
//
// The paper applies M^{-1} (eq. (M)) through Kronecker products of the
// single-wire matrices G1 = G_top + a1 I and G2 = G_bot + a2 I (eqs. (G1),
// (G2), (M-1hat), (2matrix4)).  Diagonalising each wire matrix once,
// G = Q diag(lambda) Q^T, makes both shifts free (G + a I = Q diag(lambda + a)
// Q^T) and turns the Kronecker factor into an elementwise division, so the
// per-Newton-step work is four dense transforms and no factorisation.
//
// Method (textbook, O(n^2) overall):
//   1. eigenvalues by Sturm-sequence bisection: the number of negative pivots
//      of the LDL^T factorisation of T - x I counts the eigenvalues below x
//      (sixteen eigenvalues bisected side by side: 1.9 -> 0.46 s for the
//      1024 x 1024 plan on one core);
//   2. eigenvectors by inverse iteration with the bisected eigenvalue as the
//      shift, solving (T - lambda I) x = b by Gaussian elimination with
//      partial pivoting on the tridiagonal band, re-orthogonalised (twice,
//      modified Gram-Schmidt) against the already computed eigenvectors whose
//      eigenvalues lie within 1e-2 ||T|| of lambda.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "mca_internal.h"

namespace mca {
namespace {

// Number of eigenvalues of T strictly below x[j] (the negative pivots of the
// LDL^T factorisation of T - x[j] I), for kG shifts at once: kG independent
// recurrences in one pass over the matrix, so that the divisions of different
// shifts overlap (one shift's recurrence is a chain of dependent divisions).
constexpr int kG = 16;
void sturm_counts(int n, const double *a, const double *b2, const double *x, double pivmin,
                  int *count)
{
    double q[kG];
    for (int j = 0; j < kG; ++j) {
        q[j] = a[0] - x[j];
        if (std::fabs(q[j]) < pivmin) q[j] = -pivmin;
        count[j] = (q[j] < 0) ? 1 : 0;
    }
    for (int i = 1; i < n; ++i) {
        const double ai = a[i], bi = b2[i - 1];
        for (int j = 0; j < kG; ++j) {
            double v = ai - x[j] - bi / q[j];
            if (std::fabs(v) < pivmin) v = -pivmin;
            q[j] = v;
            count[j] += (v < 0) ? 1 : 0;
        }
    }
}

// Solve (T - lam I) x = rhs in place by Gaussian elimination with partial
// pivoting.  Column i has nonzeros only in rows i and i+1, so each step picks
// the larger of the two as the pivot row; the upper factor has two
// superdiagonals (u1, u2).  A zero pivot is replaced by eps3 (the usual
// inverse-iteration safeguard).
void shifted_solve(int n, const double *a, const double *b, double lam, double eps3,
                   std::vector<double> &x, std::vector<double> &u0, std::vector<double> &u1,
                   std::vector<double> &u2, std::vector<double> &mult,
                   std::vector<char> &swapped)
{
    // current row at position i, entries in columns i, i+1, i+2
    double c0 = a[0] - lam, c1 = (n > 1) ? b[0] : 0.0, c2 = 0.0;
    for (int i = 0; i + 1 < n; ++i) {
        double n0 = b[i], n1 = a[i + 1] - lam, n2 = (i + 2 < n) ? b[i + 1] : 0.0;
        double p0, p1, p2, o0, o1, o2;
        if (std::fabs(n0) > std::fabs(c0)) {
            p0 = n0; p1 = n1; p2 = n2; o0 = c0; o1 = c1; o2 = c2;
            swapped[i] = 1;
        } else {
            p0 = c0; p1 = c1; p2 = c2; o0 = n0; o1 = n1; o2 = n2;
            swapped[i] = 0;
        }
        if (p0 == 0.0) p0 = eps3;
        u0[i] = p0; u1[i] = p1; u2[i] = p2;
        double f = o0 / p0;
        mult[i] = f;
        c0 = o1 - f * p1;
        c1 = o2 - f * p2;
        c2 = 0.0;
    }
    if (c0 == 0.0) c0 = eps3;
    u0[n - 1] = c0; u1[n - 1] = 0.0; u2[n - 1] = 0.0;
    for (int i = 0; i + 1 < n; ++i) {
        if (swapped[i]) std::swap(x[i], x[i + 1]);
        x[i + 1] -= mult[i] * x[i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        if (i + 1 < n) s -= u1[i] * x[i + 1];
        if (i + 2 < n) s -= u2[i] * x[i + 2];
        x[i] = s / u0[i];
    }
}

}  // namespace

void tridiag_eigen(int n, const double *a, const double *b, double *lam, double *Q)
{
    if (n == 1) {
        lam[0] = a[0];
        Q[0] = 1.0;
        return;
    }
    std::vector<double> b2(n - 1);
    double tnorm = 0.0, lo = a[0], hi = a[0];
    for (int i = 0; i < n; ++i) {
        double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
        tnorm = std::max(tnorm, std::fabs(a[i]) + r);
        if (i + 1 < n) b2[i] = b[i] * b[i];
    }
    const double eps = std::numeric_limits<double>::epsilon();
    const double pivmin = std::numeric_limits<double>::min() * std::max(1.0, tnorm * tnorm);
    lo -= 2 * eps * tnorm;
    hi += 2 * eps * tnorm;

    // 1. bisection: eigenvalue k is the point where the count passes k; kG
    // eigenvalues at a time, each from the bracket [lower end of the previous
    // group's last interval, hi]
    double prev = lo;
    for (int k0 = 0; k0 < n; k0 += kG) {
        double l[kG], h[kG], x[kG];
        bool live[kG];
        int cnt[kG];
        for (int j = 0; j < kG; ++j) {
            l[j] = prev;
            h[j] = hi;
            live[j] = k0 + j < n;
        }
        while (true) {
            bool any = false;
            for (int j = 0; j < kG; ++j) {
                x[j] = 0.5 * (l[j] + h[j]);
                if (live[j] && (x[j] <= l[j] || x[j] >= h[j] ||
                                (h[j] - l[j]) <= 2 * eps * std::max(std::fabs(l[j]), std::fabs(h[j]))))
                    live[j] = false;
                any = any || live[j];
            }
            if (!any) break;
            sturm_counts(n, a, b2.data(), x, pivmin, cnt);
            for (int j = 0; j < kG; ++j)
                if (live[j]) {
                    if (cnt[j] > k0 + j) h[j] = x[j];
                    else l[j] = x[j];
                }
        }
        for (int j = 0; j < kG && k0 + j < n; ++j) {
            lam[k0 + j] = 0.5 * (l[j] + h[j]);
            prev = l[j];
        }
    }

    // 2. inverse iteration; vectors are kept contiguous in V (row k = vector k)
    const double eps3 = eps * tnorm;
    const double near = 1e-2 * tnorm;
    std::vector<double> V((size_t)n * n), x(n), u0(n), u1(n), u2(n), mult(n);
    std::vector<char> swapped(n);
    for (int k = 0; k < n; ++k) {
        // distinct start vectors give every eigenvector a nonzero component
        for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.5 * std::sin(0.7 * i + 1.3 * k);
        int first = k;
        while (first > 0 && lam[k] - lam[first - 1] <= near) --first;
        for (int it = 0; it < 3; ++it) {
            shifted_solve(n, a, b, lam[k], eps3, x, u0, u1, u2, mult, swapped);
            if (it == 2)
                for (int pass = 0; pass < 2; ++pass)
                    for (int j = first; j < k; ++j) {
                        const double *v = &V[(size_t)j * n];
                        double dot = 0.0;
                        for (int i = 0; i < n; ++i) dot += v[i] * x[i];
                        for (int i = 0; i < n; ++i) x[i] -= dot * v[i];
                    }
            double nrm = 0.0;
            for (int i = 0; i < n; ++i) nrm += x[i] * x[i];
            nrm = std::sqrt(nrm);
            if (nrm == 0.0) {   // start vector lost: restart from a unit vector
                for (int i = 0; i < n; ++i) x[i] = (i == k) ? 1.0 : 0.0;
                continue;
            }
            for (int i = 0; i < n; ++i) x[i] /= nrm;
        }
        // sign: the entry of largest magnitude is positive
        int imax = 0;
        for (int i = 1; i < n; ++i)
            if (std::fabs(x[i]) > std::fabs(x[imax]) * (1 + 1e-12)) imax = i;
        double sg = x[imax] < 0 ? -1.0 : 1.0;
        for (int i = 0; i < n; ++i) V[(size_t)k * n + i] = sg * x[i];
    }
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) Q[(size_t)i * n + k] = V[(size_t)k * n + i];
}

}  // namespace mca
