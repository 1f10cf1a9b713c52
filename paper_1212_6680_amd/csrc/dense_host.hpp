// Small dense FP64 linear algebra on the host for LOBPCG's Rayleigh-Ritz
// step (matrices of order <= 3m, a few hundred): Cholesky factorisation,
// triangular inverse and the symmetric eigenproblem.
//
// The eigensolver is the textbook two-phase method (Golub and Van Loan,
// "Matrix Computations", Householder tridiagonalisation followed by the
// implicit symmetric QR iteration with Wilkinson shifts), with the bulge
// chased by Givens rotations and all transformations accumulated into the
// eigenvector matrix.  Storage is row-major, A[i*n + j].
#pragma once

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace smg {
namespace dense {

// A = L L^T; L overwrites the lower triangle (upper set to 0).  Returns false
// on a non-positive pivot or when (max L_ii / min L_ii)^2, a lower bound of
// cond(A), exceeds max_cond.
inline bool cholesky(int n, double *A, double max_cond = 1e14)
{
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        const double ljj = std::sqrt(d);
        A[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = s / ljj;
        }
        for (int k = j + 1; k < n; ++k) A[j * n + k] = 0.0;
    }
    double mx = 0.0, mn = INFINITY;
    for (int j = 0; j < n; ++j) {
        mx = std::max(mx, A[j * n + j]);
        mn = std::min(mn, A[j * n + j]);
    }
    return (mx / mn) * (mx / mn) <= max_cond;
}

// out = L^{-T} for lower-triangular L (so out is upper triangular).
inline void inv_lower_transpose(int n, const double *L, double *out)
{
    std::vector<double> X(static_cast<size_t>(n) * n, 0.0);   // X = L^{-1}, lower
    for (int j = 0; j < n; ++j) {
        X[j * n + j] = 1.0 / L[j * n + j];
        for (int i = j + 1; i < n; ++i) {
            double s = 0.0;
            for (int k = j; k < i; ++k) s += L[i * n + k] * X[k * n + j];
            X[i * n + j] = -s / L[i * n + i];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) out[i * n + j] = X[j * n + i];
}

// Symmetric eigendecomposition: on entry A holds a symmetric matrix, on exit
// V (row-major, eigenvectors in columns) and w (ascending).
inline bool sym_eig(int n, const double *A, double *V, double *w)
{
    std::vector<double> T(A, A + static_cast<size_t>(n) * n);
    // Q is kept transposed (row j of Qt is column j of Q), so that a rotation
    // of two columns and a reflection both run over contiguous rows
    std::vector<double> Qt(static_cast<size_t>(n) * n, 0.0);
    for (int i = 0; i < n; ++i) Qt[i * n + i] = 1.0;
    auto t = [&](int i, int j) -> double & { return T[static_cast<size_t>(i) * n + j]; };
    auto qrow = [&](int j) { return Qt.data() + static_cast<size_t>(j) * n; };

    // Phase 1: Householder reflections H_k = I - beta v v^T zero column k
    // below the subdiagonal; T <- H T H, Q <- Q H.
    std::vector<double> v(n), p(n), wv(n);
    for (int k = 0; k + 2 < n; ++k) {
        double alpha = 0.0;
        for (int i = k + 1; i < n; ++i) alpha += t(i, k) * t(i, k);
        alpha = std::sqrt(alpha);
        if (alpha == 0.0) continue;
        const double x0 = t(k + 1, k);
        const double r = x0 >= 0 ? -alpha : alpha;   // target value, sign avoids cancellation
        std::fill(v.begin(), v.end(), 0.0);
        v[k + 1] = x0 - r;
        for (int i = k + 2; i < n; ++i) v[i] = t(i, k);
        double vv = 0.0;
        for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        const double beta = 2.0 / vv;
        // p = beta * T v (on the trailing block, rows/cols >= k)
        for (int i = k; i < n; ++i) {
            double s = 0.0;
            for (int j = k + 1; j < n; ++j) s += t(i, j) * v[j];
            p[i] = beta * s;
        }
        double pv = 0.0;
        for (int i = k + 1; i < n; ++i) pv += p[i] * v[i];
        const double half = 0.5 * beta * pv;
        for (int i = k; i < n; ++i) wv[i] = p[i] - half * v[i];
        // T <- T - v w^T - w v^T on rows/cols >= k (v[k] = 0)
        for (int i = k; i < n; ++i)
            for (int j = k; j < n; ++j) t(i, j) -= v[i] * wv[j] + wv[i] * v[j];
        // Q <- Q H: s_i = beta sum_j Q(i, j) v_j, then Q(i, j) -= s_i v_j
        std::fill(p.begin(), p.end(), 0.0);
        for (int j = k + 1; j < n; ++j) {
            const double vj = v[j];
            const double *qj = qrow(j);
            for (int i = 0; i < n; ++i) p[i] += qj[i] * vj;
        }
        for (int j = k + 1; j < n; ++j) {
            const double vj = v[j];
            double *qj = qrow(j);
            for (int i = 0; i < n; ++i) qj[i] -= beta * p[i] * vj;
        }
    }
    std::vector<double> d(n), e(n > 1 ? n - 1 : 1, 0.0);
    for (int i = 0; i < n; ++i) d[i] = t(i, i);
    for (int i = 0; i + 1 < n; ++i) e[i] = t(i + 1, i);

    // Phase 2: implicit symmetric QR steps with Wilkinson shifts on the
    // unreduced trailing block [l, m].  The rotation R = [[c, s], [-s, c]] in
    // the (k, k+1) plane is applied as T <- R T R^T, Q <- Q R^T.
    const double eps = 2.220446049250313e-16;
    int m = n - 1, guard = 0;
    while (m > 0) {
        if (std::fabs(e[m - 1]) <= eps * (std::fabs(d[m - 1]) + std::fabs(d[m]))) {
            e[m - 1] = 0.0;
            --m;
            continue;
        }
        int l = m - 1;
        while (l > 0 && std::fabs(e[l - 1]) > eps * (std::fabs(d[l - 1]) + std::fabs(d[l]))) --l;
        if (++guard > 60 * n) return false;
        const double a = d[m - 1], b = e[m - 1], c0 = d[m];
        const double delta = 0.5 * (a - c0);
        const double denom = delta + std::copysign(std::hypot(delta, b), delta == 0.0 ? 1.0 : delta);
        const double mu = c0 - b * b / denom;
        double x = d[l] - mu, z = e[l];
        double bulge = 0.0;
        for (int k = l; k < m; ++k) {
            const double r = std::hypot(x, z);
            const double c = r == 0.0 ? 1.0 : x / r, s = r == 0.0 ? 0.0 : z / r;
            // rows/cols k, k+1 of the band; bulge lives at (k+1, k-1) before
            // this rotation and moves to (k+2, k) after it
            if (k > l) e[k - 1] = c * e[k - 1] + s * bulge;
            const double dk = d[k], dk1 = d[k + 1], ek = e[k];
            d[k] = c * c * dk + 2.0 * c * s * ek + s * s * dk1;
            d[k + 1] = s * s * dk - 2.0 * c * s * ek + c * c * dk1;
            e[k] = c * s * (dk1 - dk) + (c * c - s * s) * ek;
            if (k + 1 < m) {
                const double ek1 = e[k + 1];
                bulge = s * ek1;
                e[k + 1] = c * ek1;
                x = e[k];
                z = bulge;
            }
            double *qa = qrow(k), *qb = qrow(k + 1);
            for (int i = 0; i < n; ++i) {
                const double qk = qa[i], qk1 = qb[i];
                qa[i] = c * qk + s * qk1;
                qb[i] = -s * qk + c * qk1;
            }
        }
    }
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int i, int j) { return d[i] < d[j]; });
    for (int jj = 0; jj < n; ++jj) {
        w[jj] = d[ord[jj]];
        const double *qj = qrow(ord[jj]);
        for (int i = 0; i < n; ++i) V[static_cast<size_t>(i) * n + jj] = qj[i];
    }
    return true;
}

}  // namespace dense
}  // namespace smg
