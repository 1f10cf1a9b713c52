// Section 5 diagnostics on the GPU: the quality of a preconditioner T in the
// sense of assumption (4), ||I - c A T||_{A^{-1}} <= delta < 1, and the
// extreme eigenvalues of T A behind Theorem 2's prescaling.
//
// With r = A e, ||r||_{A^{-1}} = ||e||_A and (I - c A T) A e = A (I - c T A) e,
// so delta(c) = ||E||_A with E = I - c T A.  Its A-adjoint is
// E# = A^{-1} E^T A = I - c T^T A, and ||E||_A^2 is the largest eigenvalue of
// E# E, which is self-adjoint and non-negative in the A inner product: power
// iteration on it, normalised in the A-norm, gives Rayleigh quotients
// ||E v||_A^2 / ||v||_A^2 that increase to delta(c)^2.  For an SPD T
// (equal pre- and post-smoothing) T A is self-adjoint in the A inner product;
// power iteration on T A gives lambda_max, and on lambda_max I - T A gives
// lambda_max - lambda_min.  Every step is one or two V-cycles, stencil passes
// and deterministic dot products; the host keeps the scalars.
#include <cmath>

#include "smg_internal.h"

namespace {

using smg::device_dot2;
using smg::launch_axpby;

struct Vecs {
    size_t n;
    hipStream_t st;
    double *part;
};

// (a, b)
int dot(const Vecs &V, const double *a, const double *b, double *out)
{
    return device_dot2(a, b, nullptr, nullptr, V.n, V.part, V.st, out, nullptr);
}

}  // namespace

extern "C" {

int smg_delta(smg_handle *h, smg_handle *ht, double c, const double *v0, int32_t iters, double *work, double *delta,
              void *stream)
{
    if (!h || !ht || !v0 || !work || !delta || iters < 1 || !std::isfinite(c)) return SMG_EINVAL;
    size_t n = 0, nt = 0;
    if (smg_handle_size(h, &n) != SMG_OK || smg_handle_size(ht, &nt) != SMG_OK || n != nt) return SMG_EINVAL;
    const smg_grid *g = smg_handle_grid(h), *gt = smg_handle_grid(ht);
    if (g->nx != gt->nx || g->ny != gt->ny || g->nz != gt->nz || g->cx != gt->cx || g->cy != gt->cy ||
        g->cz != gt->cz)
        return SMG_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *v = work, *w = work + n, *t = work + 2 * n, *u = work + 3 * n, *au = work + 4 * n;
    double *part = smg::handle_partials(h);
    const Vecs V{n, st, part};
    const long long ld = static_cast<long long>(n);
    // v = v0 / ||v0||_A, w = A v
    launch_axpby(v, v0, 1.0, v0, 0.0, n, st);
    if (smg_matvec(h, v, w, 1, ld, stream) != SMG_OK) return SMG_EHIP;
    double vv = 0.0;
    if (dot(V, v, w, &vv) != SMG_OK) return SMG_EHIP;
    if (!(vv > 0.0) || !std::isfinite(vv)) return SMG_EINVAL;
    double sc = 1.0 / std::sqrt(vv);
    launch_axpby(v, v, sc, v, 0.0, n, st);
    launch_axpby(w, w, sc, w, 0.0, n, st);
    double q = 0.0;
    for (int it = 0; it < iters; ++it) {
        // u = E v = v - c T (A v); ||u||_A^2 = (u, A u) with ||v||_A = 1
        if (smg_apply(h, w, t, 1, ld, stream) != SMG_OK) return SMG_EHIP;
        launch_axpby(u, v, 1.0, t, -c, n, st);
        if (smg_matvec(h, u, au, 1, ld, stream) != SMG_OK) return SMG_EHIP;
        if (dot(V, u, au, &q) != SMG_OK) return SMG_EHIP;
        if (!std::isfinite(q)) return SMG_EBREAKDOWN;
        if (it + 1 == iters) break;
        // y = E# u = u - c T^T (A u), then v = y / ||y||_A and w = A v
        if (smg_apply(ht, au, t, 1, ld, stream) != SMG_OK) return SMG_EHIP;
        launch_axpby(v, u, 1.0, t, -c, n, st);
        if (smg_matvec(h, v, w, 1, ld, stream) != SMG_OK) return SMG_EHIP;
        double yy = 0.0;
        if (dot(V, v, w, &yy) != SMG_OK) return SMG_EHIP;
        if (!(yy > 0.0) || !std::isfinite(yy)) break;      // E# E v = 0: q is exact
        sc = 1.0 / std::sqrt(yy);
        launch_axpby(v, v, sc, v, 0.0, n, st);
        launch_axpby(w, w, sc, w, 0.0, n, st);
    }
    *delta = std::sqrt(std::fabs(q));
    return hipGetLastError() == hipSuccess ? SMG_OK : SMG_EHIP;
}

int smg_delta_min(smg_handle *h, smg_handle *ht, double c_lo, double c_hi, double tol, const double *v0,
                  int32_t iters, double *work, double *c_best, double *delta, void *stream)
{
    if (!(c_lo > 0.0) || !(c_hi > c_lo) || !(tol > 0.0) || !c_best || !delta) return SMG_EINVAL;
    // golden-section search: delta(c) = ||I - c T A||_A is convex in c
    const double g = 0.5 * (std::sqrt(5.0) - 1.0);
    double a = c_lo, b = c_hi;
    double x1 = b - g * (b - a), x2 = a + g * (b - a), f1 = 0.0, f2 = 0.0;
    int rc = smg_delta(h, ht, x1, v0, iters, work, &f1, stream);
    if (rc != SMG_OK) return rc;
    rc = smg_delta(h, ht, x2, v0, iters, work, &f2, stream);
    if (rc != SMG_OK) return rc;
    while (b - a > tol * 0.5 * (a + b)) {
        if (f1 <= f2) {
            b = x2;
            x2 = x1;
            f2 = f1;
            x1 = b - g * (b - a);
            rc = smg_delta(h, ht, x1, v0, iters, work, &f1, stream);
        } else {
            a = x1;
            x1 = x2;
            f1 = f2;
            x2 = a + g * (b - a);
            rc = smg_delta(h, ht, x2, v0, iters, work, &f2, stream);
        }
        if (rc != SMG_OK) return rc;
    }
    *c_best = f1 <= f2 ? x1 : x2;
    *delta = f1 <= f2 ? f1 : f2;
    return SMG_OK;
}

int smg_spectrum(smg_handle *h, const double *v0, int32_t iters, double *work, double *lmin, double *lmax,
                 void *stream)
{
    if (!h || !v0 || !work || !lmin || !lmax || iters < 1) return SMG_EINVAL;
    size_t n = 0;
    if (smg_handle_size(h, &n) != SMG_OK) return SMG_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *v = work, *w = work + n, *t = work + 2 * n;
    const Vecs V{n, st, smg::handle_partials(h)};
    const long long ld = static_cast<long long>(n);
    // power iteration on M = shift I - T A in the A inner product:
    // v <- M v / ||M v||_A, Rayleigh quotient (v, A M v) = shift - (A v, T A v)
    auto power = [&](double shift, double *out) {
        launch_axpby(v, v0, 1.0, v0, 0.0, n, st);
        if (smg_matvec(h, v, w, 1, ld, stream) != SMG_OK) return SMG_EHIP;
        double vv = 0.0;
        if (dot(V, v, w, &vv) != SMG_OK) return SMG_EHIP;
        if (!(vv > 0.0) || !std::isfinite(vv)) return SMG_EINVAL;
        double sc = 1.0 / std::sqrt(vv);
        launch_axpby(v, v, sc, v, 0.0, n, st);
        launch_axpby(w, w, sc, w, 0.0, n, st);
        double q = 0.0;
        for (int it = 0; it < iters; ++it) {
            if (smg_apply(h, w, t, 1, ld, stream) != SMG_OK) return SMG_EHIP;   // t = T A v
            double wt = 0.0;
            if (dot(V, w, t, &wt) != SMG_OK) return SMG_EHIP;
            q = shift - wt;
            if (it + 1 == iters) break;
            // v = M v = shift v - t, then w = A v afresh (updating w by the
            // same recurrence loses the match to A v through cancellation,
            // amplified by every normalisation)
            launch_axpby(v, v, shift, t, -1.0, n, st);
            if (smg_matvec(h, v, w, 1, ld, stream) != SMG_OK) return SMG_EHIP;
            double yy = 0.0;
            if (dot(V, v, w, &yy) != SMG_OK) return SMG_EHIP;
            if (!(yy > 0.0) || !std::isfinite(yy)) break;
            sc = 1.0 / std::sqrt(yy);
            launch_axpby(v, v, sc, v, 0.0, n, st);
            launch_axpby(w, w, sc, w, 0.0, n, st);
        }
        *out = q;
        return SMG_OK;
    };
    double qmax = 0.0, qd = 0.0;
    int rc = power(0.0, &qmax);          // shift 0: -lambda_max(T A)
    if (rc != SMG_OK) return rc;
    const double lm = -qmax;
    rc = power(lm, &qd);                 // lambda_max - lambda_min
    if (rc != SMG_OK) return rc;
    *lmax = lm;
    *lmin = lm - qd;
    return hipGetLastError() == hipSuccess ? SMG_OK : SMG_EHIP;
}

}  // extern "C"
