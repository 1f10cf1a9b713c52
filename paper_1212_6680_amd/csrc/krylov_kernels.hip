// Vector kernels of Algorithm 1 (Section 2) for gfx950.
//
// Each Krylov step outside the preconditioner is three fused HBM passes:
//   dots      (s_k, r_k) and, for equation (2), (s_k, q_{k-1}) where
//             q_{k-1} = A p_{k-1}, so that (s_k, r_k - r_{k-1}) = -alpha_{k-1}(s_k, q_{k-1});
//   p/q       p_k = s_k + beta_k p_{k-1} into the other p buffer, q_k = A p_k from
//             the same neighbour loads, and (p_k, q_k);
//   x/r       x += alpha p, r -= alpha q, and ||r||^2.
// Reductions are deterministic: a fixed grid of kRedBlocks blocks writes one
// partial per block (wave shuffles, then LDS across the block's waves), and
// a one-block finalize kernel sums the partials in a fixed order and advances
// the scalar recurrence on the device.
#include "smg_internal.h"

namespace smg {

namespace {

constexpr int kRB = 256;   // threads per reduction block

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sums v over the block; the result is valid in thread 0.
__device__ inline double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) s += lds[i];
    }
    __syncthreads();
    return s;
}

// (A x) at point c = (i, j, k) of the 7-point operator
__device__ inline double a7(const double *x, long long c, int i, int j, int k, int nx, int ny, int nz, double cx,
                            double cy, double cz)
{
    const long long pl = static_cast<long long>(nx) * ny;
    double v = (2.0 * (cx + cy + cz)) * x[c];
    if (i > 0) v -= cx * x[c - 1];
    if (i < nx - 1) v -= cx * x[c + 1];
    if (j > 0) v -= cy * x[c - nx];
    if (j < ny - 1) v -= cy * x[c + nx];
    if (k > 0) v -= cz * x[c - pl];
    if (k < nz - 1) v -= cz * x[c + pl];
    return v;
}

__global__ __launch_bounds__(256) void k_matvec7(const double *x, double *y, long long ld, int nx, int ny, int nz,
                                                 double cx, double cy, double cz)
{
    const int c2 = blockIdx.x * blockDim.x + threadIdx.x;
    if (c2 >= nx * ny) return;
    const int k = blockIdx.y, r = blockIdx.z;
    const int i = c2 % nx, j = c2 / nx;
    const long long c = static_cast<long long>(k) * nx * ny + c2;
    y[r * ld + c] = a7(x + r * ld, c, i, j, k, nx, ny, nz, cx, cy, cz);
}

__global__ __launch_bounds__(kRB) void k_init_resid(const double *b, const double *x, double *r, int x_zero, int nx,
                                                    int ny, int nz, double cx, double cy, double cz,
                                                    double *partials)
{
    __shared__ double lds[kRB / 64];
    const long long n = static_cast<long long>(nx) * ny * nz;
    double rr = 0.0, bb = 0.0;
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(gridDim.x) * blockDim.x) {
        const double bv = b[c];
        double rv = bv;
        if (!x_zero) {
            const int i = static_cast<int>(c % nx);
            const long long t = c / nx;
            const int j = static_cast<int>(t % ny), k = static_cast<int>(t / ny);
            rv -= a7(x, c, i, j, k, nx, ny, nz, cx, cy, cz);
        }
        r[c] = rv;
        rr += rv * rv;
        bb += bv * bv;
    }
    rr = block_sum(rr, lds);
    bb = block_sum(bb, lds);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = rr;
        partials[kRedBlocks + blockIdx.x] = bb;
    }
}

__global__ __launch_bounds__(kRB) void k_dots_sr_sq(const double *s, const double *r, const double *q, int want_sq,
                                                    long long n, double *partials)
{
    __shared__ double lds[kRB / 64];
    double sr = 0.0, sq = 0.0;
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(gridDim.x) * blockDim.x) {
        const double sv = s[c];
        sr += sv * r[c];
        if (want_sq) sq += sv * q[c];
    }
    sr = block_sum(sr, lds);
    sq = block_sum(sq, lds);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = sr;
        partials[kRedBlocks + blockIdx.x] = sq;
    }
}

__global__ __launch_bounds__(kRB) void k_update_p_q(const double *s, const double *p_old, double *p_new, double *q,
                                                    const KScalars *sc, int nx, int ny, int nz, double cx, double cy,
                                                    double cz, double *partials)
{
    __shared__ double lds[kRB / 64];
    const double beta = sc->beta;
    const long long pl = static_cast<long long>(nx) * ny;
    const long long n = pl * nz;
    double pq = 0.0;
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int i = static_cast<int>(c % nx);
        const long long t = c / nx;
        const int j = static_cast<int>(t % ny), k = static_cast<int>(t / ny);
        // p_k at c and at its neighbours, formed from s_k and p_{k-1}
        auto pv = [&](long long cc) { return beta == 0.0 ? s[cc] : s[cc] + beta * p_old[cc]; };
        const double p0 = pv(c);
        double qv = (2.0 * (cx + cy + cz)) * p0;
        if (i > 0) qv -= cx * pv(c - 1);
        if (i < nx - 1) qv -= cx * pv(c + 1);
        if (j > 0) qv -= cy * pv(c - nx);
        if (j < ny - 1) qv -= cy * pv(c + nx);
        if (k > 0) qv -= cz * pv(c - pl);
        if (k < nz - 1) qv -= cz * pv(c + pl);
        p_new[c] = p0;
        q[c] = qv;
        pq += p0 * qv;
    }
    pq = block_sum(pq, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = pq;
}

// The same pass as a z-marching stencil: a block owns a 64 x 8 (i, j) tile and
// a run of planes; p at k-1, k, k+1 stays in registers, the in-plane
// neighbours of plane k come from an LDS tile with a one-point halo (halo
// values are formed from s and p_{k-1} by the block itself).  s and p_{k-1}
// are read about once, p_k and q written once.
constexpr int kTX = 64, kTY = 8, kTileThreads = kTX * kTY;

__global__ __launch_bounds__(kTileThreads) void k_update_p_q_tiled(const double *s, const double *p_old,
                                                                   double *p_new, double *q, const KScalars *sc,
                                                                   int nx, int ny, int nz, double cx, double cy,
                                                                   double cz, int kchunk, double *partials)
{
    __shared__ double tile[(kTY + 2) * (kTX + 2)];
    __shared__ double lds[kTileThreads / 64];
    const double beta = sc->beta;
    const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
    const int i = blockIdx.x * kTX + tx, j = blockIdx.y * kTY + ty;
    const bool in = i < nx && j < ny;
    const long long pl = static_cast<long long>(nx) * ny;
    const long long c2 = static_cast<long long>(j) * nx + i;
    const int k0 = blockIdx.z * kchunk, k1 = min(nz, k0 + kchunk);
    auto pv = [&](long long c) { return beta == 0.0 ? s[c] : s[c] + beta * p_old[c]; };
    // halo point of this thread (threads 0..143), tile coordinates (hy, hx)
    int hy = -1, hx = -1, hi = -1, hj = -1;
    const int t = threadIdx.x;
    if (t < kTX) {
        hy = 0; hx = t + 1;
    } else if (t < 2 * kTX) {
        hy = kTY + 1; hx = t - kTX + 1;
    } else if (t < 2 * kTX + kTY) {
        hy = t - 2 * kTX + 1; hx = 0;
    } else if (t < 2 * kTX + 2 * kTY) {
        hy = t - 2 * kTX - kTY + 1; hx = kTX + 1;
    }
    if (hy >= 0) {
        hi = blockIdx.x * kTX + hx - 1;
        hj = blockIdx.y * kTY + hy - 1;
    }
    const bool hin = hy >= 0 && hi >= 0 && hi < nx && hj >= 0 && hj < ny;
    const long long hc2 = static_cast<long long>(hj) * nx + hi;
    const double diag = 2.0 * (cx + cy + cz);
    double pm = (in && k0 > 0 && k0 < nz) ? pv((k0 - 1) * pl + c2) : 0.0;
    double pc = (in && k0 < nz) ? pv(k0 * pl + c2) : 0.0;
    double pq = 0.0;
    for (int k = k0; k < k1; ++k) {
        const double pn = (in && k + 1 < nz) ? pv((k + 1) * pl + c2) : 0.0;
        tile[(ty + 1) * (kTX + 2) + tx + 1] = pc;
        if (hy >= 0) tile[hy * (kTX + 2) + hx] = hin ? pv(k * pl + hc2) : 0.0;
        __syncthreads();
        if (in) {
            const int cc = (ty + 1) * (kTX + 2) + tx + 1;
            const double qv = diag * pc - cx * (tile[cc - 1] + tile[cc + 1]) -
                              cy * (tile[cc - (kTX + 2)] + tile[cc + (kTX + 2)]) - cz * (pm + pn);
            p_new[k * pl + c2] = pc;
            q[k * pl + c2] = qv;
            pq += pc * qv;
        }
        __syncthreads();
        pm = pc;
        pc = pn;
    }
    pq = block_sum(pq, lds);
    const int nb = gridDim.x * gridDim.y * gridDim.z;
    const int bid = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    if (threadIdx.x == 0) partials[bid] = pq;
    if (bid == 0)
        for (int e = nb + threadIdx.x; e < kRedBlocks; e += blockDim.x) partials[e] = 0.0;
}

// r = b - A x with partial sums of r^2 and b^2 (x tiled through LDS, marching
// in z like k_update_p_q_tiled); block 0 zeroes the unused partial slots.
__global__ __launch_bounds__(kTileThreads) void k_resid_tiled(const double *b, const double *x, double *r, int nx,
                                                              int ny, int nz, double cx, double cy, double cz,
                                                              int kchunk, double *partials)
{
    __shared__ double tile[(kTY + 2) * (kTX + 2)];
    __shared__ double lds[kTileThreads / 64];
    const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
    const int i = blockIdx.x * kTX + tx, j = blockIdx.y * kTY + ty;
    const bool in = i < nx && j < ny;
    const long long pl = static_cast<long long>(nx) * ny;
    const long long c2 = static_cast<long long>(j) * nx + i;
    const int k0 = blockIdx.z * kchunk, k1 = min(nz, k0 + kchunk);
    int hy = -1, hx = -1, hi = -1, hj = -1;
    const int t = threadIdx.x;
    if (t < kTX) {
        hy = 0; hx = t + 1;
    } else if (t < 2 * kTX) {
        hy = kTY + 1; hx = t - kTX + 1;
    } else if (t < 2 * kTX + kTY) {
        hy = t - 2 * kTX + 1; hx = 0;
    } else if (t < 2 * kTX + 2 * kTY) {
        hy = t - 2 * kTX - kTY + 1; hx = kTX + 1;
    }
    if (hy >= 0) {
        hi = blockIdx.x * kTX + hx - 1;
        hj = blockIdx.y * kTY + hy - 1;
    }
    const bool hin = hy >= 0 && hi >= 0 && hi < nx && hj >= 0 && hj < ny;
    const long long hc2 = static_cast<long long>(hj) * nx + hi;
    const double diag = 2.0 * (cx + cy + cz);
    double xm = (in && k0 > 0 && k0 < nz) ? x[(k0 - 1) * pl + c2] : 0.0;
    double xc = (in && k0 < nz) ? x[k0 * pl + c2] : 0.0;
    double rr = 0.0, bb = 0.0;
    for (int k = k0; k < k1; ++k) {
        const double xn = (in && k + 1 < nz) ? x[(k + 1) * pl + c2] : 0.0;
        tile[(ty + 1) * (kTX + 2) + tx + 1] = xc;
        if (hy >= 0) tile[hy * (kTX + 2) + hx] = hin ? x[k * pl + hc2] : 0.0;
        __syncthreads();
        if (in) {
            const int cc = (ty + 1) * (kTX + 2) + tx + 1;
            const double ax = diag * xc - cx * (tile[cc - 1] + tile[cc + 1]) -
                              cy * (tile[cc - (kTX + 2)] + tile[cc + (kTX + 2)]) - cz * (xm + xn);
            const double bv = b[k * pl + c2];
            const double rv = bv - ax;
            r[k * pl + c2] = rv;
            rr += rv * rv;
            bb += bv * bv;
        }
        __syncthreads();
        xm = xc;
        xc = xn;
    }
    rr = block_sum(rr, lds);
    bb = block_sum(bb, lds);
    const int nb = gridDim.x * gridDim.y * gridDim.z;
    const int bid = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    if (threadIdx.x == 0) {
        partials[bid] = rr;
        partials[kRedBlocks + bid] = bb;
    }
    if (bid == 0)
        for (int e = nb + threadIdx.x; e < kRedBlocks; e += blockDim.x) {
            partials[e] = 0.0;
            partials[kRedBlocks + e] = 0.0;
        }
}

__global__ __launch_bounds__(kRB) void k_update_xr(double *x, double *r, const double *p, const double *q,
                                                   const KScalars *sc, long long n, double *partials)
{
    __shared__ double lds[kRB / 64];
    const double alpha = sc->alpha;
    double rr = 0.0;
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(gridDim.x) * blockDim.x) {
        x[c] += alpha * p[c];
        const double rv = r[c] - alpha * q[c];
        r[c] = rv;
        rr += rv * rv;
    }
    rr = block_sum(rr, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = rr;
}

__device__ inline double sum_partials(const double *p, double *lds)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) v += p[i];
    return block_sum(v, lds);
}

// method: 0 = PCG (1), 1 = FPCG (2), 2 = PSD
__global__ __launch_bounds__(kRB) void k_finalize(int which, int method, int k, const double *partials,
                                                  KScalars *sc)
{
    __shared__ double lds[kRB / 64];
    const double v0 = sum_partials(partials, lds);
    const double v1 = (which <= 1) ? sum_partials(partials + kRedBlocks, lds) : 0.0;
    if (threadIdx.x != 0) return;
    if (which == 0) {
        sc->rr = v0;
        sc->bb = v1;
        sc->breakdown = 0;
        sc->sr_prev = 0.0;
        sc->alpha_prev = 0.0;
    } else if (which == 1) {
        sc->sr = v0;
        sc->sq = v1;
        double beta = 0.0;
        if (k > 0 && method == 0) beta = v0 / sc->sr_prev;
        if (k > 0 && method == 1) beta = -sc->alpha_prev * v1 / sc->sr_prev;
        // first check of an iteration: a re-evaluation with another s_k replaces it
        sc->breakdown = (!isfinite(beta) || !isfinite(v0)) ? 1 : 0;
        sc->beta = beta;
    } else if (which == 2) {
        sc->pq = v0;
        const double alpha = sc->sr / v0;
        if (!isfinite(alpha)) sc->breakdown = 1;
        sc->alpha = alpha;
        sc->alpha_prev = alpha;
        sc->sr_prev = sc->sr;
    } else {
        sc->rr = v0;
    }
}

__global__ void k_copy(const double *src, double *dst, long long n)
{
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(gridDim.x) * blockDim.x)
        dst[c] = src[c];
}

__global__ void k_fill(double *dst, double v, long long n)
{
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(gridDim.x) * blockDim.x)
        dst[c] = v;
}

}  // namespace

void launch_fill(double *dst, double v, size_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill, dim3(kRedBlocks), dim3(256), 0, st, dst, v, static_cast<long long>(n));
}

void launch_matvec7(const double *x, double *y, long long ld, int nrhs, int nx, int ny, int nz, double cx, double cy,
                    double cz, hipStream_t st)
{
    const dim3 grid((nx * ny + 255) / 256, nz, nrhs);
    hipLaunchKernelGGL(k_matvec7, grid, dim3(256), 0, st, x, y, ld, nx, ny, nz, cx, cy, cz);
}

void launch_init_resid(const double *b, const double *x, double *r, int x_zero, int nx, int ny, int nz, double cx,
                       double cy, double cz, double *partials, hipStream_t st)
{
    const int gx = (nx + kTX - 1) / kTX, gy = (ny + kTY - 1) / kTY;
    if (!x_zero && gx * gy <= kRedBlocks) {
        int gz = kRedBlocks / (gx * gy);
        gz = gz < 1 ? 1 : (gz > nz ? nz : gz);
        const int kchunk = (nz + gz - 1) / gz;
        gz = (nz + kchunk - 1) / kchunk;
        hipLaunchKernelGGL(k_resid_tiled, dim3(gx, gy, gz), dim3(kTileThreads), 0, st, b, x, r, nx, ny, nz, cx, cy,
                           cz, kchunk, partials);
        return;
    }
    hipLaunchKernelGGL(k_init_resid, dim3(kRedBlocks), dim3(kRB), 0, st, b, x, r, x_zero, nx, ny, nz, cx, cy, cz,
                       partials);
}

void launch_dots_sr_sq(const double *s, const double *r, const double *q, int want_sq, size_t n, double *partials,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_dots_sr_sq, dim3(kRedBlocks), dim3(kRB), 0, st, s, r, q, want_sq,
                       static_cast<long long>(n), partials);
}

void launch_update_p_q(const double *s, const double *p_old, double *p_new, double *q, const KScalars *sc, int nx,
                       int ny, int nz, double cx, double cy, double cz, double *partials, hipStream_t st)
{
    const int gx = (nx + kTX - 1) / kTX, gy = (ny + kTY - 1) / kTY;
    if (gx * gy <= kRedBlocks) {
        int gz = kRedBlocks / (gx * gy);
        gz = gz < 1 ? 1 : (gz > nz ? nz : gz);
        const int kchunk = (nz + gz - 1) / gz;
        gz = (nz + kchunk - 1) / kchunk;
        hipLaunchKernelGGL(k_update_p_q_tiled, dim3(gx, gy, gz), dim3(kTileThreads), 0, st, s, p_old, p_new, q, sc,
                           nx, ny, nz, cx, cy, cz, kchunk, partials);
        return;
    }
    hipLaunchKernelGGL(k_update_p_q, dim3(kRedBlocks), dim3(kRB), 0, st, s, p_old, p_new, q, sc, nx, ny, nz, cx, cy,
                       cz, partials);
}

void launch_update_xr(double *x, double *r, const double *p, const double *q, const KScalars *sc, size_t n,
                      double *partials, hipStream_t st)
{
    hipLaunchKernelGGL(k_update_xr, dim3(kRedBlocks), dim3(kRB), 0, st, x, r, p, q, sc, static_cast<long long>(n),
                       partials);
}

void launch_finalize(int which, int method, int k, const double *partials, KScalars *sc, KScalars *host_copy,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRB), 0, st, which, method, k, partials, sc);
    if (host_copy) (void)hipMemcpyAsync(host_copy, sc, sizeof(KScalars), hipMemcpyDeviceToHost, st);
}

void launch_copy(const double *src, double *dst, size_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy, dim3(kRedBlocks), dim3(256), 0, st, src, dst, static_cast<long long>(n));
}

void launch_true_resid(const double *b, const double *x, double *tmp, int nx, int ny, int nz, double cx, double cy,
                       double cz, double *partials, hipStream_t st)
{
    launch_init_resid(b, x, tmp, 0, nx, ny, nz, cx, cy, cz, partials, st);
}

}  // namespace smg
