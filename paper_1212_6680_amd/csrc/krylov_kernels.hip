// Vector kernels of Algorithm 1 (Section 2) for gfx950.
//
// Each Krylov step outside the preconditioner is three fused HBM passes:
//   dots      (s_k, r_k) and, for equation (2), (s_k, q_{k-1}) where
//             q_{k-1} = A p_{k-1}, so that (s_k, r_k - r_{k-1}) = -alpha_{k-1}(s_k, q_{k-1});
//   p/q       p_k = s_k + beta_k p_{k-1} into the other p buffer, q_k = A p_k from
//             the same neighbour loads, and (p_k, q_k);
//   x/r       x += alpha p, r -= alpha q, and ||r||^2.
// When the FP64 V-cycle ends in the 3D prolongation chain (no post-smoothing),
// that kernel takes the dots as it stores s_k and the dots pass is skipped;
// finalize then sums its per-block partials (FinArgs::nparts).
// Reductions are deterministic: a fixed grid of kRedBlocks blocks writes one
// partial per block (wave shuffles, then LDS across the block's waves), and
// a one-block finalize kernel sums the partials in a fixed order and advances
// the scalar recurrence on the device.
#include <vector>

#include "group.h"
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


#define SMG_GROUPED_KERNEL_B(NAME, BOUNDS, ARGS, BLK)                                          \
    __global__ __launch_bounds__(BOUNDS) void NAME(ARGS a) { NAME##_body(a, BLK); }            \
    __global__ __launch_bounds__(BOUNDS) void NAME##_grp(const GroupEntry *tab, int n)         \
    {                                                                                          \
        const ARGS *a;                                                                         \
        Blk blk;                                                                               \
        if (!group_entry(tab, n, a, blk)) return;                                              \
        NAME##_body(*a, blk);                                                                  \
    }

#define SMG_GROUPED_KERNEL(NAME, BOUNDS, ARGS) SMG_GROUPED_KERNEL_B(NAME, BOUNDS, ARGS, SMG_BLK_HW)
// plain launches of the tiled stencil passes take XCD-grouped block numbers
#define SMG_GROUPED_KERNEL_XCD(NAME, BOUNDS, ARGS) SMG_GROUPED_KERNEL_B(NAME, BOUNDS, ARGS, SMG_BLK_XCD)

// r = b - A x (or r = b when x_zero) and partial sums of r^2, b^2; grid-stride
__device__ __forceinline__ void k_init_resid_body(const ResidArgs &a, const Blk &blk)
{
    __shared__ double lds[kRB / 64];
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long long n = static_cast<long long>(nx) * ny * nz;
    double rr = 0.0, bb = 0.0;
    for (long long c = static_cast<long long>(blk.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(blk.gx) * blockDim.x) {
        const double bv = a.b[c];
        double rv = bv;
        if (!a.x_zero) {
            const int i = static_cast<int>(c % nx);
            const long long t = c / nx;
            const int j = static_cast<int>(t % ny), k = static_cast<int>(t / ny);
            rv -= a7(a.x, c, i, j, k, nx, ny, nz, a.cx, a.cy, a.cz);
        }
        a.r[c] = rv;
        rr += rv * rv;
        bb += bv * bv;
    }
    rr = block_sum(rr, lds);
    bb = block_sum(bb, lds);
    if (threadIdx.x == 0) {
        a.partials[blk.x] = rr;
        a.partials[kRedBlocks + blk.x] = bb;
    }
}
SMG_GROUPED_KERNEL(k_init_resid, kRB, ResidArgs)

__device__ __forceinline__ void k_dots_sr_sq_body(const DotsArgs &a, const Blk &blk)
{
    __shared__ double lds[kRB / 64];
    double sr = 0.0, sq = 0.0;
    for (long long c = static_cast<long long>(blk.x) * blockDim.x + threadIdx.x; c < a.n;
         c += static_cast<long long>(blk.gx) * blockDim.x) {
        const double sv = a.s[c];
        sr += sv * a.r[c];
        if (a.want_sq) sq += sv * a.q[c];
    }
    sr = block_sum(sr, lds);
    sq = block_sum(sq, lds);
    if (threadIdx.x == 0) {
        a.partials[blk.x] = sr;
        a.partials[kRedBlocks + blk.x] = sq;
    }
}
SMG_GROUPED_KERNEL(k_dots_sr_sq, kRB, DotsArgs)

__device__ __forceinline__ void k_update_p_q_body(const UpdPQArgs &a, const Blk &blk)
{
    __shared__ double lds[kRB / 64];
    const double beta = a.sc->beta;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const double cx = a.cx, cy = a.cy, cz = a.cz;
    const double *s = a.s, *p_old = a.p_old;
    const long long pl = static_cast<long long>(nx) * ny;
    const long long n = pl * nz;
    double pq = 0.0;
    for (long long c = static_cast<long long>(blk.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(blk.gx) * blockDim.x) {
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
        a.p_new[c] = p0;
        a.q[c] = qv;
        pq += p0 * qv;
    }
    pq = block_sum(pq, lds);
    if (threadIdx.x == 0) a.partials[blk.x] = pq;
}
SMG_GROUPED_KERNEL(k_update_p_q, kRB, UpdPQArgs)

// The same pass as a z-marching stencil: a block owns a 64 x 8 (i, j) tile and
// a run of planes; p at k-1, k, k+1 stays in registers, the in-plane
// neighbours of plane k come from an LDS tile with a one-point halo (halo
// values are formed from s and p_{k-1} by the block itself).  s and p_{k-1}
// are read about once, p_k and q written once.
constexpr int kTX = 64, kTY = 8, kTileThreads = kTX * kTY;


// halo point of thread t of a kTX x kTY tile (threads 0 .. 2*(kTX+kTY)-1),
// in tile coordinates (hy, hx); -1 when the thread has none
__device__ inline void tile_halo(int t, int &hy, int &hx)
{
    hy = -1;
    hx = -1;
    if (t < kTX) {
        hy = 0; hx = t + 1;
    } else if (t < 2 * kTX) {
        hy = kTY + 1; hx = t - kTX + 1;
    } else if (t < 2 * kTX + kTY) {
        hy = t - 2 * kTX + 1; hx = 0;
    } else if (t < 2 * kTX + 2 * kTY) {
        hy = t - 2 * kTX - kTY + 1; hx = kTX + 1;
    }
}

__device__ __forceinline__ void k_update_p_q_tiled_body(const UpdPQArgs &a, const Blk &blk)
{
    __shared__ double tile[(kTY + 2) * (kTX + 2)];
    __shared__ double lds[kTileThreads / 64];
    const double beta = a.sc->beta;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const double cx = a.cx, cy = a.cy, cz = a.cz;
    const double *s = a.s, *p_old = a.p_old;
    const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
    const int i = blk.x * kTX + tx, j = blk.y * kTY + ty;
    const bool in = i < nx && j < ny;
    const long long pl = static_cast<long long>(nx) * ny;
    const long long c2 = static_cast<long long>(j) * nx + i;
    const int k0 = blk.z * a.kchunk, k1 = min(nz, k0 + a.kchunk);
    auto pv = [&](long long c) { return beta == 0.0 ? s[c] : s[c] + beta * p_old[c]; };
    int hy, hx;
    tile_halo(threadIdx.x, hy, hx);
    int hi = -1, hj = -1;
    if (hy >= 0) {
        hi = blk.x * kTX + hx - 1;
        hj = blk.y * kTY + hy - 1;
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
            a.p_new[k * pl + c2] = pc;
            a.q[k * pl + c2] = qv;
            pq += pc * qv;
        }
        __syncthreads();
        pm = pc;
        pc = pn;
    }
    pq = block_sum(pq, lds);
    const int nb = blk.gx * blk.gy * blk.gz;
    const int bid = (blk.z * blk.gy + blk.y) * blk.gx + blk.x;
    if (threadIdx.x == 0) a.partials[bid] = pq;
    if (bid == 0)
        for (int e = nb + threadIdx.x; e < kRedBlocks; e += blockDim.x) a.partials[e] = 0.0;
}
SMG_GROUPED_KERNEL_XCD(k_update_p_q_tiled, kTileThreads, UpdPQArgs)

// r = b - A x with partial sums of r^2 and b^2 (x tiled through LDS, marching
// in z like k_update_p_q_tiled); block 0 zeroes the unused partial slots.
__device__ __forceinline__ void k_resid_tiled_body(const ResidArgs &a, const Blk &blk)
{
    __shared__ double tile[(kTY + 2) * (kTX + 2)];
    __shared__ double lds[kTileThreads / 64];
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const double cx = a.cx, cy = a.cy, cz = a.cz;
    const double *x = a.x;
    const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
    const int i = blk.x * kTX + tx, j = blk.y * kTY + ty;
    const bool in = i < nx && j < ny;
    const long long pl = static_cast<long long>(nx) * ny;
    const long long c2 = static_cast<long long>(j) * nx + i;
    const int k0 = blk.z * a.kchunk, k1 = min(nz, k0 + a.kchunk);
    int hy, hx;
    tile_halo(threadIdx.x, hy, hx);
    int hi = -1, hj = -1;
    if (hy >= 0) {
        hi = blk.x * kTX + hx - 1;
        hj = blk.y * kTY + hy - 1;
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
            const double bv = a.b[k * pl + c2];
            const double rv = bv - ax;
            a.r[k * pl + c2] = rv;
            rr += rv * rv;
            bb += bv * bv;
        }
        __syncthreads();
        xm = xc;
        xc = xn;
    }
    rr = block_sum(rr, lds);
    bb = block_sum(bb, lds);
    const int nb = blk.gx * blk.gy * blk.gz;
    const int bid = (blk.z * blk.gy + blk.y) * blk.gx + blk.x;
    if (threadIdx.x == 0) {
        a.partials[bid] = rr;
        a.partials[kRedBlocks + bid] = bb;
    }
    if (bid == 0)
        for (int e = nb + threadIdx.x; e < kRedBlocks; e += blockDim.x) {
            a.partials[e] = 0.0;
            a.partials[kRedBlocks + e] = 0.0;
        }
}
SMG_GROUPED_KERNEL_XCD(k_resid_tiled, kTileThreads, ResidArgs)

// y = A x for nrhs columns, marching in z like k_update_p_q_tiled: a block
// owns a kTX x kTY tile, a run of kchunk planes and one column; x at k-1, k,
// k+1 stays in registers and the in-plane neighbours come from an LDS tile
// with a one-point halo, so x is read about once.
__global__ __launch_bounds__(kTileThreads) void k_matvec7_tiled(const double *x, double *y, long long ld, int nx,
                                                                int ny, int nz, double cx, double cy, double cz,
                                                                int kchunk, int nzb)
{
    __shared__ double tile[(kTY + 2) * (kTX + 2)];
    const Blk blk = blk_xcd();
    const int r = blk.z / nzb, zb = blk.z % nzb;
    const double *xr = x + r * ld;
    double *yr = y + r * ld;
    const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
    const int i = blk.x * kTX + tx, j = blk.y * kTY + ty;
    const bool in = i < nx && j < ny;
    const long long pl = static_cast<long long>(nx) * ny;
    const long long c2 = static_cast<long long>(j) * nx + i;
    const int k0 = zb * kchunk, k1 = min(nz, k0 + kchunk);
    int hy, hx;
    tile_halo(threadIdx.x, hy, hx);
    int hi = -1, hj = -1;
    if (hy >= 0) {
        hi = blk.x * kTX + hx - 1;
        hj = blk.y * kTY + hy - 1;
    }
    const bool hin = hy >= 0 && hi >= 0 && hi < nx && hj >= 0 && hj < ny;
    const long long hc2 = static_cast<long long>(hj) * nx + hi;
    const double diag = 2.0 * (cx + cy + cz);
    // the column's values one plane ahead of their use and the halo one plane
    // ahead of its staging, so a step's loads overlap the previous step
    auto col = [&](int k) { return (in && k >= 0 && k < nz) ? xr[k * pl + c2] : 0.0; };
    auto halo = [&](int k) { return (hin && k < k1) ? xr[k * pl + hc2] : 0.0; };
    double xm = k0 > 0 ? col(k0 - 1) : 0.0;
    double xc = col(k0), xn = col(k0 + 1), hv = halo(k0);
    for (int k = k0; k < k1; ++k) {
        const double xnn = col(k + 2), hvn = halo(k + 1);
        tile[(ty + 1) * (kTX + 2) + tx + 1] = xc;
        if (hy >= 0) tile[hy * (kTX + 2) + hx] = hv;
        __syncthreads();
        if (in) {
            const int cc = (ty + 1) * (kTX + 2) + tx + 1;
            yr[k * pl + c2] = diag * xc - cx * (tile[cc - 1] + tile[cc + 1]) -
                              cy * (tile[cc - (kTX + 2)] + tile[cc + (kTX + 2)]) - cz * (xm + xn);
        }
        __syncthreads();
        xm = xc;
        xc = xn;
        xn = xnn;
        hv = hvn;
    }
}

__device__ __forceinline__ void k_update_xr_body(const UpdXRArgs &a, const Blk &blk)
{
    __shared__ double lds[kRB / 64];
    const double alpha = a.sc->alpha;
    double rr = 0.0;
    for (long long c = static_cast<long long>(blk.x) * blockDim.x + threadIdx.x; c < a.n;
         c += static_cast<long long>(blk.gx) * blockDim.x) {
        a.x[c] += alpha * a.p[c];
        const double rv = a.r[c] - alpha * a.q[c];
        a.r[c] = rv;
        rr += rv * rv;
    }
    rr = block_sum(rr, lds);
    if (threadIdx.x == 0) a.partials[blk.x] = rr;
}
SMG_GROUPED_KERNEL(k_update_xr, kRB, UpdXRArgs)

// Block sums of p[0, np) and, with two, p[np, 2 np), valid in thread 0.  Each
// thread keeps U running sums over entries blockDim apart, advancing U
// entries at a time, so a long array (the 3D chain's per-block partials) has
// 2 U loads in flight per thread; entries past the last full step go to the
// first sum.  The order is fixed, and for np <= (U - 1) blockDim every entry
// goes to the first sum, as a plain strided loop would add them.
__device__ inline void sum_partials(const double *p, int np, bool two, double *lds, double &v0, double &v1)
{
    constexpr int U = 16;
    double a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] = b[u] = 0.0;
    const int bd = static_cast<int>(blockDim.x);
    int i = threadIdx.x;
    for (; i + (U - 1) * bd < np; i += U * bd) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] += p[i + u * bd];
            if (two) b[u] += p[np + i + u * bd];
        }
    }
    for (; i < np; i += bd) {
        a[0] += p[i];
        if (two) b[0] += p[np + i];
    }
#pragma unroll
    for (int w = U / 2; w > 0; w /= 2)
#pragma unroll
        for (int u = 0; u < w; ++u) {
            a[u] += a[u + w];
            b[u] += b[u + w];
        }
    v0 = block_sum(a[0], lds);
    v1 = two ? block_sum(b[0], lds) : 0.0;
}

// Stage 2 of the reductions and the scalar recurrence.  method: 0 = PCG (1),
// 1 = FPCG (2), 2 = PSD.  which: 0 = start (rr, bb), 1 = beta (sr, sq),
// 2 = alpha (pq), 3 = rr, 4 = true residual.  With a.batched the iteration
// index and the stopping test live on the device (KScalars::iters, active),
// using the same expressions as the host loop: ||r||/||b|| > rtol and
// iters < max_iter.
__device__ __forceinline__ void k_finalize_body(const FinArgs &a, const Blk &)
{
    __shared__ double lds[kRB / 64];
    KScalars *sc = a.sc;
    const int np = a.nparts > 0 ? a.nparts : kRedBlocks;
    double v0, v1;
    sum_partials(a.partials, np, a.which <= 1, lds, v0, v1);
    if (threadIdx.x != 0) return;
    if (a.which == 0) {
        sc->rr = v0;
        sc->bb = v1;
        sc->breakdown = 0;
        sc->sr_prev = 0.0;
        sc->alpha_prev = 0.0;
        if (a.batched) {
            const double bn = sqrt(v1);
            const double bden = bn > 0.0 ? bn : 1.0;
            sc->bden = bden;
            sc->rtol = a.rtol;
            sc->max_iter = a.max_iter;
            sc->iters = 0;
            const bool finite = isfinite(v0) && isfinite(v1);
            sc->nonfinite = finite ? 0 : 1;
            sc->active = (finite && a.max_iter > 0 && sqrt(v0) / bden > a.rtol) ? 1 : 0;
        }
    } else if (a.which == 1) {
        const int k = a.batched ? sc->iters : a.k;
        sc->sr = v0;
        sc->sq = v1;
        double beta = 0.0;
        if (k > 0 && a.method == 0) beta = v0 / sc->sr_prev;
        if (k > 0 && a.method == 1) beta = -sc->alpha_prev * v1 / sc->sr_prev;
        // first check of an iteration: a re-evaluation with another s_k replaces it
        sc->breakdown = (!isfinite(beta) || !isfinite(v0)) ? 1 : 0;
        sc->beta = beta;
    } else if (a.which == 2) {
        sc->pq = v0;
        const double alpha = sc->sr / v0;
        if (!isfinite(alpha)) sc->breakdown = 1;
        sc->alpha = alpha;
        sc->alpha_prev = alpha;
        sc->sr_prev = sc->sr;
    } else if (a.which == 3) {
        sc->rr = v0;
        if (a.batched) {
            if (sc->breakdown) {
                sc->active = 0;
            } else {
                sc->iters += 1;
                const double rel = sqrt(v0) / sc->bden;
                sc->active = (isfinite(rel) && rel > sc->rtol && sc->iters < sc->max_iter) ? 1 : 0;
            }
        }
    } else {
        sc->true_rr = v0;
    }
}
SMG_GROUPED_KERNEL(k_finalize, kRB, FinArgs)

__device__ __forceinline__ void k_copy_body(const CopyArgs &a, const Blk &blk)
{
    for (long long c = static_cast<long long>(blk.x) * blockDim.x + threadIdx.x; c < a.n;
         c += static_cast<long long>(blk.gx) * blockDim.x)
        a.dst[c] = a.src[c];
}
SMG_GROUPED_KERNEL(k_copy, 256, CopyArgs)

__device__ __forceinline__ void k_fill_body(const FillArgs &a, const Blk &blk)
{
    for (long long c = static_cast<long long>(blk.x) * blockDim.x + threadIdx.x; c < a.n;
         c += static_cast<long long>(blk.gx) * blockDim.x)
        a.dst[c] = a.v;
}
SMG_GROUPED_KERNEL(k_fill, 256, FillArgs)

// out = alpha a + beta b (grid-stride)
__global__ __launch_bounds__(256) void k_axpby(double *out, const double *a, double alpha, const double *b,
                                               double beta, long long n)
{
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(gridDim.x) * blockDim.x)
        out[c] = alpha * a[c] + beta * b[c];
}

// partial sums of (a1, b1) and (a2, b2), one slot per block (fixed grid of
// kRedBlocks blocks; a2 may be null)
__global__ __launch_bounds__(kRB) void k_dot2(const double *a1, const double *b1, const double *a2, const double *b2,
                                              long long n, double *partials)
{
    __shared__ double lds[kRB / 64];
    double d1 = 0.0, d2 = 0.0;
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(gridDim.x) * blockDim.x) {
        d1 += a1[c] * b1[c];
        if (a2) d2 += a2[c] * b2[c];
    }
    d1 = block_sum(d1, lds);
    d2 = block_sum(d2, lds);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = d1;
        partials[kRedBlocks + blockIdx.x] = d2;
    }
}

}  // namespace

void launch_axpby(double *out, const double *a, double alpha, const double *b, double beta, size_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_axpby, dim3(kRedBlocks), dim3(256), 0, st, out, a, alpha, b, beta,
                       static_cast<long long>(n));
}

int device_dot2(const double *a1, const double *b1, const double *a2, const double *b2, size_t n, double *partials,
                hipStream_t st, double *d1, double *d2)
{
    hipLaunchKernelGGL(k_dot2, dim3(kRedBlocks), dim3(kRB), 0, st, a1, b1, a2, b2, static_cast<long long>(n),
                       partials);
    std::vector<double> h(2 * kRedBlocks);
    if (hipMemcpyAsync(h.data(), partials, h.size() * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess)
        return SMG_EHIP;
    double s1 = 0.0, s2 = 0.0;
    for (int i = 0; i < kRedBlocks; ++i) {
        s1 += h[i];
        s2 += h[kRedBlocks + i];
    }
    if (d1) *d1 = s1;
    if (d2) *d2 = s2;
    return SMG_OK;
}

void launch_fill(double *dst, double v, size_t n, hipStream_t st)
{
    const FillArgs a{dst, v, static_cast<long long>(n)};
    SMG_LAUNCH_G(LaunchEv{}, k_fill, k_fill_grp, dim3(kRedBlocks), dim3(256), 0, st, a);
}

void launch_matvec7(const double *x, double *y, long long ld, int nrhs, int nx, int ny, int nz, double cx, double cy,
                    double cz, hipStream_t st)
{
    // enough blocks to fill the chip; each marches kchunk planes of one column
    const long long gx = (nx + kTX - 1) / kTX, gy = (ny + kTY - 1) / kTY;
    long long nzb = 2048 / (gx * gy * nrhs);
    nzb = nzb < 1 ? 1 : (nzb > nz ? nz : nzb);
    const int kchunk = static_cast<int>((nz + nzb - 1) / nzb);
    nzb = (nz + kchunk - 1) / kchunk;
    if (gx * gy <= 65535 && nzb * nrhs <= 65535) {
        hipLaunchKernelGGL(k_matvec7_tiled, dim3(static_cast<unsigned>(gx), static_cast<unsigned>(gy),
                                                 static_cast<unsigned>(nzb * nrhs)),
                           dim3(kTileThreads), 0, st, x, y, ld, nx, ny, nz, cx, cy, cz, kchunk, static_cast<int>(nzb));
        return;
    }
    const dim3 grid((nx * ny + 255) / 256, nz, nrhs);
    hipLaunchKernelGGL(k_matvec7, grid, dim3(256), 0, st, x, y, ld, nx, ny, nz, cx, cy, cz);
}

// z-chunking of the tiled stencil passes: at most kRedBlocks blocks, so each
// block owns one partial-sum slot
static bool tile_grid(int nx, int ny, int nz, dim3 &grid, int &kchunk)
{
    const int gx = (nx + kTX - 1) / kTX, gy = (ny + kTY - 1) / kTY;
    if (gx * gy > kRedBlocks) return false;
    int gz = kRedBlocks / (gx * gy);
    gz = gz < 1 ? 1 : (gz > nz ? nz : gz);
    kchunk = (nz + gz - 1) / gz;
    gz = (nz + kchunk - 1) / kchunk;
    grid = dim3(gx, gy, gz);
    return true;
}

void launch_init_resid(const double *b, const double *x, double *r, int x_zero, int nx, int ny, int nz, double cx,
                       double cy, double cz, double *partials, hipStream_t st)
{
    ResidArgs a{b, x, r, nx, ny, nz, cx, cy, cz, 0, x_zero, partials};
    dim3 grid;
    if (!x_zero && tile_grid(nx, ny, nz, grid, a.kchunk)) {
        SMG_LAUNCH_G(LaunchEv{}, k_resid_tiled, k_resid_tiled_grp, grid, dim3(kTileThreads), 0, st, a);
        return;
    }
    SMG_LAUNCH_G(LaunchEv{}, k_init_resid, k_init_resid_grp, dim3(kRedBlocks), dim3(kRB), 0, st, a);
}

void launch_dots_sr_sq(const double *s, const double *r, const double *q, int want_sq, size_t n, double *partials,
                       hipStream_t st)
{
    const DotsArgs a{s, r, q, want_sq, static_cast<long long>(n), partials};
    SMG_LAUNCH_G(LaunchEv{}, k_dots_sr_sq, k_dots_sr_sq_grp, dim3(kRedBlocks), dim3(kRB), 0, st, a);
}

void launch_update_p_q(const double *s, const double *p_old, double *p_new, double *q, const KScalars *sc, int nx,
                       int ny, int nz, double cx, double cy, double cz, double *partials, hipStream_t st)
{
    UpdPQArgs a{s, p_old, p_new, q, sc, nx, ny, nz, cx, cy, cz, 0, partials};
    dim3 grid;
    if (tile_grid(nx, ny, nz, grid, a.kchunk)) {
        SMG_LAUNCH_G(LaunchEv{}, k_update_p_q_tiled, k_update_p_q_tiled_grp, grid, dim3(kTileThreads), 0, st, a);
        return;
    }
    SMG_LAUNCH_G(LaunchEv{}, k_update_p_q, k_update_p_q_grp, dim3(kRedBlocks), dim3(kRB), 0, st, a);
}

void launch_update_xr(double *x, double *r, const double *p, const double *q, const KScalars *sc, size_t n,
                      double *partials, hipStream_t st)
{
    const UpdXRArgs a{x, r, p, q, sc, static_cast<long long>(n), partials};
    SMG_LAUNCH_G(LaunchEv{}, k_update_xr, k_update_xr_grp, dim3(kRedBlocks), dim3(kRB), 0, st, a);
}

void launch_finalize(int which, int method, int k, const double *partials, KScalars *sc, KScalars *host_copy,
                     hipStream_t st, int nparts)
{
    FinArgs a{};
    a.which = which;
    a.method = method;
    a.k = k;
    a.partials = partials;
    a.sc = sc;
    a.nparts = nparts;
    SMG_LAUNCH_G(LaunchEv{}, k_finalize, k_finalize_grp, dim3(1), dim3(kRB), 0, st, a);
    if (host_copy) (void)hipMemcpyAsync(host_copy, sc, sizeof(KScalars), hipMemcpyDeviceToHost, st);
}

void launch_finalize_batched(int which, int method, const double *partials, KScalars *sc, double rtol, int max_iter,
                             hipStream_t st, int nparts)
{
    FinArgs a{};
    a.which = which;
    a.method = method;
    a.partials = partials;
    a.sc = sc;
    a.nparts = nparts;
    a.batched = 1;
    a.rtol = rtol;
    a.max_iter = max_iter;
    SMG_LAUNCH_G(LaunchEv{}, k_finalize, k_finalize_grp, dim3(1), dim3(kRB), 0, st, a);
}

void launch_copy(const double *src, double *dst, size_t n, hipStream_t st)
{
    const CopyArgs a{src, dst, static_cast<long long>(n)};
    SMG_LAUNCH_G(LaunchEv{}, k_copy, k_copy_grp, dim3(kRedBlocks), dim3(256), 0, st, a);
}

void launch_true_resid(const double *b, const double *x, double *tmp, int nx, int ny, int nz, double cx, double cy,
                       double cz, double *partials, hipStream_t st)
{
    launch_init_resid(b, x, tmp, 0, nx, ny, nz, cx, cy, cz, partials, st);
}

}  // namespace smg
