// Fused 2D/3D V-cycle kernels (gfx950, wave64).
//
// The stage-by-stage schedule of smg_kernels.hip launches four kernels per 2D
// level (F relax, C relax, residual+restriction, prolongation+correction),
// i.e. ~600 mostly tiny launches per 256^3 V-cycle.  These kernels cover the
// same arithmetic with far fewer launches:
//   k2_down   one launch per fine 2D level: for a strip of S coarse lines a
//             workgroup solves the F lines it needs (zero initial guess), then
//             the C lines, keeps both in LDS, writes its own lines of x, and
//             forms the restricted residual of its coarse lines;
//   k2_coarse one workgroup per plane runs the whole remaining 2D sub-cycle on
//             the small levels with every line in LDS;
//   k2_chain  without post-smoothing the upward half of the 2D cycle is a
//             chain of prolongations, x_0 + P(x_1 + P(x_2 + ...)), evaluated
//             per fine point in one pass and added straight into the 3D
//             iterate (the 3D correction step);
//   k2_up     with one post-smoothing step: prolongation, C-line and F-line
//             relaxation of a strip (with a two-line halo) in one launch;
//   k3_chain  the same prolongation chain over the 3D levels.
// Lines are held in registers by one wave (E = ceil(nx/64) points per lane)
// and stored in LDS lane-interleaved (element e of lane l at [e*64 + l]), so
// LDS accesses are conflict-free.
#include "smg_internal.h"

namespace smg {

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

template <typename T, typename A, int E>
__device__ inline void gload(A (&v)[E], const T *row, int nx, int lane)
{
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = lane * E + e;
        v[e] = i < nx ? static_cast<A>(ldv(row + i)) : A(0);
    }
}

template <typename T, typename A, int E>
__device__ inline void gstore(T *row, const A (&v)[E], int nx, int lane)
{
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = lane * E + e;
        if (i < nx) stv(row + i, v[e]);
    }
}

template <typename A, int E>
__device__ inline void sload(A (&v)[E], const A *s, int lane)
{
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = s[e * 64 + lane];
}

template <typename A, int E>
__device__ inline void sstore(A *s, const A (&v)[E], int lane)
{
#pragma unroll
    for (int e = 0; e < E; ++e) s[e * 64 + lane] = v[e];
}

// f -= (a*Tx + b*I) w   (w zero beyond nx)
template <typename A, int E>
__device__ inline void sub_op(A (&f)[E], const A (&w)[E], A a, A b, int lane)
{
    if (a != A(0)) {
        A left = __shfl_up(w[E - 1], 1, 64);
        A right = __shfl_down(w[0], 1, 64);
        if (lane == 0) left = A(0);
        if (lane == 63) right = A(0);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const A wl = e > 0 ? w[e - 1] : left;
            const A wr = e < E - 1 ? w[e + 1] : right;
            f[e] -= a * (A(2) * w[e] - wl - wr) + b * w[e];
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) f[e] -= b * w[e];
    }
}

// Exact solve of one line in place: Thomas recurrences as two lane scans.
template <typename A, int E>
__device__ inline void thomas(A (&f)[E], const Fac<A> *fac, int lane)
{
    const int i0 = lane * E;
    A h[E], pr[E];
    A acc = A(0), prod = A(1);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const Fac<A> fe = fac[i0 + e];
        h[e] = fe.h;
        acc = fe.g * f[e] + fe.h * acc;
        prod *= fe.h;
        f[e] = acc;
        pr[e] = prod;
    }
    A sa = pr[E - 1], sb = f[E - 1];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const A pa = __shfl_up(sa, off, 64);
        const A pb = __shfl_up(sb, off, 64);
        if (lane >= off) {
            sb = sa * pb + sb;
            sa = sa * pa;
        }
    }
    A carry = __shfl_up(sb, 1, 64);
    if (lane == 0) carry = A(0);
#pragma unroll
    for (int e = 0; e < E; ++e) f[e] += pr[e] * carry;
    acc = A(0);
    prod = A(1);
#pragma unroll
    for (int e = E - 1; e >= 0; --e) {
        acc = f[e] + h[e] * acc;
        prod *= h[e];
        f[e] = acc;
        pr[e] = prod;
    }
    sa = pr[0];
    sb = f[0];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const A pa = __shfl_down(sa, off, 64);
        const A pb = __shfl_down(sb, off, 64);
        if (lane + off < 64) {
            sb = sa * pb + sb;
            sa = sa * pa;
        }
    }
    carry = __shfl_down(sb, 1, 64);
    if (lane == 63) carry = A(0);
#pragma unroll
    for (int e = 0; e < E; ++e) f[e] += pr[e] * carry;
}

template <typename A>
__device__ inline const LineCoef<A> *plane_lines(const PlaneCoef<A> *pc, int k, const LineCoef<A> *lc0, int lines_total)
{
    return lc0 + static_cast<size_t>(pc[k].pt) * lines_total;
}

// ---------------------------------------------------------------------------
// k2_down: one pre-smoothing zebra sweep (F then C, zero initial guess) of a
// strip of coarse lines [J0, J0+S), the own lines of x, and the restricted
// residual b_c[J] = 1/2 r_{2J} + r_{2J+1} + 1/2 r_{2J+2}.
// LDS slot s holds fine line j = 2*J0 - 2 + s, s in [0, 2S+5).
// ---------------------------------------------------------------------------
template <typename T, typename A, int E>
__global__ __launch_bounds__(kThreads) void k2_down(Down2Args<T, A> a)
{
    extern __shared__ unsigned char smem_raw[];
    A *xs = reinterpret_cast<A *>(smem_raw);
    const int lane = threadIdx.x & 63, w = wave_id();
    const int nstrip = (a.nyc + a.S - 1) / a.S;
    const int strip = blockIdx.x % nstrip;
    const int p = (blockIdx.x / nstrip) % a.np;
    const int r = blockIdx.x / (nstrip * a.np);
    const int J0 = strip * a.S, J1 = min(J0 + a.S, a.nyc);
    const int ny = a.ny, nx = a.nx, nxp = a.nxp;
    const int base = 2 * J0 - 2;
    const int jlo = max(0, base), jhi = min(ny - 1, 2 * J1 + 2);
    const int k = p * a.kmul + a.koff;
    const LineCoef<A> *lc = plane_lines(a.pc, k, a.lc, a.lines_total);
    const T *bpl = a.b + r * a.brs + p * a.bps;
    T *xpl = a.x + r * a.xrs + p * a.xps;

    // F lines: x_j = L_j^{-1} b_j
    {
        const int f0 = jlo + (jlo & 1);
        const int nf = f0 <= jhi ? (jhi - f0) / 2 + 1 : 0;
        for (int t = w; t < nf; t += kWaves) {
            const int j = f0 + 2 * t;
            A f[E];
            gload<T, A, E>(f, bpl + static_cast<long long>(j) * nx, nx, lane);
            thomas<A, E>(f, a.fac + static_cast<size_t>(lc[j].fac) * nxp, lane);
            sstore<A, E>(xs + (j - base) * nxp, f, lane);
        }
    }
    __syncthreads();
    // C lines: x_j = L_j^{-1} (b_j - V_{j-1} x_{j-1} - V_j x_{j+1})
    {
        const int c0 = jlo | 1;
        const int nc = c0 <= jhi ? (jhi - c0) / 2 + 1 : 0;
        for (int t = w; t < nc; t += kWaves) {
            const int j = c0 + 2 * t;
            A f[E], v[E];
            gload<T, A, E>(f, bpl + static_cast<long long>(j) * nx, nx, lane);
            const LineCoef<A> cm = lc[j - 1];
            sload<A, E>(v, xs + (j - 1 - base) * nxp, lane);
            sub_op<A, E>(f, v, cm.va, cm.vb, lane);
            if (j + 1 < ny) {
                const LineCoef<A> cj = lc[j];
                sload<A, E>(v, xs + (j + 1 - base) * nxp, lane);
                sub_op<A, E>(f, v, cj.va, cj.vb, lane);
            }
            thomas<A, E>(f, a.fac + static_cast<size_t>(lc[j].fac) * nxp, lane);
            sstore<A, E>(xs + (j - base) * nxp, f, lane);
        }
    }
    __syncthreads();
    // own lines of x: [2 J0, 2 J1), plus the last fine line for the last strip
    {
        const int o0 = 2 * J0;
        const int o1 = (J1 == a.nyc) ? ny : 2 * J1;
        for (int j = o0 + w; j < o1; j += kWaves) {
            A v[E];
            sload<A, E>(v, xs + (j - base) * nxp, lane);
            gstore<T, A, E>(xpl + static_cast<long long>(j) * nx, v, nx, lane);
        }
    }
    // restricted residual of the strip's coarse lines
    T *bcpl = a.bc + r * a.crs + p * a.cps;
    for (int J = J0 + w; J < J1; J += kWaves) {
        A acc[E];
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = A(0);
        for (int d = 0; d < 3; ++d) {
            const int j = 2 * J + d;
            if (j >= ny) break;
            A f[E], v[E];
            gload<T, A, E>(f, bpl + static_cast<long long>(j) * nx, nx, lane);
            const LineCoef<A> cj = lc[j];
            sload<A, E>(v, xs + (j - base) * nxp, lane);
            sub_op<A, E>(f, v, cj.la, cj.lb, lane);
            if (j > 0) {
                const LineCoef<A> cm = lc[j - 1];
                sload<A, E>(v, xs + (j - 1 - base) * nxp, lane);
                sub_op<A, E>(f, v, cm.va, cm.vb, lane);
            }
            if (j + 1 < ny) {
                sload<A, E>(v, xs + (j + 1 - base) * nxp, lane);
                sub_op<A, E>(f, v, cj.va, cj.vb, lane);
            }
            const A wgt = d == 1 ? A(1) : A(0.5);
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] += wgt * f[e];
        }
        gstore<T, A, E>(bcpl + static_cast<long long>(J) * nx, acc, nx, lane);
    }
}

// ---------------------------------------------------------------------------
// k2_coarse: the 2D sub-cycle from level l0 down, every line in LDS; one
// workgroup per (plane, rhs).  Generic smoothing counts, F-then-C order.
// ---------------------------------------------------------------------------
template <typename A, int E>
__device__ inline void lds_relax(A *xs, const A *bs, const LineCoef<A> *lc, const Fac<A> *fac, int ny, int nxp,
                                 int colour, bool nbr_zero, int lane, int w)
{
    const int n = colour == 0 ? (ny + 1) / 2 : ny / 2;
    for (int t = w; t < n; t += kWaves) {
        const int j = 2 * t + colour;
        A f[E], v[E];
        sload<A, E>(f, bs + j * nxp, lane);
        if (!nbr_zero) {
            if (j > 0) {
                const LineCoef<A> cm = lc[j - 1];
                sload<A, E>(v, xs + (j - 1) * nxp, lane);
                sub_op<A, E>(f, v, cm.va, cm.vb, lane);
            }
            if (j + 1 < ny) {
                const LineCoef<A> cj = lc[j];
                sload<A, E>(v, xs + (j + 1) * nxp, lane);
                sub_op<A, E>(f, v, cj.va, cj.vb, lane);
            }
        }
        thomas<A, E>(f, fac + static_cast<size_t>(lc[j].fac) * nxp, lane);
        sstore<A, E>(xs + j * nxp, f, lane);
    }
}

template <typename T, typename A, int E>
__global__ __launch_bounds__(kThreads) void k2_coarse(Coarse2Args<T, A> a)
{
    extern __shared__ unsigned char smem_raw[];
    A *sm = reinterpret_cast<A *>(smem_raw);
    const int lane = threadIdx.x & 63, w = wave_id();
    const int p = blockIdx.x % a.np, r = blockIdx.x / a.np;
    const int nx = a.nx, nxp = a.nxp;
    const int k = p * a.kmul + a.koff;
    const LineCoef<A> *lcp = plane_lines(a.pc, k, a.lc, a.lines_total);
    // LDS: x and b of every level l0..L-1, line offsets lo[l]
    int lo[16];
    int off = 0;
    for (int l = a.l0; l < a.nlev; ++l) {
        lo[l] = off;
        off += a.ny2[l];
    }
    A *xs = sm, *bs = sm + static_cast<size_t>(off) * nxp;
    // right-hand side of level l0
    {
        const T *bpl = a.b + r * a.brs + p * a.bps;
        for (int j = w; j < a.ny2[a.l0]; j += kWaves) {
            A v[E];
            gload<T, A, E>(v, bpl + static_cast<long long>(j) * nx, nx, lane);
            sstore<A, E>(bs + (lo[a.l0] + j) * nxp, v, lane);
        }
    }
    __syncthreads();
    // downward half
    for (int l = a.l0; l < a.nlev - 1; ++l) {
        const int ny = a.ny2[l], nyc = a.ny2[l + 1];
        const LineCoef<A> *lc = lcp + a.lev_off[l];
        A *x = xs + lo[l] * nxp, *b = bs + lo[l] * nxp, *bc = bs + lo[l + 1] * nxp;
        for (int s = 0; s < a.ipre; ++s) {
            lds_relax<A, E>(x, b, lc, a.fac, ny, nxp, 0, s == 0, lane, w);
            __syncthreads();
            lds_relax<A, E>(x, b, lc, a.fac, ny, nxp, 1, false, lane, w);
            __syncthreads();
        }
        if (a.ipre == 0) {
            for (int j = w; j < ny; j += kWaves)
#pragma unroll
                for (int e = 0; e < E; ++e) x[j * nxp + e * 64 + lane] = A(0);
            __syncthreads();
        }
        for (int J = w; J < nyc; J += kWaves) {
            A acc[E];
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] = A(0);
            for (int d = 0; d < 3; ++d) {
                const int j = 2 * J + d;
                if (j >= ny) break;
                A f[E], v[E];
                sload<A, E>(f, b + j * nxp, lane);
                const LineCoef<A> cj = lc[j];
                sload<A, E>(v, x + j * nxp, lane);
                sub_op<A, E>(f, v, cj.la, cj.lb, lane);
                if (j > 0) {
                    const LineCoef<A> cm = lc[j - 1];
                    sload<A, E>(v, x + (j - 1) * nxp, lane);
                    sub_op<A, E>(f, v, cm.va, cm.vb, lane);
                }
                if (j + 1 < ny) {
                    sload<A, E>(v, x + (j + 1) * nxp, lane);
                    sub_op<A, E>(f, v, cj.va, cj.vb, lane);
                }
                const A wgt = d == 1 ? A(1) : A(0.5);
#pragma unroll
                for (int e = 0; e < E; ++e) acc[e] += wgt * f[e];
            }
            sstore<A, E>(bc + J * nxp, acc, lane);
        }
        __syncthreads();
    }
    // coarsest level: one exact line solve
    {
        const int l = a.nlev - 1;
        if (w == 0) {
            A f[E];
            sload<A, E>(f, bs + lo[l] * nxp, lane);
            thomas<A, E>(f, a.fac + static_cast<size_t>((lcp + a.lev_off[l])[0].fac) * nxp, lane);
            sstore<A, E>(xs + lo[l] * nxp, f, lane);
        }
        __syncthreads();
    }
    // upward half
    for (int l = a.nlev - 2; l >= a.l0; --l) {
        const int ny = a.ny2[l], nyc = a.ny2[l + 1];
        const LineCoef<A> *lc = lcp + a.lev_off[l];
        A *x = xs + lo[l] * nxp, *b = bs + lo[l] * nxp;
        const A *xc = xs + lo[l + 1] * nxp;
        for (int j = w; j < ny; j += kWaves) {
            A v[E], c[E];
            sload<A, E>(v, x + j * nxp, lane);
            if (j & 1) {
                sload<A, E>(c, xc + (j >> 1) * nxp, lane);
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] += c[e];
            } else {
                const int J = j >> 1;
                if (J - 1 >= 0) {
                    sload<A, E>(c, xc + (J - 1) * nxp, lane);
#pragma unroll
                    for (int e = 0; e < E; ++e) v[e] += A(0.5) * c[e];
                }
                if (J < nyc) {
                    sload<A, E>(c, xc + J * nxp, lane);
#pragma unroll
                    for (int e = 0; e < E; ++e) v[e] += A(0.5) * c[e];
                }
            }
            sstore<A, E>(x + j * nxp, v, lane);
        }
        __syncthreads();
        for (int s = 0; s < a.ipost; ++s) {
            lds_relax<A, E>(x, b, lc, a.fac, ny, nxp, 1, false, lane, w);
            __syncthreads();
            lds_relax<A, E>(x, b, lc, a.fac, ny, nxp, 0, false, lane, w);
            __syncthreads();
        }
    }
    // result of level l0
    {
        T *opl = a.out + r * a.ors + p * a.ops;
        for (int j = w; j < a.ny2[a.l0]; j += kWaves) {
            A v[E];
            sload<A, E>(v, xs + (lo[a.l0] + j) * nxp, lane);
            T *row = opl + static_cast<long long>(j) * nx;
            if (a.accumulate) {
                A o[E];
                gload<T, A, E>(o, row, nx, lane);
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] += o[e];
            }
            gstore<T, A, E>(row, v, nx, lane);
        }
    }
}

// ---------------------------------------------------------------------------
// k2_chain: y = x_0 + P_0(x_1 + P_1(... + P x_lc)) per fine point, then
// out = y or out += y.  Coarse levels 1..lc are packed; x_lc is complete.
// ---------------------------------------------------------------------------
template <typename T, typename A>
__global__ __launch_bounds__(256) void k2_chain(Chain2Args<T, A> a)
{
    const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const long long total = static_cast<long long>(a.nx) * a.ny2[0] * a.np * a.nrhs;
    if (idx >= total) return;
    const int i = static_cast<int>(idx % a.nx);
    long long t = idx / a.nx;
    const int j = static_cast<int>(t % a.ny2[0]);
    t /= a.ny2[0];
    const int p = static_cast<int>(t % a.np);
    const int r = static_cast<int>(t / a.np);
    // index windows [lo_l, lo_l + 2] of the lines each level contributes
    int lo[16], hi[16];
    lo[0] = hi[0] = j;
    for (int l = 0; l < a.lc; ++l) {
        lo[l + 1] = max(0, (lo[l] - 1) >> 1);
        hi[l + 1] = min(a.ny2[l + 1] - 1, hi[l] >> 1);
    }
    A v[3];
    {
        const int l = a.lc;
        const T *xl = a.xc[l] + r * a.crs[l] + p * a.cps[l];
        for (int q = 0; q < 3; ++q) {
            const int jj = lo[l] + q;
            v[q] = jj <= hi[l] ? static_cast<A>(ldv(xl + static_cast<long long>(jj) * a.nx + i)) : A(0);
        }
    }
    for (int l = a.lc - 1; l >= 0; --l) {
        const T *xl = l == 0 ? a.x0 + r * a.x0rs + p * a.x0ps : a.xc[l] + r * a.crs[l] + p * a.cps[l];
        const int nyc = a.ny2[l + 1];
        A nv[3];
        for (int q = 0; q < 3; ++q) {
            const int jj = lo[l] + q;
            if (jj > hi[l]) {
                nv[q] = A(0);
                continue;
            }
            A s = ldv(xl + static_cast<long long>(jj) * a.nx + i);
            if (jj & 1) {
                s += v[((jj - 1) >> 1) - lo[l + 1]];
            } else {
                const int J = jj >> 1;
                if (J - 1 >= 0) s += A(0.5) * v[J - 1 - lo[l + 1]];
                if (J < nyc) s += A(0.5) * v[J - lo[l + 1]];
            }
            nv[q] = s;
        }
        v[0] = nv[0];
        v[1] = nv[1];
        v[2] = nv[2];
    }
    T *o = a.out + r * a.ors + p * a.ops + static_cast<long long>(j) * a.nx + i;
    stv(o, a.accumulate ? static_cast<A>(ldv(o)) + v[0] : v[0]);
}

// ---------------------------------------------------------------------------
// k2_up: prolongation and one post-smoothing sweep (C then F) of a strip of
// fine lines [j0, j0 + 2S).  LDS slot s holds fine line j0 - 2 + s.
// x_pre: this level after pre-smoothing; xc: the coarser level's result;
// out: this level's result (a different buffer), assigned or accumulated.
// ---------------------------------------------------------------------------
template <typename T, typename A, int E>
__global__ __launch_bounds__(kThreads) void k2_up(Up2Args<T, A> a)
{
    extern __shared__ unsigned char smem_raw[];
    A *xs = reinterpret_cast<A *>(smem_raw);
    const int lane = threadIdx.x & 63, w = wave_id();
    const int ny = a.ny, nyc = a.nyc, nx = a.nx, nxp = a.nxp;
    const int nstrip = (ny + 2 * a.S - 1) / (2 * a.S);
    const int strip = blockIdx.x % nstrip;
    const int p = (blockIdx.x / nstrip) % a.np;
    const int r = blockIdx.x / (nstrip * a.np);
    const int j0 = strip * 2 * a.S, j1 = min(j0 + 2 * a.S, ny);
    const int base = j0 - 2;
    const int jlo = max(0, j0 - 2), jhi = min(ny - 1, j1 + 1);
    const int k = p * a.kmul + a.koff;
    const LineCoef<A> *lc = plane_lines(a.pc, k, a.lc, a.lines_total);
    const T *xp = a.xpre + r * a.xrs + p * a.xps;
    const T *cp = a.xc + r * a.crs + p * a.cps;
    const T *bp = a.b + r * a.brs + p * a.bps;
    // prolongation + correction on [jlo, jhi]
    for (int j = jlo + w; j <= jhi; j += kWaves) {
        A v[E], c[E];
        gload<T, A, E>(v, xp + static_cast<long long>(j) * nx, nx, lane);
        if (j & 1) {
            gload<T, A, E>(c, cp + static_cast<long long>(j >> 1) * nx, nx, lane);
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] += c[e];
        } else {
            const int J = j >> 1;
            if (J - 1 >= 0) {
                gload<T, A, E>(c, cp + static_cast<long long>(J - 1) * nx, nx, lane);
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] += A(0.5) * c[e];
            }
            if (J < nyc) {
                gload<T, A, E>(c, cp + static_cast<long long>(J) * nx, nx, lane);
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] += A(0.5) * c[e];
            }
        }
        sstore<A, E>(xs + (j - base) * nxp, v, lane);
    }
    __syncthreads();
    // C lines in [j0 - 1, j1] , then F lines in [j0, j1)
    for (int colour = 1; colour >= 0; --colour) {
        const int lo = colour == 1 ? max(1, (j0 - 1) | 1) : j0 + (j0 & 1);
        const int hi = colour == 1 ? min(ny - 1, j1) : j1 - 1;
        const int n = lo <= hi ? (hi - lo) / 2 + 1 : 0;
        for (int t = w; t < n; t += kWaves) {
            const int j = lo + 2 * t;
            A f[E], v[E];
            gload<T, A, E>(f, bp + static_cast<long long>(j) * nx, nx, lane);
            if (j > 0) {
                const LineCoef<A> cm = lc[j - 1];
                sload<A, E>(v, xs + (j - 1 - base) * nxp, lane);
                sub_op<A, E>(f, v, cm.va, cm.vb, lane);
            }
            if (j + 1 < ny) {
                const LineCoef<A> cj = lc[j];
                sload<A, E>(v, xs + (j + 1 - base) * nxp, lane);
                sub_op<A, E>(f, v, cj.va, cj.vb, lane);
            }
            thomas<A, E>(f, a.fac + static_cast<size_t>(lc[j].fac) * nxp, lane);
            sstore<A, E>(xs + (j - base) * nxp, f, lane);
        }
        __syncthreads();
    }
    // own lines out
    T *op = a.out + r * a.ors + p * a.ops;
    for (int j = j0 + w; j < j1; j += kWaves) {
        A v[E];
        sload<A, E>(v, xs + (j - base) * nxp, lane);
        T *row = op + static_cast<long long>(j) * nx;
        if (a.accumulate) {
            A o[E];
            gload<T, A, E>(o, row, nx, lane);
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] += o[e];
        }
        gstore<T, A, E>(row, v, nx, lane);
    }
}

// ---------------------------------------------------------------------------
// k3_chain: s = x_0 + P(x_1 + P(... + P x_L)) over the 3D levels, in place on
// level 0 (each point reads its own x_0 value and writes it back).
// ---------------------------------------------------------------------------
template <typename T, typename A>
__global__ __launch_bounds__(256) void k3_chain(Chain3Args<T, A> a)
{
    const long long pl = static_cast<long long>(a.nx) * a.ny;
    const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= pl) return;
    const int k = blockIdx.y, r = blockIdx.z;
    int lo[24], hi[24];
    lo[0] = hi[0] = k;
    for (int l = 0; l < a.L; ++l) {
        lo[l + 1] = max(0, (lo[l] - 1) >> 1);
        hi[l + 1] = min(a.nz[l + 1] - 1, hi[l] >> 1);
    }
    A v[3];
    {
        const int l = a.L;
        const T *xl = a.x[l] + r * a.rs[l];
        for (int q = 0; q < 3; ++q) {
            const int kk = lo[l] + q;
            v[q] = kk <= hi[l] ? static_cast<A>(ldv(xl + kk * pl + c)) : A(0);
        }
    }
    for (int l = a.L - 1; l >= 0; --l) {
        const T *xl = a.x[l] + r * a.rs[l];
        const int nzc = a.nz[l + 1];
        A nv[3];
        for (int q = 0; q < 3; ++q) {
            const int kk = lo[l] + q;
            if (kk > hi[l]) {
                nv[q] = A(0);
                continue;
            }
            A s = ldv(xl + kk * pl + c);
            if (kk & 1) {
                s += v[((kk - 1) >> 1) - lo[l + 1]];
            } else {
                const int K = kk >> 1;
                if (K - 1 >= 0) s += A(0.5) * v[K - 1 - lo[l + 1]];
                if (K < nzc) s += A(0.5) * v[K - lo[l + 1]];
            }
            nv[q] = s;
        }
        v[0] = nv[0];
        v[1] = nv[1];
        v[2] = nv[2];
    }
    T *o = a.x[0] + r * a.rs[0] + k * pl + c;
    stv(o, v[0]);
}

inline unsigned nb(long long n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

}  // namespace

#define SMG_E_SWITCH(E, CALL)                 \
    switch (E) {                              \
    case 1: { constexpr int EE = 1; CALL; } break; \
    case 2: { constexpr int EE = 2; CALL; } break; \
    case 3: { constexpr int EE = 3; CALL; } break; \
    case 4: { constexpr int EE = 4; CALL; } break; \
    case 5: { constexpr int EE = 5; CALL; } break; \
    case 6: { constexpr int EE = 6; CALL; } break; \
    case 7: { constexpr int EE = 7; CALL; } break; \
    case 8: { constexpr int EE = 8; CALL; } break; \
    default: break;                           \
    }

template <typename T, typename A>
void launch_down2(const Down2Args<T, A> &a, hipStream_t st, const LaunchEv &ev)
{
    const int nstrip = (a.nyc + a.S - 1) / a.S;
    const long long nblk = static_cast<long long>(nstrip) * a.np * a.nrhs;
    if (nblk == 0) return;
    const size_t lds = static_cast<size_t>(2 * a.S + 5) * a.nxp * sizeof(A);
    SMG_E_SWITCH(a.nxp / 64, SMG_LAUNCH(ev, (k2_down<T, A, EE>), dim3(static_cast<unsigned>(nblk)),
                                                dim3(kThreads), lds, st, a));
}

template <typename T, typename A>
void launch_coarse2(const Coarse2Args<T, A> &a, size_t lds_bytes, hipStream_t st, const LaunchEv &ev)
{
    const long long nblk = static_cast<long long>(a.np) * a.nrhs;
    if (nblk == 0) return;
    SMG_E_SWITCH(a.nxp / 64, SMG_LAUNCH(ev, (k2_coarse<T, A, EE>), dim3(static_cast<unsigned>(nblk)),
                                                dim3(kThreads), lds_bytes, st, a));
}

template <typename T, typename A>
void launch_chain2(const Chain2Args<T, A> &a, hipStream_t st, const LaunchEv &ev)
{
    const long long n = static_cast<long long>(a.nx) * a.ny2[0] * a.np * a.nrhs;
    if (n == 0) return;
    SMG_LAUNCH(ev, (k2_chain<T, A>), dim3(nb(n, 256)), dim3(256), 0, st, a);
}

template <typename T, typename A>
void launch_up2(const Up2Args<T, A> &a, hipStream_t st, const LaunchEv &ev)
{
    const int nstrip = (a.ny + 2 * a.S - 1) / (2 * a.S);
    const long long nblk = static_cast<long long>(nstrip) * a.np * a.nrhs;
    if (nblk == 0) return;
    const size_t lds = static_cast<size_t>(2 * a.S + 4) * a.nxp * sizeof(A);
    SMG_E_SWITCH(a.nxp / 64, SMG_LAUNCH(ev, (k2_up<T, A, EE>), dim3(static_cast<unsigned>(nblk)),
                                                dim3(kThreads), lds, st, a));
}

template <typename T, typename A>
void launch_chain3(const Chain3Args<T, A> &a, int nrhs, hipStream_t st, const LaunchEv &ev)
{
    const dim3 grid(nb(static_cast<long long>(a.nx) * a.ny, 256), a.nz[0], nrhs);
    SMG_LAUNCH(ev, (k3_chain<T, A>), grid, dim3(256), 0, st, a);
}

#define SMG_FUSED_INSTANTIATE(T, A)                                                          \
    template void launch_down2<T, A>(const Down2Args<T, A> &, hipStream_t, const LaunchEv &);             \
    template void launch_coarse2<T, A>(const Coarse2Args<T, A> &, size_t, hipStream_t, const LaunchEv &); \
    template void launch_chain2<T, A>(const Chain2Args<T, A> &, hipStream_t, const LaunchEv &);           \
    template void launch_up2<T, A>(const Up2Args<T, A> &, hipStream_t, const LaunchEv &);                 \
    template void launch_chain3<T, A>(const Chain3Args<T, A> &, int, hipStream_t, const LaunchEv &);

SMG_FUSED_INSTANTIATE(double, double)
SMG_FUSED_INSTANTIATE(float, float)
SMG_FUSED_INSTANTIATE(bf16, float)

}  // namespace smg
