// SMG V-cycle kernels for gfx950 (wave64).
//
// Stages of one V-cycle (Section 3 reading: z-semicoarsening, zebra plane
// relaxation whose plane solves are 2D y-semicoarsening cycles with zebra
// x-line relaxation and exact line solves):
//   k_line_relax  - exact solves of a batch of x-lines (one wave per line),
//                   right-hand side b_j - V_{j-1} x_{j-1} - V_j x_{j+1};
//   k_restrict2   - 2D residual + restriction P_y^T (fused);
//   k_prolong2    - 2D prolongation P_y + correction;
//   k_resid3v     - 3D residual of the planes of one colour (15-point),
//                   V consecutive points of a row per thread;
//   k_correct3    - x_k += y_k for the planes of one colour;
//   k_restrict3   - 3D residual + restriction P_z^T (fused; k_restrict3_march
//                   marches z with V points of a row per thread);
//   k_prolong3    - 3D prolongation P_z + correction.
// Every kernel is batched over planes and right-hand sides and is bound by
// HBM bandwidth; the line solve needs no LDS: a line of nx <= 512 points
// lives in the registers of one wave (E = ceil(nx/64) points per lane) and
// the two first-order recurrences of the Thomas algorithm are evaluated as
// affine-map scans across the 64 lanes.
#include "group.h"
#include "smg_internal.h"

namespace smg {

namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kBlock = 64 * kWavesPerBlock;

__device__ inline int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// f -= (va*Tx + vb*I) w for the E points of this lane of one line.
template <typename T, typename A, int E>
__device__ inline void sub_coupling(A (&f)[E], const T *row, int i0, int nx, A va, A vb, int lane)
{
    A w[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = i0 + e;
        w[e] = i < nx ? static_cast<A>(ldv(row + i)) : A(0);
    }
    if (va != A(0)) {
        A left = __shfl_up(w[E - 1], 1, 64);
        A right = __shfl_down(w[0], 1, 64);
        if (lane == 0) left = A(0);
        if (lane == 63) right = A(0);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const A wl = e > 0 ? w[e - 1] : left;
            const A wr = e < E - 1 ? w[e + 1] : right;
            f[e] -= va * (A(2) * w[e] - wl - wr) + vb * w[e];
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) f[e] -= vb * w[e];
    }
}

template <typename T, typename A, int E>
__global__ __launch_bounds__(kBlock) void k_line_relax(LineRelaxArgs<T, A> a)
{
    const int lane = threadIdx.x & 63;
    const long long wave = static_cast<long long>(blockIdx.x) * kWavesPerBlock + wave_uniform(threadIdx.x >> 6);
    const long long total = static_cast<long long>(a.nq) * a.np * a.nrhs;
    if (wave >= total) return;   // whole waves only: no barrier below
    const int q = static_cast<int>(wave % a.nq);
    const long long t = wave / a.nq;
    const int p = static_cast<int>(t % a.np);
    const int r = static_cast<int>(t / a.np);
    const int j = a.ny == 1 ? 0 : 2 * q + a.colour;
    const int k = p * a.kmul + a.koff;
    const LineCoef<A> *lc = a.lc + static_cast<size_t>(a.pc[k].pt) * a.lines_total;
    const LineCoef<A> cj = lc[j];
    const Fac<A> *fac = a.fac + static_cast<size_t>(cj.fac) * a.nxp;

    const int nx = a.nx;
    const int i0 = lane * E;
    const T *brow = a.b + r * a.brs + p * a.bps + static_cast<long long>(j) * nx;
    T *xpl = a.x + r * a.xrs + p * a.xps;

    A f[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = i0 + e;
        f[e] = i < nx ? static_cast<A>(ldv(brow + i)) : A(0);
    }
    if (!a.nbr_zero) {
        if (j > 0) {
            const LineCoef<A> cm = lc[j - 1];
            sub_coupling<T, A, E>(f, xpl + static_cast<long long>(j - 1) * nx, i0, nx, cm.va, cm.vb, lane);
        }
        if (j < a.ny - 1)
            sub_coupling<T, A, E>(f, xpl + static_cast<long long>(j + 1) * nx, i0, nx, cj.va, cj.vb, lane);
    }

    // Forward recurrence y_i = g_i f_i + h_i y_{i-1}: lane-local pass with a
    // zero carry, then an inclusive scan of the lanes' affine maps.
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

    // Backward recurrence u_i = y_i + h_i u_{i+1}, scanned from the top lane.
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
    T *xrow = xpl + static_cast<long long>(j) * nx;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = i0 + e;
        if (i < nx) stv(xrow + i, f[e] + pr[e] * carry);
    }
}

// (la*Tx + lb*I) applied to row at point i
template <typename T, typename A>
__device__ inline A line_op(A la, A lb, const T *row, int i, int nx)
{
    const A v = ldv(row + i);
    if (la == A(0)) return lb * v;
    const A vl = i > 0 ? static_cast<A>(ldv(row + i - 1)) : A(0);
    const A vr = i < nx - 1 ? static_cast<A>(ldv(row + i + 1)) : A(0);
    return la * (A(2) * v - vl - vr) + lb * v;
}

template <typename T, typename A>
__device__ inline A resid2(const Restrict2Args<T, A> &a, const LineCoef<A> *lc, const T *xpl, const T *bpl, int j,
                           int i)
{
    const int nx = a.nx;
    A v = ldv(bpl + static_cast<long long>(j) * nx + i);
    if (a.x_zero) return v;
    const LineCoef<A> cj = lc[j];
    v -= line_op<T, A>(cj.la, cj.lb, xpl + static_cast<long long>(j) * nx, i, nx);
    if (j > 0) {
        const LineCoef<A> cm = lc[j - 1];
        v -= line_op<T, A>(cm.va, cm.vb, xpl + static_cast<long long>(j - 1) * nx, i, nx);
    }
    if (j < a.ny - 1) v -= line_op<T, A>(cj.va, cj.vb, xpl + static_cast<long long>(j + 1) * nx, i, nx);
    return v;
}

template <typename T, typename A>
__global__ __launch_bounds__(256) void k_restrict2(Restrict2Args<T, A> a)
{
    const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const long long total = static_cast<long long>(a.nx) * a.nyc * a.np * a.nrhs;
    if (idx >= total) return;
    const int i = static_cast<int>(idx % a.nx);
    long long t = idx / a.nx;
    const int J = static_cast<int>(t % a.nyc);
    t /= a.nyc;
    const int p = static_cast<int>(t % a.np);
    const int r = static_cast<int>(t / a.np);
    const int k = p * a.kmul + a.koff;
    const LineCoef<A> *lc = a.lc + static_cast<size_t>(a.pc[k].pt) * a.lines_total;
    const T *xpl = a.x + r * a.xrs + p * a.xps;
    const T *bpl = a.b + r * a.brs + p * a.bps;
    A v = A(0.5) * resid2(a, lc, xpl, bpl, 2 * J, i) + resid2(a, lc, xpl, bpl, 2 * J + 1, i);
    if (2 * J + 2 < a.ny) v += A(0.5) * resid2(a, lc, xpl, bpl, 2 * J + 2, i);
    stv(a.bc + r * a.crs + p * a.cps + static_cast<long long>(J) * a.nx + i, v);
}

template <typename T, typename A>
__global__ __launch_bounds__(256) void k_prolong2(Prolong2Args<T, A> a)
{
    const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const long long total = static_cast<long long>(a.nx) * a.ny * a.np * a.nrhs;
    if (idx >= total) return;
    const int i = static_cast<int>(idx % a.nx);
    long long t = idx / a.nx;
    const int j = static_cast<int>(t % a.ny);
    t /= a.ny;
    const int p = static_cast<int>(t % a.np);
    const int r = static_cast<int>(t / a.np);
    const T *cpl = a.xc + r * a.crs + p * a.cps;
    A v;
    if (j & 1) {
        v = ldv(cpl + static_cast<long long>(j >> 1) * a.nx + i);
    } else {
        const int J = j >> 1;
        v = A(0);
        if (J - 1 >= 0) v += A(0.5) * static_cast<A>(ldv(cpl + static_cast<long long>(J - 1) * a.nx + i));
        if (J < a.nyc) v += A(0.5) * static_cast<A>(ldv(cpl + static_cast<long long>(J) * a.nx + i));
    }
    T *xp = a.x + r * a.xrs + p * a.xps + static_cast<long long>(j) * a.nx + i;
    stv(xp, a.x_zero ? v : static_cast<A>(ldv(xp)) + v);
}

// (ma*T2 + mb*I) applied to plane pl at (i, j)
template <typename T, typename A>
__device__ inline A plane_op(A ma, A mb, A cx, A cy, const T *pl, int i, int j, int nx, int ny)
{
    const long long c = static_cast<long long>(j) * nx + i;
    const A v = ldv(pl + c);
    if (ma == A(0)) return mb * v;
    const A xl = i > 0 ? static_cast<A>(ldv(pl + c - 1)) : A(0);
    const A xr = i < nx - 1 ? static_cast<A>(ldv(pl + c + 1)) : A(0);
    const A yl = j > 0 ? static_cast<A>(ldv(pl + c - nx)) : A(0);
    const A yr = j < ny - 1 ? static_cast<A>(ldv(pl + c + nx)) : A(0);
    return ma * (cx * (A(2) * v - xl - xr) + cy * (A(2) * v - yl - yr)) + mb * v;
}

// b_k - (A_l x)_k at point (i, j) of plane k
template <typename T, typename A>
__device__ inline A resid3_point(const T *x, const T *b, const PlaneCoef<A> *pc, A cx, A cy, int nx, int ny,
                                 int nz, int k, int i, int j, bool self_zero, bool x_zero = false)
{
    const long long pl = static_cast<long long>(nx) * ny;
    A v = ldv(b + k * pl + static_cast<long long>(j) * nx + i);
    if (x_zero) return v;
    const PlaneCoef<A> ck = pc[k];
    if (!self_zero) v -= plane_op<T, A>(ck.ca, ck.cb, cx, cy, x + k * pl, i, j, nx, ny);
    if (k > 0) {
        const PlaneCoef<A> cm = pc[k - 1];
        v -= plane_op<T, A>(cm.ua, cm.ub, cx, cy, x + (k - 1) * pl, i, j, nx, ny);
    }
    if (k < nz - 1) v -= plane_op<T, A>(ck.ua, ck.ub, cx, cy, x + (k + 1) * pl, i, j, nx, ny);
    return v;
}

// The colour residual r_k = b_k - (A_l x)_k on the planes of one colour, with
// V consecutive points of a row per thread (the launcher takes V > 1 when nx
// and every plane and right-hand-side offset are multiples of V, else V = 1):
// the row is read as V-wide accesses and the x-neighbours inside it are
// taken from the registers; the arithmetic per point does not depend on V.
template <typename T, typename A, int V>
__device__ inline void plane_op_v(A (&o)[V], A ma, A mb, A cx, A cy, const T *pl, int i, int j, int nx, int ny)
{
    const long long c = static_cast<long long>(j) * nx + i;
    A v[V];
    vld<T, A, V>(v, pl + c, V);
    if (ma == A(0)) {
#pragma unroll
        for (int e = 0; e < V; ++e) o[e] = mb * v[e];
        return;
    }
    A yl[V], yr[V];
    vld<T, A, V>(yl, pl + c - nx, j > 0 ? V : 0);
    vld<T, A, V>(yr, pl + c + nx, j < ny - 1 ? V : 0);
    const A xl0 = i > 0 ? static_cast<A>(ldv(pl + c - 1)) : A(0);
    const A xrv = i + V < nx ? static_cast<A>(ldv(pl + c + V)) : A(0);
#pragma unroll
    for (int e = 0; e < V; ++e) {
        const A xl = e > 0 ? v[e - 1] : xl0;
        const A xr = e < V - 1 ? v[e + 1] : xrv;
        const A dx = A(2) * v[e] - xl - xr, dy = A(2) * v[e] - yl[e] - yr[e];
        o[e] = fmadd(ma, fmadd(cx, dx, cy * dy), mb * v[e]);
    }
}

template <typename T, typename A, int V>
__device__ __forceinline__ void k_resid3v_body(const Resid3Args<T, A> &a, const Blk &blk)
{
    const long long c = (static_cast<long long>(blk.x) * blockDim.x + threadIdx.x) * V;
    const long long pl = static_cast<long long>(a.nx) * a.ny;
    if (c >= pl) return;
    const int i = static_cast<int>(c % a.nx), j = static_cast<int>(c / a.nx);
    const int p = blk.y, r = blk.z;
    const int k = p * a.kmul + a.koff;
    const T *x = a.x + r * a.xrs;
    A v[V], o[V];
    vld<T, A, V>(v, a.b + r * a.brs + k * pl + c, V);
    const PlaneCoef<A> ck = a.pc[k];
    if (!a.self_zero) {
        plane_op_v<T, A, V>(o, ck.ca, ck.cb, a.cx, a.cy, x + k * pl, i, j, a.nx, a.ny);
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] -= o[e];
    }
    if (k > 0) {
        const PlaneCoef<A> cm = a.pc[k - 1];
        plane_op_v<T, A, V>(o, cm.ua, cm.ub, a.cx, a.cy, x + (k - 1) * pl, i, j, a.nx, a.ny);
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] -= o[e];
    }
    if (k < a.nz - 1) {
        plane_op_v<T, A, V>(o, ck.ua, ck.ub, a.cx, a.cy, x + (k + 1) * pl, i, j, a.nx, a.ny);
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] -= o[e];
    }
    vst<T, A, V>(a.r + r * a.rrs + p * a.rps + c, v, V);
}

template <typename T, typename A, int V>
__global__ __launch_bounds__(256) void k_resid3v(Resid3Args<T, A> a)
{
    k_resid3v_body<T, A, V>(a, SMG_BLK_XCD);
}

template <typename T, typename A, int V>
__global__ __launch_bounds__(256) void k_resid3v_grp(const GroupEntry *tab, int n)
{
    const Resid3Args<T, A> *a;
    Blk blk;
    if (!group_entry(tab, n, a, blk)) return;
    k_resid3v_body<T, A, V>(*a, blk);
}

template <typename T, typename A>
__global__ __launch_bounds__(256) void k_correct3(Correct3Args<T, A> a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const long long pl = static_cast<long long>(a.nx) * a.ny;
    if (c >= pl) return;
    const int p = blockIdx.y, r = blockIdx.z;
    const int k = p * a.kmul + a.koff;
    T *xp = a.x + r * a.xrs + k * pl + c;
    stv(xp, static_cast<A>(ldv(xp)) + static_cast<A>(ldv(a.y + r * a.yrs + p * a.yps + c)));
}

template <typename T, typename A>
__device__ __forceinline__ void k_restrict3_body(const Restrict3Args<T, A> &a, const Blk &blk)
{
    const int c = blk.x * blockDim.x + threadIdx.x;
    if (c >= a.nx * a.ny) return;
    const int i = c % a.nx, j = c / a.nx;
    const int K = blk.y, r = blk.z;
    const T *x = a.x + r * a.xrs;
    const T *b = a.b + r * a.brs;
    const bool xz = a.x_zero != 0;
    A v = A(0.5) * resid3_point<T, A>(x, b, a.pc, a.cx, a.cy, a.nx, a.ny, a.nz, 2 * K, i, j, false, xz)
          + resid3_point<T, A>(x, b, a.pc, a.cx, a.cy, a.nx, a.ny, a.nz, 2 * K + 1, i, j, false, xz);
    if (2 * K + 2 < a.nz)
        v += A(0.5) * resid3_point<T, A>(x, b, a.pc, a.cx, a.cy, a.nx, a.ny, a.nz, 2 * K + 2, i, j, false, xz);
    const long long pl = static_cast<long long>(a.nx) * a.ny;
    stv(a.bc + r * a.crs + K * pl + c, v);
}

template <typename T, typename A>
__global__ __launch_bounds__(256) void k_restrict3(Restrict3Args<T, A> a)
{
    k_restrict3_body<T, A>(a, SMG_BLK_XCD);
}

template <typename T, typename A>
__global__ __launch_bounds__(256) void k_restrict3_grp(const GroupEntry *tab, int n)
{
    const Restrict3Args<T, A> *a;
    Blk blk;
    if (!group_entry(tab, n, a, blk)) return;
    k_restrict3_body<T, A>(*a, blk);
}

template <typename T, typename A>
__global__ __launch_bounds__(256) void k_prolong3(Prolong3Args<T, A> a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const long long pl = static_cast<long long>(a.nx) * a.ny;
    if (c >= pl) return;
    const int k = blockIdx.y, r = blockIdx.z;
    const T *xc = a.xc + r * a.crs;
    A v;
    if (k & 1) {
        v = ldv(xc + (k >> 1) * pl + c);
    } else {
        const int K = k >> 1;
        v = A(0);
        if (K - 1 >= 0) v += A(0.5) * static_cast<A>(ldv(xc + (K - 1) * pl + c));
        if (K < a.nzc) v += A(0.5) * static_cast<A>(ldv(xc + K * pl + c));
    }
    T *xp = a.x + r * a.xrs + k * pl + c;
    stv(xp, a.x_zero ? v : static_cast<A>(ldv(xp)) + v);
}

// Thomas factors of (la*Tx + lb*I): pivots m_0 = 2la+lb, m_i = m_0 - off*(off/m_{i-1})
// with off = -la; g_i = 1/m_i, h_i = -off/m_i.  Computed in FP64.
template <typename A>
__global__ void k_thomas_tables(const LineCoef<double> *ab, int nfac, int nx, int nxp, Fac<A> *out)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nfac) return;
    const double la = ab[f].la, lb = ab[f].lb;
    const double diag = 2.0 * la + lb, off = -la;
    double m = diag;
    Fac<A> *o = out + static_cast<size_t>(f) * nxp;
    for (int i = 0; i < nxp; ++i) {
        if (i >= nx) {
            o[i].g = A(0);
            o[i].h = A(0);
            continue;
        }
        if (i > 0) m = diag - off * (off / m);
        o[i].g = static_cast<A>(1.0 / m);
        o[i].h = static_cast<A>(-off / m);
    }
}

template <typename T>
__global__ void k_convert_in(const double *src, long long lds, T *dst, long long ldd, size_t n)
{
    const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = blockIdx.y;
    stv(dst + r * ldd + i, static_cast<typename Arith<T>::type>(src[r * lds + i]));
}

template <typename T>
__global__ void k_convert_out(const T *src, long long lds, double *dst, long long ldd, size_t n)
{
    const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = blockIdx.y;
    dst[r * ldd + i] = static_cast<double>(ldv(src + r * lds + i));
}

// Residual + restriction marching in z.  A block owns a 64 x 4 (i, j) tile and
// a run of coarse planes [K0, K1).  Every fine x plane is staged once in an
// LDS tile with a one-point halo, its in-plane product T2 x is formed once,
// and a window of three planes (x and T2 x) in registers feeds the 15-point
// residuals r_k = b_k - C_k x_k - U_{k-1} x_{k-1} - U_k x_{k+1}, which are
// combined into b_c[K] = 1/2 r_{2K} + r_{2K+1} + 1/2 r_{2K+2} as the march
// passes.  x and b are read about once, a few planes ahead of their use; two
// LDS tiles alternate, so each plane takes one barrier.
constexpr int kRTX = 64, kRTY = 4, kRThreads = kRTX * kRTY;
static_assert(2 * (kRTX + kRTY) <= kRThreads, "every halo point needs a thread");

// V: consecutive points per thread along x (the tile is 64 V wide); the
// top and bottom halo rows are read V-wide like the tile, the side columns
// point by point.  The arithmetic per point does not depend on V.
template <typename T, typename A, int V>
__device__ __forceinline__ void k_restrict3_march_body(const Restrict3Args<T, A> &a, const Blk &blk)
{
    constexpr int TW = kRTX * V, TS = TW + 2;   // tile width and LDS row stride (with halo)
    __shared__ A tiles[2][(kRTY + 2) * TS];      // alternate planes: one barrier per plane
    const int tx = threadIdx.x % kRTX, ty = threadIdx.x / kRTX;
    const int i = blk.x * TW + tx * V, j = blk.y * kRTY + ty;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int nok = j < ny && i < nx ? min(V, nx - i) : 0;
    const long long pl = static_cast<long long>(nx) * ny;
    const long long c2 = static_cast<long long>(j) * nx + i;
    const int r = blk.z / ((a.nzc + a.kchunk - 1) / a.kchunk);
    const int K0 = (blk.z % ((a.nzc + a.kchunk - 1) / a.kchunk)) * a.kchunk;
    const int K1 = min(a.nzc, K0 + a.kchunk);
    const T *x = a.x + r * a.xrs;
    const T *b = a.b + r * a.brs;
    // this thread's halo points, if any: V of the top or bottom row, or one
    // of the side columns
    int hy = -1, hx = -1, hw = 0;
    const int t = threadIdx.x;
    if (t < kRTX) { hy = 0; hx = t * V + 1; hw = V; }
    else if (t < 2 * kRTX) { hy = kRTY + 1; hx = (t - kRTX) * V + 1; hw = V; }
    else if (t < 2 * kRTX + kRTY) { hy = t - 2 * kRTX + 1; hx = 0; hw = 1; }
    else if (t < 2 * kRTX + 2 * kRTY) { hy = t - 2 * kRTX - kRTY + 1; hx = TW + 1; hw = 1; }
    const int hi = blk.x * TW + hx - 1, hj = blk.y * kRTY + hy - 1;
    const int hn = hy >= 0 && hi >= 0 && hi < nx && hj >= 0 && hj < ny ? min(hw, nx - hi) : 0;
    const long long hc2 = static_cast<long long>(hj) * nx + hi;
    const int cc = (ty + 1) * TS + tx * V + 1;
    const A cx = a.cx, cy = a.cy;
    // planes this block reads: x up to 2 K1 + 1, b up to 2 K1
    const int kx_last = min(nz - 1, 2 * K1 + 1), kb_last = min(nz - 1, 2 * K1);
    // the next kPre planes of x (centre and halo points) and of b are loaded
    // ahead into small register rings, so that a step waits on a load issued
    // kPre steps before rather than on its own (two: a deeper ring costs
    // registers, and eight waves per SIMD hide more than the ring does)
    constexpr int kPre = 2;
    // loaded planes are held as stored (BF16 packed) until a step uses them
    auto load_x = [&](int k, Held<T, V> &xc, Held<T, V> &xh) {
        const bool live = k >= 0 && k <= kx_last && !a.x_zero;
        hld<T, V>(xc, x + k * pl + c2, live ? nok : 0);
        if constexpr (V == 1) {
            hld<T, V>(xh, x + k * pl + hc2, live ? hn : 0);
        } else {
            if (hw == V)
                hld<T, V>(xh, x + k * pl + hc2, live ? hn : 0);
            else   // a side-column point: element 0 only
                xh.p.e[0] = live && hn ? x[k * pl + hc2] : T{};
        }
    };
    auto load_b = [&](int k, Held<T, V> &v) { hld<T, V>(v, b + k * pl + c2, k <= kb_last ? nok : 0); };
    // window of planes kl-2, kl-1, kl: x and T2 x at this thread's points
    A xw0[V], xw1[V], xw2[V], tw0[V], tw1[V], tw2[V];
#pragma unroll
    for (int e = 0; e < V; ++e) xw0[e] = xw1[e] = xw2[e] = tw0[e] = tw1[e] = tw2[e] = A(0);
    int kl = 2 * K0 - 2;   // next advance takes plane kl + 1
    int kb = 2 * K0;       // next residual plane
    Held<T, V> xq[kPre], hq[kPre], bq[kPre];
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
        hq[q].p = VecPack<T, V>{};
        load_x(kl + 1 + q, xq[q], hq[q]);
        load_b(kb + q, bq[q]);
    }
    int buf = 0;
    auto advance = [&]() {
        ++kl;
        A xc[V], xh[V];
        unpack<T, A, V>(xc, xq[0]);
        unpack<T, A, V>(xh, hq[0]);
        A *tile = tiles[buf];
        buf ^= 1;
#pragma unroll
        for (int e = 0; e < V; ++e) tile[cc + e] = xc[e];
        if (hy >= 0) {
            if (V > 1 && hw == V) {
#pragma unroll
                for (int e = 0; e < V; ++e) tile[hy * TS + hx + e] = xh[e];
            } else {
                tile[hy * TS + hx] = xh[0];
            }
        }
#pragma unroll
        for (int q = 0; q + 1 < kPre; ++q) {
            xq[q] = xq[q + 1];
            hq[q] = hq[q + 1];
        }
        load_x(kl + kPre, xq[kPre - 1], hq[kPre - 1]);
        // a tile is rewritten two planes later, after the next plane's barrier:
        // every read of it is done by then
        __syncthreads();
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const int ce = cc + e;
            const A dx = A(2) * xc[e] - tile[ce - 1] - tile[ce + 1];
            const A dy = A(2) * xc[e] - tile[ce - TS] - tile[ce + TS];
            const A t2 = fmadd(cx, dx, cy * dy);
            xw0[e] = xw1[e]; xw1[e] = xw2[e]; xw2[e] = xc[e];
            tw0[e] = tw1[e]; tw1[e] = tw2[e]; tw2[e] = t2;
        }
    };
    // residual of fine plane k = kb (0 <= k < nz); needs planes k-1, k, k+1 loaded
    auto resid = [&](int k, A (&v)[V]) {
        while (kl < k + 1) advance();
        unpack<T, A, V>(v, bq[0]);
#pragma unroll
        for (int q = 0; q + 1 < kPre; ++q) bq[q] = bq[q + 1];
        load_b(++kb + kPre - 1, bq[kPre - 1]);
        const PlaneCoef<A> ck = a.pc[k];
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] -= fmadd(ck.ca, tw1[e], ck.cb * xw1[e]);
        if (k > 0) {
            const PlaneCoef<A> cm = a.pc[k - 1];
#pragma unroll
            for (int e = 0; e < V; ++e) v[e] -= fmadd(cm.ua, tw0[e], cm.ub * xw0[e]);
        }
        if (k < nz - 1) {
#pragma unroll
            for (int e = 0; e < V; ++e) v[e] -= fmadd(ck.ua, tw2[e], ck.ub * xw2[e]);
        }
    };
    A r_even[V], r_odd[V], r_next[V], out[V];
    resid(2 * K0, r_even);
    for (int K = K0; K < K1; ++K) {
        resid(2 * K + 1, r_odd);
        if (2 * K + 2 < nz) {
            resid(2 * K + 2, r_next);
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) r_next[e] = A(0);
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
            out[e] = fmadd(A(0.5), r_next[e], fmadd(A(0.5), r_even[e], r_odd[e]));
            r_even[e] = r_next[e];
        }
        vst<T, A, V>(a.bc + r * a.crs + K * pl + c2, out, nok);
    }
}

template <typename T, typename A, int V>
__global__ __launch_bounds__(kRThreads) void k_restrict3_march(Restrict3Args<T, A> a)
{
    k_restrict3_march_body<T, A, V>(a, SMG_BLK_XCD);
}

template <typename T, typename A, int V>
__global__ __launch_bounds__(kRThreads) void k_restrict3_march_grp(const GroupEntry *tab, int n)
{
    const Restrict3Args<T, A> *a;
    Blk blk;
    if (!group_entry(tab, n, a, blk)) return;
    k_restrict3_march_body<T, A, V>(*a, blk);
}

inline unsigned blocks_for(long long n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

}  // namespace

template <typename T, typename A, int E>
static void line_relax_e(const LineRelaxArgs<T, A> &a, dim3 grid, hipStream_t st, const LaunchEv &ev)
{
    SMG_LAUNCH(ev, (k_line_relax<T, A, E>), grid, dim3(kBlock), 0, st, a);
}

template <typename T, typename A>
void launch_line_relax(const LineRelaxArgs<T, A> &a, hipStream_t st, const LaunchEv &ev)
{
    const long long waves = static_cast<long long>(a.nq) * a.np * a.nrhs;
    if (waves == 0) return;
    const dim3 grid(blocks_for(waves, kWavesPerBlock));
    const int E = (a.nx + 63) / 64;
    switch (E) {
    case 1: line_relax_e<T, A, 1>(a, grid, st, ev); break;
    case 2: line_relax_e<T, A, 2>(a, grid, st, ev); break;
    case 3: line_relax_e<T, A, 3>(a, grid, st, ev); break;
    case 4: line_relax_e<T, A, 4>(a, grid, st, ev); break;
    case 5: line_relax_e<T, A, 5>(a, grid, st, ev); break;
    case 6: line_relax_e<T, A, 6>(a, grid, st, ev); break;
    case 7: line_relax_e<T, A, 7>(a, grid, st, ev); break;
    case 8: line_relax_e<T, A, 8>(a, grid, st, ev); break;
    default: break;   // nx > 512 is rejected at setup
    }
}

template <typename T, typename A>
void launch_restrict2(const Restrict2Args<T, A> &a, hipStream_t st, const LaunchEv &ev)
{
    const long long n = static_cast<long long>(a.nx) * a.nyc * a.np * a.nrhs;
    if (n == 0) return;
    SMG_LAUNCH(ev, (k_restrict2<T, A>), dim3(blocks_for(n, 256)), dim3(256), 0, st, a);
}

template <typename T, typename A>
void launch_prolong2(const Prolong2Args<T, A> &a, hipStream_t st, const LaunchEv &ev)
{
    const long long n = static_cast<long long>(a.nx) * a.ny * a.np * a.nrhs;
    if (n == 0) return;
    SMG_LAUNCH(ev, (k_prolong2<T, A>), dim3(blocks_for(n, 256)), dim3(256), 0, st, a);
}

template <typename T, typename A>
void launch_resid3(const Resid3Args<T, A> &a, hipStream_t st, const LaunchEv &ev)
{
    if (a.np == 0) return;
    // few registers per point: 16-byte accesses in every precision
    constexpr int V = static_cast<int>(16 / sizeof(T));
    if (V > 1 && a.vmax != 1) {
        auto aligned = [](const void *q) { return reinterpret_cast<uintptr_t>(q) % (V * sizeof(T)) == 0; };
        if (a.nx % V == 0 && a.xrs % V == 0 && a.brs % V == 0 && a.rrs % V == 0 && a.rps % V == 0 &&
            aligned(a.x) && aligned(a.b) && aligned(a.r)) {
            const long long pts = static_cast<long long>(a.nx) * a.ny / V;
            const dim3 grid(blocks_for(pts, 256), a.np, a.nrhs);
            SMG_LAUNCH_G(ev, (k_resid3v<T, A, V>), (k_resid3v_grp<T, A, V>), grid, dim3(256), 0, st, a);
            return;
        }
    }
    const dim3 grid(blocks_for(static_cast<long long>(a.nx) * a.ny, 256), a.np, a.nrhs);
    SMG_LAUNCH_G(ev, (k_resid3v<T, A, 1>), (k_resid3v_grp<T, A, 1>), grid, dim3(256), 0, st, a);
}

template <typename T, typename A>
void launch_correct3(const Correct3Args<T, A> &a, hipStream_t st, const LaunchEv &ev)
{
    if (a.np == 0) return;
    const dim3 grid(blocks_for(static_cast<long long>(a.nx) * a.ny, 256), a.np, a.nrhs);
    SMG_LAUNCH(ev, (k_correct3<T, A>), grid, dim3(256), 0, st, a);
}

template <typename T, typename A, int V>
void launch_restrict3_march(const Restrict3Args<T, A> &a, hipStream_t st, const LaunchEv &ev)
{
    const int gx = (a.nx + kRTX * V - 1) / (kRTX * V), gy = (a.ny + kRTY - 1) / kRTY;
    // enough blocks to fill the chip; each marches kchunk coarse planes
    int nzb = 2048 / (gx * gy * a.nrhs);
    nzb = nzb < 1 ? 1 : (nzb > a.nzc ? a.nzc : nzb);
    const int kchunk = (a.nzc + nzb - 1) / nzb;
    nzb = (a.nzc + kchunk - 1) / kchunk;
    const dim3 grid(gx, gy, nzb * a.nrhs);
    Restrict3Args<T, A> am = a;
    am.kchunk = kchunk;
    SMG_LAUNCH_G(ev, (k_restrict3_march<T, A, V>), (k_restrict3_march_grp<T, A, V>), grid, dim3(kRThreads), 0, st,
                 am);
}

template <typename T, typename A>
void launch_restrict3(const Restrict3Args<T, A> &a, hipStream_t st, const LaunchEv &ev)
{
    if (a.nzc >= 2) {
        // FP64 rows take 16-byte accesses (two points), narrower types 8 bytes
        constexpr int kWidest = sizeof(T) == 8 ? 2 : stream_vec<T>();
        int v = a.vmax == 1 ? 1 : tile_vec<T>(a.nx, kWidest);
        auto aligned = [&](const void *q) { return reinterpret_cast<uintptr_t>(q) % (v * sizeof(T)) == 0; };
        if (v > 1 && !(a.xrs % v == 0 && a.brs % v == 0 && a.crs % v == 0 && aligned(a.x) && aligned(a.b) &&
                       aligned(a.bc)))
            v = 1;
        if (v == 4) {
            if constexpr (kWidest >= 4) launch_restrict3_march<T, A, 4>(a, st, ev);
        } else if (v == 2) {
            if constexpr (kWidest >= 2) launch_restrict3_march<T, A, 2>(a, st, ev);
        } else {
            launch_restrict3_march<T, A, 1>(a, st, ev);
        }
        return;
    }
    const dim3 grid(blocks_for(static_cast<long long>(a.nx) * a.ny, 256), a.nzc, a.nrhs);
    SMG_LAUNCH_G(ev, (k_restrict3<T, A>), (k_restrict3_grp<T, A>), grid, dim3(256), 0, st, a);
}

template <typename T, typename A>
void launch_prolong3(const Prolong3Args<T, A> &a, hipStream_t st, const LaunchEv &ev)
{
    const dim3 grid(blocks_for(static_cast<long long>(a.nx) * a.ny, 256), a.nz, a.nrhs);
    SMG_LAUNCH(ev, (k_prolong3<T, A>), grid, dim3(256), 0, st, a);
}

template <typename A>
void launch_thomas_tables(const LineCoef<double> *uniq_ab, int nfac, int nx, int nxp, Fac<A> *out, hipStream_t st)
{
    hipLaunchKernelGGL((k_thomas_tables<A>), dim3(blocks_for(nfac, 64)), dim3(64), 0, st, uniq_ab, nfac, nx, nxp,
                       out);
}

template <typename T>
void launch_convert_in(const double *src, long long lds, T *dst, long long ldd, size_t n, int nrhs, hipStream_t st)
{
    hipLaunchKernelGGL((k_convert_in<T>), dim3(blocks_for(static_cast<long long>(n), 256), nrhs), dim3(256), 0, st,
                       src, lds, dst, ldd, n);
}

template <typename T>
void launch_convert_out(const T *src, long long lds, double *dst, long long ldd, size_t n, int nrhs, hipStream_t st)
{
    hipLaunchKernelGGL((k_convert_out<T>), dim3(blocks_for(static_cast<long long>(n), 256), nrhs), dim3(256), 0, st,
                       src, lds, dst, ldd, n);
}

#define SMG_INSTANTIATE(T, A)                                                          \
    template void launch_line_relax<T, A>(const LineRelaxArgs<T, A> &, hipStream_t, const LaunchEv &); \
    template void launch_restrict2<T, A>(const Restrict2Args<T, A> &, hipStream_t, const LaunchEv &);     \
    template void launch_prolong2<T, A>(const Prolong2Args<T, A> &, hipStream_t, const LaunchEv &);       \
    template void launch_resid3<T, A>(const Resid3Args<T, A> &, hipStream_t, const LaunchEv &);           \
    template void launch_correct3<T, A>(const Correct3Args<T, A> &, hipStream_t, const LaunchEv &);       \
    template void launch_restrict3<T, A>(const Restrict3Args<T, A> &, hipStream_t, const LaunchEv &);     \
    template void launch_prolong3<T, A>(const Prolong3Args<T, A> &, hipStream_t, const LaunchEv &);

SMG_INSTANTIATE(double, double)
SMG_INSTANTIATE(float, float)
SMG_INSTANTIATE(bf16, float)

template void launch_thomas_tables<double>(const LineCoef<double> *, int, int, int, Fac<double> *, hipStream_t);
template void launch_thomas_tables<float>(const LineCoef<double> *, int, int, int, Fac<float> *, hipStream_t);
template void launch_convert_in<float>(const double *, long long, float *, long long, size_t, int, hipStream_t);
template void launch_convert_in<bf16>(const double *, long long, bf16 *, long long, size_t, int, hipStream_t);
template void launch_convert_out<float>(const float *, long long, double *, long long, size_t, int, hipStream_t);
template void launch_convert_out<bf16>(const bf16 *, long long, double *, long long, size_t, int, hipStream_t);

}  // namespace smg
