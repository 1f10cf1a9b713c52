// Fused 2D/3D V-cycle kernels (gfx950, wave64).
//
// The stage-by-stage schedule of smg_kernels.hip launches four kernels per 2D
// level (F relax, C relax, residual+restriction, prolongation+correction),
// ~600 mostly tiny launches per 256^3 V-cycle.  These kernels cover the same
// arithmetic with far fewer launches:
//   k2_down   one launch per fine 2D level: for a strip of S coarse lines a
//             workgroup solves the F lines it needs (zero initial guess), then
//             the C lines, keeps both in LDS, writes its own lines of x, and
//             forms the restricted residual of its coarse lines;
//   k2_coarse one workgroup per plane runs the whole remaining 2D sub-cycle on
//             the small levels with every line in LDS;
//   k2_chain  without post-smoothing the upward half of the 2D cycle is a
//             chain of prolongations, x_0 + P(x_1 + P(x_2 + ...)); a workgroup
//             stages the coarse windows of a run of fine lines in LDS once and
//             adds the result straight into the 3D iterate;
//   k2_up     with one post-smoothing step: prolongation, C-line and F-line
//             relaxation of a strip (with a two-line halo) in one launch;
//   k3_chain  the prolongation chain over the 3D levels, tiled the same way.
// Workgroups have W = 16 waves so that each wave handles one line per phase;
// every global load a workgroup needs is issued before its first barrier.
// Lines are held in registers (E = ceil(nx/64) points per lane) and stored in
// LDS lane-interleaved (point e of lane l at [e*64 + l]): conflict-free.
#include "group.h"
#include "line_ops.hpp"

namespace smg {

namespace {

using namespace lineops;

constexpr int kW = 16;                 // waves per workgroup
constexpr int kThreads = 64 * kW;

__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

template <typename A>
__device__ inline const LineCoef<A> *plane_lines(const PlaneCoef<A> *pc, int k, const LineCoef<A> *lc0, int lines_total)
{
    return lc0 + static_cast<size_t>(pc[k].pt) * lines_total;
}

// ---------------------------------------------------------------------------
// k2_down: one pre-smoothing zebra sweep (F then C, zero initial guess) of a
// strip of coarse lines [J0, J1), the strip's own lines of x, and the
// restricted residual b_c[J] = 1/2 r_{2J} + r_{2J+1} + 1/2 r_{2J+2}.  After
// such a sweep r_{2J+1} = 0 (the C line was solved against its final
// neighbours) and r_j = -V_{j-1} x_{j-1} - V_j x_{j+1} on an F line (it was
// solved with zero neighbours, so b_j - L_j x_j = 0): the restriction needs
// the C lines only.  Equal to the explicit residual up to rounding.
// LDS slot s holds fine line j = 2*J0 - 2 + s, s in [0, 2S+5).  The host
// keeps S <= W - 3 so that every phase is one line per wave.
// ---------------------------------------------------------------------------
template <typename T, typename A, int E>
__device__ __forceinline__ void k2_down_body(const Down2Args<T, A> &a, const Blk &blk)
{
    extern __shared__ unsigned char smem_raw[];
    A *xs = reinterpret_cast<A *>(smem_raw);
    const int lane = threadIdx.x & 63, w = wave_id();
    const int nstrip = (a.nyc + a.S - 1) / a.S;
    const int strip = blk.x % nstrip;
    const int p = (blk.x / nstrip) % a.np;
    const int r = blk.x / (nstrip * a.np);
    const int J0 = strip * a.S, J1 = min(J0 + a.S, a.nyc);
    const int ny = a.ny, nx = a.nx, nxp = a.nxp;
    const int base = 2 * J0 - 2;
    const int jlo = max(0, base), jhi = min(ny - 1, 2 * J1 + 2);
    const int k = p * a.kmul + a.koff;
    const LineCoef<A> *lc = plane_lines(a.pc, k, a.lc, a.lines_total);
    const T *bpl = a.b + r * a.brs + p * a.bps;
    T *xpl = a.x + r * a.xrs + p * a.xps;

    const int f0 = jlo + (jlo & 1), c0 = jlo | 1;
    const int nf = f0 <= jhi ? (jhi - f0) / 2 + 1 : 0;
    const int nc = c0 <= jhi ? (jhi - c0) / 2 + 1 : 0;
    const int jf = f0 + 2 * w, jc = c0 + 2 * w, J = J0 + w;
    const bool hf = w < nf, hc = w < nc, hr = J < J1;

    // every global read of the workgroup, issued up front
    A fb[E], cb[E];
    if (hf) gload<T, A, E>(fb, bpl + static_cast<long long>(jf) * nx, nx, lane);
    if (hc) gload<T, A, E>(cb, bpl + static_cast<long long>(jc) * nx, nx, lane);
    // F lines: x_j = L_j^{-1} b_j
    if (hf) {
        thomas<A, E>(fb, a.fac + static_cast<size_t>(lc[jf].fac) * nxp, lane);
        sstore<A, E>(xs + (jf - base) * nxp, fb, lane);
    }
    __syncthreads();
    // C lines: x_j = L_j^{-1} (b_j - V_{j-1} x_{j-1} - V_j x_{j+1})
    if (hc) {
        A v[E];
        const LineCoef<A> cm = lc[jc - 1];
        sload<A, E>(v, xs + (jc - 1 - base) * nxp, lane);
        sub_op<A, E>(cb, v, cm.va, cm.vb);
        if (jc + 1 < ny) {
            const LineCoef<A> cj = lc[jc];
            sload<A, E>(v, xs + (jc + 1 - base) * nxp, lane);
            sub_op<A, E>(cb, v, cj.va, cj.vb);
        }
        thomas<A, E>(cb, a.fac + static_cast<size_t>(lc[jc].fac) * nxp, lane);
        sstore<A, E>(xs + (jc - base) * nxp, cb, lane);
    }
    __syncthreads();
    // own lines of x: [2 J0, 2 J1), plus the last fine line for the last strip
    {
        const int o0 = 2 * J0;
        const int o1 = (J1 == a.nyc) ? ny : 2 * J1;
        for (int j = o0 + w; j < o1; j += kW) {
            A v[E];
            sload<A, E>(v, xs + (j - base) * nxp, lane);
            gstore<T, A, E>(xpl + static_cast<long long>(j) * nx, v, nx, lane);
        }
    }
    // restricted residual of coarse line J after one sweep from zero: the C
    // lines' residuals are zero and an F line's is -V_{j-1} x_{j-1} - V_j x_{j+1}
    if (hr) {
        A acc[E], t[E], v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = A(0);
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const int j = 2 * J + 2 * d;   // F lines 2J and 2J + 2
            if (j >= ny) break;
#pragma unroll
            for (int e = 0; e < E; ++e) t[e] = A(0);
            if (j > 0) {
                const LineCoef<A> cm = lc[j - 1];
                sload<A, E>(v, xs + (j - 1 - base) * nxp, lane);
                sub_op<A, E>(t, v, cm.va, cm.vb);
            }
            if (j + 1 < ny) {
                const LineCoef<A> cj = lc[j];
                sload<A, E>(v, xs + (j + 1 - base) * nxp, lane);
                sub_op<A, E>(t, v, cj.va, cj.vb);
            }
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] += A(0.5) * t[e];
        }
        gstore<T, A, E>(a.bc + r * a.crs + p * a.cps + static_cast<long long>(J) * nx, acc, nx, lane);
    }
}

template <typename T, typename A, int E>
__global__ __launch_bounds__(kThreads) void k2_down(Down2Args<T, A> a)
{
    k2_down_body<T, A, E>(a, SMG_BLK_HW);
}

template <typename T, typename A, int E>
__global__ __launch_bounds__(kThreads) void k2_down_grp(const GroupEntry *tab, int n)
{
    const Down2Args<T, A> *a;
    Blk blk;
    if (!group_entry(tab, n, a, blk)) return;
    k2_down_body<T, A, E>(*a, blk);
}

// grouped launch for any E <= 4 (boxes of different widths share one launch)
template <typename T, typename A>
__global__ __launch_bounds__(kThreads) void k2_down_grp_e4(const GroupEntry *tab, int n)
{
    const Down2Args<T, A> *a;
    Blk blk;
    if (!group_entry(tab, n, a, blk)) return;
    switch (a->nxp / 64) {
    case 1: k2_down_body<T, A, 1>(*a, blk); break;
    case 2: k2_down_body<T, A, 2>(*a, blk); break;
    case 3: k2_down_body<T, A, 3>(*a, blk); break;
    default: k2_down_body<T, A, 4>(*a, blk); break;
    }
}

// ---------------------------------------------------------------------------
// k2_down_reg: the same stage with one wave per coarse line J and nothing but
// registers: the wave solves the F lines 2J-2, 2J, 2J+2, 2J+4 and the C lines
// 2J-1, 2J+1, 2J+3 it needs (its neighbours solve some of them again), forms
// b_c[J], and writes its own lines 2J and 2J+1 (and the last line of an odd
// level).  No barrier and no LDS: a wave never waits for another.  Used when a
// line fits in 4 points per lane (nx <= 256).
// ---------------------------------------------------------------------------
template <typename T, typename A, int E>
__device__ __forceinline__ void k2_down_reg_body(const Down2Args<T, A> &a, const Blk &blk)
{
    const int lane = threadIdx.x & 63;
    const long long wv = static_cast<long long>(blk.x) * 4 + wave_id();
    const long long total = static_cast<long long>(a.nyc) * a.np * a.nrhs;
    if (wv >= total) return;   // whole waves
    const int J = static_cast<int>(wv % a.nyc);
    const long long t = wv / a.nyc;
    const int p = static_cast<int>(t % a.np), r = static_cast<int>(t / a.np);
    const int ny = a.ny, nx = a.nx, nxp = a.nxp;
    const int k = p * a.kmul + a.koff;
    const LineCoef<A> *lc = plane_lines(a.pc, k, a.lc, a.lines_total);
    const T *bpl = a.b + r * a.brs + p * a.bps;
    T *xpl = a.x + r * a.xrs + p * a.xps;
    const int j0 = 2 * J;   // lines j0-2 .. j0+4 around the coarse line
    const bool has_m2 = j0 >= 2, has_p2 = j0 + 2 < ny, has_p3 = j0 + 3 < ny, has_p4 = j0 + 4 < ny;

    // all right-hand sides first (F: j0-2, j0, j0+2, j0+4; C: j0-1, j0+1, j0+3)
    A fm2[E], f0[E], fp2[E], fp4[E], cm1[E], cp1[E], cp3[E];
#pragma unroll
    for (int e = 0; e < E; ++e) fm2[e] = fp2[e] = fp4[e] = cm1[e] = cp3[e] = A(0);
    if (has_m2) {
        gload<T, A, E>(fm2, bpl + static_cast<long long>(j0 - 2) * nx, nx, lane);
        gload<T, A, E>(cm1, bpl + static_cast<long long>(j0 - 1) * nx, nx, lane);
    }
    gload<T, A, E>(f0, bpl + static_cast<long long>(j0) * nx, nx, lane);
    gload<T, A, E>(cp1, bpl + static_cast<long long>(j0 + 1) * nx, nx, lane);
    if (has_p2) gload<T, A, E>(fp2, bpl + static_cast<long long>(j0 + 2) * nx, nx, lane);
    if (has_p3) gload<T, A, E>(cp3, bpl + static_cast<long long>(j0 + 3) * nx, nx, lane);
    if (has_p4) gload<T, A, E>(fp4, bpl + static_cast<long long>(j0 + 4) * nx, nx, lane);
    // interior lines share one Thomas table: plan it once
    const int fi = lc[j0].fac;
    LinePlan<A, E> plan;
    make_plan<A, E>(plan, a.fac + static_cast<size_t>(fi) * nxp, lane);
    auto solve = [&](A (&x)[E], int j) {
        const int fj = lc[j].fac;
        if (fj == fi)
            solve_plan<A, E>(x, plan, lane);
        else
            thomas<A, E>(x, a.fac + static_cast<size_t>(fj) * nxp, lane);
    };
    if (has_m2) solve(fm2, j0 - 2);
    solve(f0, j0);
    if (has_p2) solve(fp2, j0 + 2);
    if (has_p4) solve(fp4, j0 + 4);
    // C line j: (b_j - V_{j-1} x_{j-1} - V_j x_{j+1}), then the exact solve
    auto solve_c = [&](A (&x)[E], int j, const A (&xl)[E], const A (&xr)[E]) {
        const LineCoef<A> cm = lc[j - 1];
        sub_op<A, E>(x, xl, cm.va, cm.vb);
        if (j + 1 < ny) {
            const LineCoef<A> cj = lc[j];
            sub_op<A, E>(x, xr, cj.va, cj.vb);
        }
        solve(x, j);
    };
    if (has_m2) solve_c(cm1, j0 - 1, fm2, f0);
    solve_c(cp1, j0 + 1, f0, fp2);            // j0 + 1 < ny always (J < nyc)
    if (has_p3) solve_c(cp3, j0 + 3, fp2, fp4);
    // own lines
    gstore<T, A, E>(xpl + static_cast<long long>(j0) * nx, f0, nx, lane);
    gstore<T, A, E>(xpl + static_cast<long long>(j0 + 1) * nx, cp1, nx, lane);
    if (J == a.nyc - 1 && has_p2) gstore<T, A, E>(xpl + static_cast<long long>(j0 + 2) * nx, fp2, nx, lane);
    // b_c[J] = 1/2 r_j0 + r_j0+1 + 1/2 r_j0+2 after one sweep from zero: the
    // C line's residual is zero (just solved against its final neighbours)
    // and an F line's is -V_{j-1} x_{j-1} - V_j x_{j+1} (b_j - L_j x_j = 0:
    // it was solved with zero neighbours)
    A acc[E], rf[E];
#pragma unroll
    for (int e = 0; e < E; ++e) rf[e] = A(0);
    if (has_m2) {
        const LineCoef<A> cm = lc[j0 - 1];
        sub_op<A, E>(rf, cm1, cm.va, cm.vb);
    }
    {
        const LineCoef<A> cj = lc[j0];
        sub_op<A, E>(rf, cp1, cj.va, cj.vb);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = A(0.5) * rf[e];
    if (has_p2) {
#pragma unroll
        for (int e = 0; e < E; ++e) rf[e] = A(0);
        const LineCoef<A> cm = lc[j0 + 1];
        sub_op<A, E>(rf, cp1, cm.va, cm.vb);
        if (has_p3) {
            const LineCoef<A> cj = lc[j0 + 2];
            sub_op<A, E>(rf, cp3, cj.va, cj.vb);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] += A(0.5) * rf[e];
    }
    gstore<T, A, E>(a.bc + r * a.crs + p * a.cps + static_cast<long long>(J) * nx, acc, nx, lane);
}

template <typename T, typename A, int E>
__global__ __launch_bounds__(256) void k2_down_reg(Down2Args<T, A> a)
{
    k2_down_reg_body<T, A, E>(a, SMG_BLK_HW);
}

template <typename T, typename A, int E>
__global__ __launch_bounds__(256) void k2_down_reg_grp(const GroupEntry *tab, int n)
{
    const Down2Args<T, A> *a;
    Blk blk;
    if (!group_entry(tab, n, a, blk)) return;
    k2_down_reg_body<T, A, E>(*a, blk);
}

// grouped launch for any E <= 4 (boxes of different widths share one launch)
template <typename T, typename A>
__global__ __launch_bounds__(256) void k2_down_reg_grp_e4(const GroupEntry *tab, int n)
{
    const Down2Args<T, A> *a;
    Blk blk;
    if (!group_entry(tab, n, a, blk)) return;
    switch (a->nxp / 64) {
    case 1: k2_down_reg_body<T, A, 1>(*a, blk); break;
    case 2: k2_down_reg_body<T, A, 2>(*a, blk); break;
    case 3: k2_down_reg_body<T, A, 3>(*a, blk); break;
    default: k2_down_reg_body<T, A, 4>(*a, blk); break;
    }
}

// ---------------------------------------------------------------------------
// k2_down_march: the same stage with one wave per run of K = a.kr coarse lines
// J0 .. J0+K-1, marching upward in y.  The wave keeps x_{2J}, x_{2J+1},
// x_{2J+2}, the residual r_{2J} and the right-hand sides b_{2J+1}, b_{2J+2};
// each step solves F line 2J+4 and C line 2J+3 and forms r_{2J+1}, r_{2J+2}
// and b_c[J].  A run costs 2K + 5 line solves for 2K lines (K = 1: the seven
// solves of k2_down_reg) and reads each right-hand side once, apart from the
// five lines its start-up shares with the previous run.  The right-hand sides
// of the next step are loaded one step ahead.  Arithmetic per line is that of
// k2_down_reg (up to how the compiler fuses multiply-adds).
// ---------------------------------------------------------------------------
template <typename T, typename A, int E>
__device__ __forceinline__ void k2_down_march_body(const Down2Args<T, A> &a, const Blk &blk)
{
    const int lane = threadIdx.x & 63;
    const int K = a.kr;
    const int nrun = (a.nyc + K - 1) / K;
    const long long wv = static_cast<long long>(blk.x) * 4 + wave_id();
    const long long total = static_cast<long long>(nrun) * a.np * a.nrhs;
    if (wv >= total) return;   // whole waves
    const int run = static_cast<int>(wv % nrun);
    const long long t = wv / nrun;
    const int p = static_cast<int>(t % a.np), r = static_cast<int>(t / a.np);
    const int ny = a.ny, nx = a.nx, nxp = a.nxp;
    const int k = p * a.kmul + a.koff;
    const LineCoef<A> *lc = plane_lines(a.pc, k, a.lc, a.lines_total);
    const T *bpl = a.b + r * a.brs + p * a.bps;
    T *xpl = a.x + r * a.xrs + p * a.xps;
    T *bcpl = a.bc + r * a.crs + p * a.cps;
    const int J0 = run * K, J1 = min(J0 + K, a.nyc);
    const int j0 = 2 * J0;

    const int fi = lc[j0].fac;
    LinePlan<A, E> plan;
    make_plan<A, E>(plan, a.fac + static_cast<size_t>(fi) * nxp, lane);
    auto solve = [&](A (&x)[E], int j) {
        const int fj = lc[j].fac;
        if (fj == fi)
            solve_plan<A, E>(x, plan, lane);
        else
            thomas<A, E>(x, a.fac + static_cast<size_t>(fj) * nxp, lane);
    };
    auto solve_c = [&](A (&x)[E], int j, const A (&xl)[E], const A (&xr)[E]) {
        const LineCoef<A> cm = lc[j - 1];
        sub_op<A, E>(x, xl, cm.va, cm.vb);
        if (j + 1 < ny) {
            const LineCoef<A> cj = lc[j];
            sub_op<A, E>(x, xr, cj.va, cj.vb);
        }
        solve(x, j);
    };
    auto zero = [](A (&v)[E]) {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = A(0);
    };
    auto copy = [](A (&d)[E], const A (&v)[E]) {
#pragma unroll
        for (int e = 0; e < E; ++e) d[e] = v[e];
    };

    // b_c[J] = 1/2 (r_{2J} + r_{2J+2}) with the F-line residuals of one sweep
    // from zero, r_j = -V_{j-1} x_{j-1} - V_j x_{j+1} (the C lines' are zero)
    auto f_resid = [&](A (&rr)[E], int j, const A (&xl)[E], const A (&xr)[E]) {
#pragma unroll
        for (int e = 0; e < E; ++e) rr[e] = A(0);
        if (j > 0) {
            const LineCoef<A> cm = lc[j - 1];
            sub_op<A, E>(rr, xl, cm.va, cm.vb);
        }
        if (j + 1 < ny) {
            const LineCoef<A> cj = lc[j];
            sub_op<A, E>(rr, xr, cj.va, cj.vb);
        }
    };
    // start-up: x_{j0-2}, x_{j0-1} (first run: none), x_{j0}, x_{j0+1}, x_{j0+2}, r_{j0}
    A xa[E], xc[E], xb[E], rp[E], n3[E], n4[E];
    {
        A fm2[E], cm1[E];
        zero(fm2);
        zero(cm1);
        zero(xb);
        zero(n3);
        zero(n4);
        const bool has_m2 = j0 >= 2;
        if (has_m2) {
            gload<T, A, E>(fm2, bpl + static_cast<long long>(j0 - 2) * nx, nx, lane);
            gload<T, A, E>(cm1, bpl + static_cast<long long>(j0 - 1) * nx, nx, lane);
        }
        gload<T, A, E>(xa, bpl + static_cast<long long>(j0) * nx, nx, lane);
        gload<T, A, E>(xc, bpl + static_cast<long long>(j0 + 1) * nx, nx, lane);
        if (j0 + 2 < ny) gload<T, A, E>(xb, bpl + static_cast<long long>(j0 + 2) * nx, nx, lane);
        if (j0 + 3 < ny) gload<T, A, E>(n3, bpl + static_cast<long long>(j0 + 3) * nx, nx, lane);
        if (j0 + 4 < ny) gload<T, A, E>(n4, bpl + static_cast<long long>(j0 + 4) * nx, nx, lane);
        if (has_m2) solve(fm2, j0 - 2);
        solve(xa, j0);
        if (j0 + 2 < ny) solve(xb, j0 + 2);
        if (has_m2) solve_c(cm1, j0 - 1, fm2, xa);
        solve_c(xc, j0 + 1, xa, xb);   // j0 + 1 < ny always (J0 < nyc)
        f_resid(rp, j0, cm1, xc);
    }
    for (int J = J0; J < J1; ++J) {
        // state: xa = x_j, xc = x_{j+1}, xb = x_{j+2}, rp = r_j,
        // n3 = b_{j+3}, n4 = b_{j+4} (zero beyond the level)
        const int j = 2 * J;
        const bool h2 = j + 2 < ny, h3 = j + 3 < ny, h4 = j + 4 < ny;
        A xe[E], xd[E];
        copy(xe, n3);
        copy(xd, n4);
        if (J + 1 < J1) {   // the next step's right-hand sides, one step ahead
            zero(n3);
            zero(n4);
            if (j + 5 < ny) gload<T, A, E>(n3, bpl + static_cast<long long>(j + 5) * nx, nx, lane);
            if (j + 6 < ny) gload<T, A, E>(n4, bpl + static_cast<long long>(j + 6) * nx, nx, lane);
        }
        gstore<T, A, E>(xpl + static_cast<long long>(j) * nx, xa, nx, lane);
        gstore<T, A, E>(xpl + static_cast<long long>(j + 1) * nx, xc, nx, lane);
        if (J == a.nyc - 1 && h2) gstore<T, A, E>(xpl + static_cast<long long>(j + 2) * nx, xb, nx, lane);
        // x_{j+4}, x_{j+3}
        if (h4) solve(xd, j + 4);
        if (h3) solve_c(xe, j + 3, xb, xd);
        A acc[E];
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = A(0.5) * rp[e];
        if (h2) {
            f_resid(rp, j + 2, xc, xe);   // r_{j+2}
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] += A(0.5) * rp[e];
        }
        gstore<T, A, E>(bcpl + static_cast<long long>(J) * nx, acc, nx, lane);
        copy(xa, xb);
        copy(xc, xe);
        copy(xb, xd);
    }
}

template <typename T, typename A, int E>
__global__ __launch_bounds__(256) void k2_down_march(Down2Args<T, A> a)
{
    k2_down_march_body<T, A, E>(a, SMG_BLK_HW);
}

template <typename T, typename A>
__global__ __launch_bounds__(256) void k2_down_march_grp_e4(const GroupEntry *tab, int n)
{
    const Down2Args<T, A> *a;
    Blk blk;
    if (!group_entry(tab, n, a, blk)) return;
    switch (a->nxp / 64) {
    case 1: k2_down_march_body<T, A, 1>(*a, blk); break;
    case 2: k2_down_march_body<T, A, 2>(*a, blk); break;
    case 3: k2_down_march_body<T, A, 3>(*a, blk); break;
    default: k2_down_march_body<T, A, 4>(*a, blk); break;
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
    for (int t = w; t < n; t += kW) {
        const int j = 2 * t + colour;
        A f[E], v[E];
        sload<A, E>(f, bs + j * nxp, lane);
        if (!nbr_zero) {
            if (j > 0) {
                const LineCoef<A> cm = lc[j - 1];
                sload<A, E>(v, xs + (j - 1) * nxp, lane);
                sub_op<A, E>(f, v, cm.va, cm.vb);
            }
            if (j + 1 < ny) {
                const LineCoef<A> cj = lc[j];
                sload<A, E>(v, xs + (j + 1) * nxp, lane);
                sub_op<A, E>(f, v, cj.va, cj.vb);
            }
        }
        thomas<A, E>(f, fac + static_cast<size_t>(lc[j].fac) * nxp, lane);
        sstore<A, E>(xs + j * nxp, f, lane);
    }
}

// k2_coarse in down-only mode: levels l0 .. nlev-1 of the downward half of
// the 2D cycle (one sweep from zero, no post-smoothing).  LDS holds the
// current level's b and x only: after the C half-sweep a level's b is dead
// (the restriction needs the C lines alone), so b_{l+1} overwrites it in
// place.  Each solved line also goes to xl[l] for the prolongation chain,
// which runs from the coarsest level in the next launch.
template <typename T, typename A, int E>
__device__ __forceinline__ void k2_coarse_down_body(const Coarse2Args<T, A> &a, const Blk &blk)
{
    extern __shared__ unsigned char smem_raw[];
    A *sm = reinterpret_cast<A *>(smem_raw);
    const int lane = threadIdx.x & 63, w = wave_id();
    const int p = blk.x % a.np, r = blk.x / a.np;
    const int nx = a.nx, nxp = a.nxp;
    const int k = p * a.kmul + a.koff;
    const LineCoef<A> *lcp = plane_lines(a.pc, k, a.lc, a.lines_total);
    const int n0 = a.ny2[a.l0];
    int total = 0;
    for (int l = a.l0; l < a.nlev; ++l) total += a.ny2[l];
    A *xs = sm, *bs = sm + static_cast<size_t>(n0) * nxp;
    LineCoef<A> *lcs = reinterpret_cast<LineCoef<A> *>(bs + static_cast<size_t>(n0) * nxp);
    auto off = [&](int l) {
        int o = 0;
        for (int m = a.l0; m < l; ++m) o += a.ny2[m];
        return o;
    };
    auto xrow = [&](int l, int j) {
        const long long ps = static_cast<long long>(nx) * a.ny2[l];
        return a.xl[l] + r * (a.P2 * ps) + p * ps + static_cast<long long>(j) * nx;
    };
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
        int l = a.l0, o = 0;
        while (i >= o + a.ny2[l]) o += a.ny2[l++];
        lcs[i] = lcp[a.lev_off[l] + (i - o)];
    }
    {
        const T *bpl = a.b + r * a.brs + p * a.bps;
        for (int j = w; j < n0; j += kW) {
            A v[E];
            gload<T, A, E>(v, bpl + static_cast<long long>(j) * nx, nx, lane);
            sstore<A, E>(bs + j * nxp, v, lane);
        }
    }
    __syncthreads();
    // the Thomas table rows of the line this wave solves next, loaded one
    // phase ahead (its global latency then hides behind a solve and a barrier)
    LinePlan<A, E> P;
    int pf = -1;
    auto prefetch = [&](int l, int j) {
        pf = -1;
        if (l < a.nlev && j < a.ny2[l]) {
            pf = __builtin_amdgcn_readfirstlane(lcs[off(l) + j].fac);
            load_fac<A, E>(P.g, P.h, a.fac + static_cast<size_t>(pf) * nxp, lane);
        }
    };
    auto solve = [&](A (&f)[E], int fi) {
        fi = __builtin_amdgcn_readfirstlane(fi);
        if (fi != pf) load_fac<A, E>(P.g, P.h, a.fac + static_cast<size_t>(fi) * nxp, lane);
        plan_products<A, E>(P, lane);
        solve_plan<A, E>(f, P, lane);
        pf = -1;
    };
    prefetch(a.l0, 2 * w);
    for (int l = a.l0; l < a.nlev - 1; ++l) {
        const int ny = a.ny2[l], nyc = a.ny2[l + 1];
        const LineCoef<A> *lc = lcs + off(l);
        // F lines from b alone, then C lines against them
        for (int colour = 0; colour < 2; ++colour) {
            const int n = colour == 0 ? (ny + 1) / 2 : ny / 2;
            for (int t = w; t < n; t += kW) {
                const int j = 2 * t + colour;
                A f[E], v[E];
                sload<A, E>(f, bs + j * nxp, lane);
                if (colour == 1) {
                    const LineCoef<A> cm = lc[j - 1];
                    sload<A, E>(v, xs + (j - 1) * nxp, lane);
                    sub_op<A, E>(f, v, cm.va, cm.vb);
                    if (j + 1 < ny) {
                        const LineCoef<A> cj = lc[j];
                        sload<A, E>(v, xs + (j + 1) * nxp, lane);
                        sub_op<A, E>(f, v, cj.va, cj.vb);
                    }
                }
                solve(f, lc[j].fac);
                sstore<A, E>(xs + j * nxp, f, lane);
                gstore<T, A, E>(xrow(l, j), f, nx, lane);
            }
            // next: this level's C line, or the next level's F line (the
            // coarsest level's line for wave 0)
            if (colour == 0)
                prefetch(l, 2 * w + 1);
            else if (l + 1 < a.nlev - 1)
                prefetch(l + 1, 2 * w);
            else if (w == 0)
                prefetch(a.nlev - 1, 0);
            __syncthreads();
        }
        // b_{l+1}[J] = 1/2 (r_{2J} + r_{2J+2}), r_j = -V_{j-1} x_{j-1} - V_j x_{j+1}
        for (int J = w; J < nyc; J += kW) {
            A acc[E];
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] = A(0);
            for (int d = 0; d < 2; ++d) {
                const int j = 2 * J + 2 * d;
                if (j >= ny) break;
                A f[E], v[E];
#pragma unroll
                for (int e = 0; e < E; ++e) f[e] = A(0);
                if (j > 0) {
                    const LineCoef<A> cm = lc[j - 1];
                    sload<A, E>(v, xs + (j - 1) * nxp, lane);
                    sub_op<A, E>(f, v, cm.va, cm.vb);
                }
                if (j + 1 < ny) {
                    const LineCoef<A> cj = lc[j];
                    sload<A, E>(v, xs + (j + 1) * nxp, lane);
                    sub_op<A, E>(f, v, cj.va, cj.vb);
                }
#pragma unroll
                for (int e = 0; e < E; ++e) acc[e] += A(0.5) * f[e];
            }
            sstore<A, E>(bs + J * nxp, acc, lane);
        }
        __syncthreads();
    }
    if (w == 0) {   // the coarsest level: one line
        const int l = a.nlev - 1;
        A f[E];
        sload<A, E>(f, bs, lane);
        solve(f, lcs[off(l)].fac);
        gstore<T, A, E>(xrow(l, 0), f, nx, lane);
    }
}

template <typename T, typename A, int E>
__device__ __forceinline__ void k2_coarse_body(const Coarse2Args<T, A> &a, const Blk &blk)
{
    if (a.down_only) {
        k2_coarse_down_body<T, A, E>(a, blk);
        return;
    }
    extern __shared__ unsigned char smem_raw[];
    A *sm = reinterpret_cast<A *>(smem_raw);
    const int lane = threadIdx.x & 63, w = wave_id();
    const int p = blk.x % a.np, r = blk.x / a.np;
    const int nx = a.nx, nxp = a.nxp;
    const int k = p * a.kmul + a.koff;
    const LineCoef<A> *lcp = plane_lines(a.pc, k, a.lc, a.lines_total);
    int total = 0;
    for (int l = a.l0; l < a.nlev; ++l) total += a.ny2[l];
    A *xs = sm, *bs = sm + static_cast<size_t>(total) * nxp;
    // line rows of the levels held here, copied next to the lines: the
    // relaxations then wait on one global load (the Thomas table), not two
    LineCoef<A> *lcs = reinterpret_cast<LineCoef<A> *>(bs + static_cast<size_t>(total) * nxp);
    // line offset of level l inside xs / bs / lcs
    auto off = [&](int l) {
        int o = 0;
        for (int m = a.l0; m < l; ++m) o += a.ny2[m];
        return o;
    };
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
        int l = a.l0, o = 0;
        while (i >= o + a.ny2[l]) o += a.ny2[l++];
        lcs[i] = lcp[a.lev_off[l] + (i - o)];
    }
    {
        const T *bpl = a.b + r * a.brs + p * a.bps;
        for (int j = w; j < a.ny2[a.l0]; j += kW) {
            A v[E];
            gload<T, A, E>(v, bpl + static_cast<long long>(j) * nx, nx, lane);
            sstore<A, E>(bs + j * nxp, v, lane);
        }
    }
    __syncthreads();
    for (int l = a.l0; l < a.nlev - 1; ++l) {
        const int ny = a.ny2[l], nyc = a.ny2[l + 1];
        const LineCoef<A> *lc = lcs + off(l);
        const int ol = off(l), oc = ol + ny;
        A *x = xs + ol * nxp, *b = bs + ol * nxp, *bc = bs + oc * nxp;
        for (int s = 0; s < a.ipre; ++s) {
            lds_relax<A, E>(x, b, lc, a.fac, ny, nxp, 0, s == 0, lane, w);
            __syncthreads();
            lds_relax<A, E>(x, b, lc, a.fac, ny, nxp, 1, false, lane, w);
            __syncthreads();
        }
        if (a.ipre == 0) {
            for (int j = w; j < ny; j += kW)
#pragma unroll
                for (int e = 0; e < E; ++e) x[j * nxp + e * 64 + lane] = A(0);
            __syncthreads();
        }
        for (int J = w; J < nyc; J += kW) {
            A acc[E];
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] = A(0);
            if (a.ipre == 1) {
                // after one sweep from zero the C lines' residuals are zero and
                // an F line's is -V_{j-1} x_{j-1} - V_j x_{j+1}
                for (int d = 0; d < 2; ++d) {
                    const int j = 2 * J + 2 * d;
                    if (j >= ny) break;
                    A f[E], v[E];
#pragma unroll
                    for (int e = 0; e < E; ++e) f[e] = A(0);
                    if (j > 0) {
                        const LineCoef<A> cm = lc[j - 1];
                        sload<A, E>(v, x + (j - 1) * nxp, lane);
                        sub_op<A, E>(f, v, cm.va, cm.vb);
                    }
                    if (j + 1 < ny) {
                        const LineCoef<A> cj = lc[j];
                        sload<A, E>(v, x + (j + 1) * nxp, lane);
                        sub_op<A, E>(f, v, cj.va, cj.vb);
                    }
#pragma unroll
                    for (int e = 0; e < E; ++e) acc[e] += A(0.5) * f[e];
                }
                sstore<A, E>(bc + J * nxp, acc, lane);
                continue;
            }
            for (int d = 0; d < 3; ++d) {
                const int j = 2 * J + d;
                if (j >= ny) break;
                A f[E], v[E];
                sload<A, E>(f, b + j * nxp, lane);
                const LineCoef<A> cj = lc[j];
                sload<A, E>(v, x + j * nxp, lane);
                sub_op<A, E>(f, v, cj.la, cj.lb);
                if (j > 0) {
                    const LineCoef<A> cm = lc[j - 1];
                    sload<A, E>(v, x + (j - 1) * nxp, lane);
                    sub_op<A, E>(f, v, cm.va, cm.vb);
                }
                if (j + 1 < ny) {
                    sload<A, E>(v, x + (j + 1) * nxp, lane);
                    sub_op<A, E>(f, v, cj.va, cj.vb);
                }
                const A wgt = d == 1 ? A(1) : A(0.5);
#pragma unroll
                for (int e = 0; e < E; ++e) acc[e] += wgt * f[e];
            }
            sstore<A, E>(bc + J * nxp, acc, lane);
        }
        __syncthreads();
    }
    {
        const int l = a.nlev - 1, ol = off(l);
        if (w == 0) {
            A f[E];
            sload<A, E>(f, bs + ol * nxp, lane);
            thomas<A, E>(f, a.fac + static_cast<size_t>(lcs[ol].fac) * nxp, lane);
            sstore<A, E>(xs + ol * nxp, f, lane);
        }
        __syncthreads();
    }
    for (int l = a.nlev - 2; l >= a.l0; --l) {
        const int ny = a.ny2[l], nyc = a.ny2[l + 1];
        const LineCoef<A> *lc = lcs + off(l);
        const int ol = off(l), oc = ol + ny;
        A *x = xs + ol * nxp, *b = bs + ol * nxp;
        const A *xc = xs + oc * nxp;
        for (int j = w; j < ny; j += kW) {
            A v[E], c[E];
            sload<A, E>(v, x + j * nxp, lane);
            if (j & 1) {
                sload<A, E>(c, xc + (j >> 1) * nxp, lane);
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] += c[e];
            } else {
                const int Jc = j >> 1;
                if (Jc - 1 >= 0) {
                    sload<A, E>(c, xc + (Jc - 1) * nxp, lane);
#pragma unroll
                    for (int e = 0; e < E; ++e) v[e] += A(0.5) * c[e];
                }
                if (Jc < nyc) {
                    sload<A, E>(c, xc + Jc * nxp, lane);
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
    {
        T *opl = a.out + r * a.ors + p * a.ops;
        for (int j = w; j < a.ny2[a.l0]; j += kW) {
            A v[E];
            sload<A, E>(v, xs + j * nxp, lane);
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

template <typename T, typename A, int E>
__global__ __launch_bounds__(kThreads) void k2_coarse(Coarse2Args<T, A> a)
{
    k2_coarse_body<T, A, E>(a, SMG_BLK_HW);
}

template <typename T, typename A, int E>
__global__ __launch_bounds__(kThreads) void k2_coarse_grp(const GroupEntry *tab, int n)
{
    const Coarse2Args<T, A> *a;
    Blk blk;
    if (!group_entry(tab, n, a, blk)) return;
    k2_coarse_body<T, A, E>(*a, blk);
}

// grouped launch for any E <= 4 (boxes of different widths share one launch)
template <typename T, typename A>
__global__ __launch_bounds__(kThreads) void k2_coarse_grp_e4(const GroupEntry *tab, int n)
{
    const Coarse2Args<T, A> *a;
    Blk blk;
    if (!group_entry(tab, n, a, blk)) return;
    switch (a->nxp / 64) {
    case 1: k2_coarse_body<T, A, 1>(*a, blk); break;
    case 2: k2_coarse_body<T, A, 2>(*a, blk); break;
    case 3: k2_coarse_body<T, A, 3>(*a, blk); break;
    default: k2_coarse_body<T, A, 4>(*a, blk); break;
    }
}

// ---------------------------------------------------------------------------
// Prolongation chains.  For a run [j0, j1) of fine indices the chain needs,
// at every coarser level, the index window [lo, hi] with lo = floor((lo_f-1)/2)
// (clamped at 0) and hi = floor(hi_f/2) (clamped at the level size).  A
// workgroup of 256 threads owns 64 columns (i) and a run of RUN fine lines
// (or planes); it stages every level's window in LDS, evaluates
// v_l = x_l + P v_{l+1} from the coarsest level down, and writes the fine run.
// ---------------------------------------------------------------------------
constexpr int kChainCols = 64;
constexpr int kChainRun = 32;
constexpr int kChainWin = 24;     // window lines per level: RUN/2 + 3 fits at level 1

struct Win {
    int lo, hi;
};

__device__ inline Win coarser(Win f, int nc)
{
    Win c;
    c.lo = f.lo - 1 < 0 ? 0 : (f.lo - 1) >> 1;
    c.hi = f.hi >> 1;
    if (c.hi > nc - 1) c.hi = nc - 1;
    return c;
}

// v (LDS, window wf of level l) = x_l(window wf) + P v_c (window wc of level l+1),
// for the V columns from col of a window whose lines are W values apart
template <typename A, int V, int W>
__device__ inline void prolong_point(A (&s)[V], const A *vc, Win wc, int jj, int nc, int col)
{
#pragma unroll
    for (int e = 0; e < V; ++e) s[e] = A(0);
    if (jj & 1) {
        const A *u = vc + (((jj - 1) >> 1) - wc.lo) * W + col;
#pragma unroll
        for (int e = 0; e < V; ++e) s[e] += u[e];
    } else {
        const int Jc = jj >> 1;
        if (Jc - 1 >= 0) {
            const A *u = vc + (Jc - 1 - wc.lo) * W + col;
#pragma unroll
            for (int e = 0; e < V; ++e) s[e] += A(0.5) * u[e];
        }
        if (Jc < nc) {
            const A *u = vc + (Jc - wc.lo) * W + col;
#pragma unroll
            for (int e = 0; e < V; ++e) s[e] += A(0.5) * u[e];
        }
    }
}

// Window lines (planes) per thread (4 rows of threads) of chain level l for a
// fine run of 32: the windows hold at most 17, 9, 5 and then 3 lines (any
// level sizes), so 5, 3, 2 and then 1 per thread.
constexpr int kChainPre = 8;   // chain levels whose reads are issued up front
__host__ __device__ constexpr int chain_rows(int l) { return l == 1 ? 5 : l == 2 ? 3 : l == 3 ? 2 : 1; }
__host__ __device__ constexpr int chain_off(int l)
{
    int o = 0;
    for (int m = 1; m < l; ++m) o += chain_rows(m);
    return o;
}
static_assert(kChainRun == 32, "chain_rows assumes runs of 32 fine planes");

// V: consecutive columns per thread (a block owns 64 V columns), read and
// written as one aligned access; the launcher takes V > 1 only when every row
// and plane offset is a multiple of V.
template <typename T, typename A, bool ACC, int V>
__device__ __forceinline__ void k2_chain_body(const Chain2Args<T, A> &a, const Blk &blk)
{
    constexpr int W = kChainCols * V;
    __shared__ A vs[2][kChainWin * W];
    constexpr int kRows0 = kChainRun / 4;       // fine lines per thread
    const int nx = a.nx;
    const int ncol = (nx + W - 1) / W;
    const int nrun = (a.ny2[0] + kChainRun - 1) / kChainRun;
    int bid = blk.x;
    const int ct = bid % ncol;
    bid /= ncol;
    const int rt = bid % nrun;
    bid /= nrun;
    const int p = bid % a.np, r = bid / a.np;
    const int col = (threadIdx.x & (kChainCols - 1)) * V, row0 = threadIdx.x >> 6;   // 4 rows of 64 lanes
    const int i = ct * W + col;
    const int nok = i < nx ? min(V, nx - i) : 0;   // columns of this thread inside the row
    const Win w0{rt * kChainRun, min(a.ny2[0], rt * kChainRun + kChainRun) - 1};
    // windows of every level (uniform; recomputed from the fine run)
    auto win = [&](int l) {
        Win wv = w0;
        for (int m = 0; m < l; ++m) wv = coarser(wv, a.ny2[m + 1]);
        return wv;
    };
    auto level_row = [&](int l, const Win &wl, int jj, A (&v)[V]) {
        const T *xl = a.xc[l] + r * a.crs[l] + p * a.cps[l];
        vld<T, A, V>(v, xl + static_cast<long long>(jj) * nx + i, jj <= wl.hi ? nok : 0);
    };
    // every global read of chain levels 1..kChainPre and of the fine run
    // (x and the accumulated output), issued before the first barrier and
    // held as stored until used
    Held<T, V> pre[chain_off(kChainPre + 1)];
#pragma unroll
    for (int l = 1; l <= kChainPre; ++l) {
        if (l > a.lc) break;
        const Win wl = win(l);
        const T *xl = a.xc[l] + r * a.crs[l] + p * a.cps[l];
#pragma unroll
        for (int t = 0; t < chain_rows(l); ++t) {
            const int jj = wl.lo + row0 + 4 * t;
            hld<T, V>(pre[chain_off(l) + t], xl + static_cast<long long>(jj) * nx + i, jj <= wl.hi ? nok : 0);
        }
    }
    const T *x0 = a.x0 + r * a.x0rs + p * a.x0ps;
    T *out = a.out + r * a.ors + p * a.ops;
    Held<T, V> xf[kRows0], of[kRows0];
#pragma unroll
    for (int t = 0; t < kRows0; ++t) {
        const int jj = w0.lo + row0 + 4 * t;
        const long long o = static_cast<long long>(jj) * nx + i;
        const int n = jj <= w0.hi ? nok : 0;
        hld<T, V>(xf[t], x0 + o, n);
        if constexpr (ACC) hld<T, V>(of[t], out + o, n);
    }
    int cur = 0;
    bool first = true;   // the coarsest level is stored as it is
    auto step = [&](int l, int nrows, auto &&xval) {
        const Win wl = win(l);
        if (first) {
            for (int t = 0; t < nrows; ++t) {
                const int jj = wl.lo + row0 + 4 * t;
                if (jj <= wl.hi) {
                    A v[V];
                    xval(t, jj, wl, v);
#pragma unroll
                    for (int e = 0; e < V; ++e) vs[cur][(jj - wl.lo) * W + col + e] = v[e];
                }
            }
            first = false;
        } else {
            const Win wc = win(l + 1);
            for (int t = 0; t < nrows; ++t) {
                const int jj = wl.lo + row0 + 4 * t;
                if (jj > wl.hi) break;
                A v[V], pv[V];
                xval(t, jj, wl, v);
                prolong_point<A, V, W>(pv, vs[cur], wc, jj, a.ny2[l + 1], col);
#pragma unroll
                for (int e = 0; e < V; ++e) vs[cur ^ 1][(jj - wl.lo) * W + col + e] = v[e] + pv[e];
            }
            cur ^= 1;
        }
        __syncthreads();
    };
    for (int l = a.lc; l > kChainPre; --l)
        step(l, kChainWin / 4, [&](int, int jj, const Win &wl, A (&v)[V]) { level_row(l, wl, jj, v); });
#pragma unroll
    for (int l = kChainPre; l >= 1; --l) {
        if (l > a.lc) continue;
        step(l, chain_rows(l), [&](int t, int, const Win &, A (&v)[V]) { unpack<T, A, V>(v, pre[chain_off(l) + t]); });
    }
    if (nok == 0) return;   // after the last barrier
    const Win wc = win(1);
#pragma unroll
    for (int t = 0; t < kRows0; ++t) {
        const int jj = w0.lo + row0 + 4 * t;
        if (jj > w0.hi) break;
        A pv[V], v[V], o[V];
        prolong_point<A, V, W>(pv, vs[cur], wc, jj, a.ny2[1], col);
        unpack<T, A, V>(v, xf[t]);
        if constexpr (ACC) unpack<T, A, V>(o, of[t]);
#pragma unroll
        for (int e = 0; e < V; ++e) {
            v[e] = v[e] + pv[e];
            if constexpr (ACC) v[e] += o[e];
        }
        vst<T, A, V>(out + static_cast<long long>(jj) * nx + i, v, nok);
    }
}

// ACC: the output is accumulated into (read back) rather than assigned; the
// assigning kernel keeps no registers for the read-back
template <typename T, typename A, bool ACC, int V>
__global__ __launch_bounds__(256) void k2_chain(Chain2Args<T, A> a)
{
    k2_chain_body<T, A, ACC, V>(a, SMG_BLK_XCD);
}

template <typename T, typename A, bool ACC, int V>
__global__ __launch_bounds__(256) void k2_chain_grp(const GroupEntry *tab, int n)
{
    const Chain2Args<T, A> *a;
    Blk blk;
    if (!group_entry(tab, n, a, blk)) return;
    k2_chain_body<T, A, ACC, V>(*a, blk);
}


// V: consecutive in-plane points per thread, as in the 2D chain
template <typename T, typename A, int V>
__device__ __forceinline__ void k3_chain_body(const Chain3Args<T, A> &a, const Blk &blk)
{
    constexpr int W = kChainCols * V;
    __shared__ A vs[2][kChainWin * W];
    constexpr int kRows0 = kChainRun / 4;       // fine planes per thread
    const long long pl = static_cast<long long>(a.nx) * a.ny;
    const int ncol = static_cast<int>((pl + W - 1) / W);
    const int ct = blk.x % ncol;
    const int rt = blk.x / ncol;
    const int r = blk.y;
    const int col = (threadIdx.x & (kChainCols - 1)) * V, row0 = threadIdx.x >> 6;
    const long long c = static_cast<long long>(ct) * W + col;
    const int nok = c < pl ? static_cast<int>(pl - c < V ? pl - c : V) : 0;
    const Win w0{rt * kChainRun, min(a.nz[0], rt * kChainRun + kChainRun) - 1};
    auto win = [&](int l) {
        Win wv = w0;
        for (int m = 0; m < l; ++m) wv = coarser(wv, a.nz[m + 1]);
        return wv;
    };
    auto level_row = [&](int l, const Win &wl, int kk, A (&v)[V]) {
        const T *xl = a.x[l] + r * a.rs[l];
        vld<T, A, V>(v, xl + kk * pl + c, kk <= wl.hi ? nok : 0);
    };
    // every global read of chain levels 1..kChainPre and of the fine run,
    // issued before the first barrier and held as stored until used
    Held<T, V> pre[chain_off(kChainPre + 1)];
#pragma unroll
    for (int l = 1; l <= kChainPre; ++l) {
        if (l > a.L) break;
        const Win wl = win(l);
        const T *xl = a.x[l] + r * a.rs[l];
#pragma unroll
        for (int t = 0; t < chain_rows(l); ++t) {
            const int kk = wl.lo + row0 + 4 * t;
            hld<T, V>(pre[chain_off(l) + t], xl + kk * pl + c, kk <= wl.hi ? nok : 0);
        }
    }
    T *x0 = a.x[0] + r * a.rs[0];
    Held<T, V> xf[kRows0];
#pragma unroll
    for (int t = 0; t < kRows0; ++t) {
        const int kk = w0.lo + row0 + 4 * t;
        hld<T, V>(xf[t], x0 + kk * pl + c, kk <= w0.hi ? nok : 0);
    }
    int cur = 0;
    bool first = true;   // the coarsest level is stored as it is
    auto step = [&](int l, int nrows, auto &&xval) {
        const Win wl = win(l);
        if (first) {
            for (int t = 0; t < nrows; ++t) {
                const int kk = wl.lo + row0 + 4 * t;
                if (kk <= wl.hi) {
                    A v[V];
                    xval(t, kk, wl, v);
#pragma unroll
                    for (int e = 0; e < V; ++e) vs[cur][(kk - wl.lo) * W + col + e] = v[e];
                }
            }
            first = false;
        } else {
            const Win wc = win(l + 1);
            for (int t = 0; t < nrows; ++t) {
                const int kk = wl.lo + row0 + 4 * t;
                if (kk > wl.hi) break;
                A v[V], pv[V];
                xval(t, kk, wl, v);
                prolong_point<A, V, W>(pv, vs[cur], wc, kk, a.nz[l + 1], col);
#pragma unroll
                for (int e = 0; e < V; ++e) vs[cur ^ 1][(kk - wl.lo) * W + col + e] = v[e] + pv[e];
            }
            cur ^= 1;
        }
        __syncthreads();
    };
    for (int l = a.L; l > kChainPre; --l)
        step(l, kChainWin / 4, [&](int, int kk, const Win &wl, A (&v)[V]) { level_row(l, wl, kk, v); });
#pragma unroll
    for (int l = kChainPre; l >= 1; --l) {
        if (l > a.L) continue;
        step(l, chain_rows(l), [&](int t, int, const Win &, A (&v)[V]) { unpack<T, A, V>(v, pre[chain_off(l) + t]); });
    }
    constexpr bool kDots = std::is_same<T, double>::value;
    const bool dots = kDots && a.dpart != nullptr;
    double sr = 0.0, sq = 0.0;
    if (nok > 0) {
        const Win wc = win(1);
#pragma unroll
        for (int t = 0; t < kRows0; ++t) {
            const int kk = w0.lo + row0 + 4 * t;
            if (kk > w0.hi) break;
            A pv[V], v[V];
            prolong_point<A, V, W>(pv, vs[cur], wc, kk, a.nz[1], col);
            unpack<T, A, V>(v, xf[t]);
#pragma unroll
            for (int e = 0; e < V; ++e) v[e] = v[e] + pv[e];
            vst<T, A, V>(x0 + kk * pl + c, v, nok);
            if constexpr (kDots) {
                if (dots) {
                    for (int e = 0; e < nok; ++e) {
                        const long long g = kk * pl + c + e;
                        sr = fmadd(v[e], a.dr[g], sr);
                        if (a.want_sq) sq = fmadd(v[e], a.dq[g], sq);
                    }
                }
            }
        }
    }
    if constexpr (kDots) {
        // one partial per block: wave sums, then the four waves in order
        if (!dots) return;
        __shared__ double red[2][4];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            sr += __shfl_down(sr, off, 64);
            sq += __shfl_down(sq, off, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            red[0][threadIdx.x >> 6] = sr;
            red[1][threadIdx.x >> 6] = sq;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            a.dpart[blk.x] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
            a.dpart[blk.gx + blk.x] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
        }
    }
}

template <typename T, typename A, int V>
__global__ __launch_bounds__(256) void k3_chain(Chain3Args<T, A> a)
{
    k3_chain_body<T, A, V>(a, SMG_BLK_HW);
}

template <typename T, typename A, int V>
__global__ __launch_bounds__(256) void k3_chain_grp(const GroupEntry *tab, int n)
{
    const Chain3Args<T, A> *a;
    Blk blk;
    if (!group_entry(tab, n, a, blk)) return;
    k3_chain_body<T, A, V>(*a, blk);
}

// ---------------------------------------------------------------------------
// k2_up: prolongation and one post-smoothing sweep (C then F) of a strip of
// fine lines [j0, j0 + 2S).  LDS slot s holds fine line j0 - 2 + s.
// x_pre: this level after pre-smoothing; xc: the coarser level's result;
// out: this level's result (a different buffer), assigned or accumulated.
// ---------------------------------------------------------------------------
template <typename T, typename A, int E>
__device__ __forceinline__ void k2_up_body(const Up2Args<T, A> &a, const Blk &blk)
{
    extern __shared__ unsigned char smem_raw[];
    A *xs = reinterpret_cast<A *>(smem_raw);
    const int lane = threadIdx.x & 63, w = wave_id();
    const int ny = a.ny, nyc = a.nyc, nx = a.nx, nxp = a.nxp;
    const int nstrip = (ny + 2 * a.S - 1) / (2 * a.S);
    const int strip = blk.x % nstrip;
    const int p = (blk.x / nstrip) % a.np;
    const int r = blk.x / (nstrip * a.np);
    const int j0 = strip * 2 * a.S, j1 = min(j0 + 2 * a.S, ny);
    const int base = j0 - 2;
    const int jlo = max(0, j0 - 2), jhi = min(ny - 1, j1 + 1);
    const int k = p * a.kmul + a.koff;
    const LineCoef<A> *lc = plane_lines(a.pc, k, a.lc, a.lines_total);
    const T *xp = a.xpre + r * a.xrs + p * a.xps;
    const T *cp = a.xc + r * a.crs + p * a.cps;
    const T *bp = a.b + r * a.brs + p * a.bps;
    for (int j = jlo + w; j <= jhi; j += kW) {
        A v[E], c[E];
        gload<T, A, E>(v, xp + static_cast<long long>(j) * nx, nx, lane);
        if (j & 1) {
            gload<T, A, E>(c, cp + static_cast<long long>(j >> 1) * nx, nx, lane);
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] += c[e];
        } else {
            const int Jc = j >> 1;
            if (Jc - 1 >= 0) {
                gload<T, A, E>(c, cp + static_cast<long long>(Jc - 1) * nx, nx, lane);
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] += A(0.5) * c[e];
            }
            if (Jc < nyc) {
                gload<T, A, E>(c, cp + static_cast<long long>(Jc) * nx, nx, lane);
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] += A(0.5) * c[e];
            }
        }
        sstore<A, E>(xs + (j - base) * nxp, v, lane);
    }
    __syncthreads();
    for (int colour = 1; colour >= 0; --colour) {
        const int lo = colour == 1 ? max(1, (j0 - 1) | 1) : j0 + (j0 & 1);
        const int hi = colour == 1 ? min(ny - 1, j1) : j1 - 1;
        const int n = lo <= hi ? (hi - lo) / 2 + 1 : 0;
        for (int t = w; t < n; t += kW) {
            const int j = lo + 2 * t;
            A f[E], v[E];
            gload<T, A, E>(f, bp + static_cast<long long>(j) * nx, nx, lane);
            if (j > 0) {
                const LineCoef<A> cm = lc[j - 1];
                sload<A, E>(v, xs + (j - 1 - base) * nxp, lane);
                sub_op<A, E>(f, v, cm.va, cm.vb);
            }
            if (j + 1 < ny) {
                const LineCoef<A> cj = lc[j];
                sload<A, E>(v, xs + (j + 1 - base) * nxp, lane);
                sub_op<A, E>(f, v, cj.va, cj.vb);
            }
            thomas<A, E>(f, a.fac + static_cast<size_t>(lc[j].fac) * nxp, lane);
            sstore<A, E>(xs + (j - base) * nxp, f, lane);
        }
        __syncthreads();
    }
    T *op = a.out + r * a.ors + p * a.ops;
    for (int j = j0 + w; j < j1; j += kW) {
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

template <typename T, typename A, int E>
__global__ __launch_bounds__(kThreads) void k2_up(Up2Args<T, A> a)
{
    k2_up_body<T, A, E>(a, SMG_BLK_HW);
}

template <typename T, typename A, int E>
__global__ __launch_bounds__(kThreads) void k2_up_grp(const GroupEntry *tab, int n)
{
    const Up2Args<T, A> *a;
    Blk blk;
    if (!group_entry(tab, n, a, blk)) return;
    k2_up_body<T, A, E>(*a, blk);
}

// grouped launch for any E <= 4 (boxes of different widths share one launch)
template <typename T, typename A>
__global__ __launch_bounds__(kThreads) void k2_up_grp_e4(const GroupEntry *tab, int n)
{
    const Up2Args<T, A> *a;
    Blk blk;
    if (!group_entry(tab, n, a, blk)) return;
    switch (a->nxp / 64) {
    case 1: k2_up_body<T, A, 1>(*a, blk); break;
    case 2: k2_up_body<T, A, 2>(*a, blk); break;
    case 3: k2_up_body<T, A, 3>(*a, blk); break;
    default: k2_up_body<T, A, 4>(*a, blk); break;
    }
}

// grouped twin for width E: the any-E kernel up to E = 4, else the E-specific one
template <int E, typename K4, typename KE>
inline const void *grouped_e4(K4 k4, KE ke)
{
    return E <= 4 ? reinterpret_cast<const void *>(k4) : reinterpret_cast<const void *>(ke);
}

template <typename K>
inline void allow_lds(K kernel, size_t bytes)
{
    if (bytes > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  static_cast<int>(bytes));
}

}  // namespace

#define SMG_E_SWITCH(E, CALL)                      \
    switch (E) {                                   \
    case 1: { constexpr int EE = 1; CALL; } break; \
    case 2: { constexpr int EE = 2; CALL; } break; \
    case 3: { constexpr int EE = 3; CALL; } break; \
    case 4: { constexpr int EE = 4; CALL; } break; \
    case 5: { constexpr int EE = 5; CALL; } break; \
    case 6: { constexpr int EE = 6; CALL; } break; \
    case 7: { constexpr int EE = 7; CALL; } break; \
    case 8: { constexpr int EE = 8; CALL; } break; \
    default: break;                                \
    }

int fused_waves() { return kW; }

template <typename T, typename A>
void launch_down2(const Down2Args<T, A> &a, hipStream_t st, const LaunchEv &ev)
{
    const int E = a.nxp / 64;
    if (E <= 4) {   // register-only variants: one wave per coarse line, or per run of them
        const long long waves = static_cast<long long>(a.nyc) * a.np * a.nrhs;
        if (waves == 0) return;
        int kr = 1;
        if (a.march_waves > 0)
            for (const int c : {8, 4, 2})
                if (waves / c >= a.march_waves) {
                    kr = c;
                    break;
                }
        if (kr > 1) {
            Down2Args<T, A> m = a;
            m.kr = kr;
            const long long mw = static_cast<long long>((a.nyc + kr - 1) / kr) * a.np * a.nrhs;
            const dim3 mgrid(static_cast<unsigned>((mw + 3) / 4));
            switch (E) {
            case 1: SMG_LAUNCH_G(ev, (k2_down_march<T, A, 1>), (k2_down_march_grp_e4<T, A>), mgrid, dim3(256), 0, st, m); break;
            case 2: SMG_LAUNCH_G(ev, (k2_down_march<T, A, 2>), (k2_down_march_grp_e4<T, A>), mgrid, dim3(256), 0, st, m); break;
            case 3: SMG_LAUNCH_G(ev, (k2_down_march<T, A, 3>), (k2_down_march_grp_e4<T, A>), mgrid, dim3(256), 0, st, m); break;
            default: SMG_LAUNCH_G(ev, (k2_down_march<T, A, 4>), (k2_down_march_grp_e4<T, A>), mgrid, dim3(256), 0, st, m); break;
            }
            return;
        }
        const dim3 grid(static_cast<unsigned>((waves + 3) / 4));
        switch (E) {
        case 1: SMG_LAUNCH_G(ev, (k2_down_reg<T, A, 1>), (k2_down_reg_grp_e4<T, A>), grid, dim3(256), 0, st, a); break;
        case 2: SMG_LAUNCH_G(ev, (k2_down_reg<T, A, 2>), (k2_down_reg_grp_e4<T, A>), grid, dim3(256), 0, st, a); break;
        case 3: SMG_LAUNCH_G(ev, (k2_down_reg<T, A, 3>), (k2_down_reg_grp_e4<T, A>), grid, dim3(256), 0, st, a); break;
        default: SMG_LAUNCH_G(ev, (k2_down_reg<T, A, 4>), (k2_down_reg_grp_e4<T, A>), grid, dim3(256), 0, st, a); break;
        }
        return;
    }
    const int nstrip = (a.nyc + a.S - 1) / a.S;
    const long long nblk = static_cast<long long>(nstrip) * a.np * a.nrhs;
    if (nblk == 0) return;
    const size_t lds = static_cast<size_t>(2 * a.S + 5) * a.nxp * sizeof(A);
    SMG_E_SWITCH(a.nxp / 64, allow_lds(k2_down<T, A, EE>, lds); allow_lds(k2_down_grp<T, A, EE>, lds);
                 allow_lds(k2_down_grp_e4<T, A>, lds);
                 SMG_LAUNCH_G(ev, (k2_down<T, A, EE>), (grouped_e4<EE>(k2_down_grp_e4<T, A>, k2_down_grp<T, A, EE>)),
                              dim3(static_cast<unsigned>(nblk)), dim3(kThreads), lds, st, a));
}

template <typename T, typename A>
void launch_coarse2(const Coarse2Args<T, A> &a, size_t lds_bytes, hipStream_t st, const LaunchEv &ev)
{
    const long long nblk = static_cast<long long>(a.np) * a.nrhs;
    if (nblk == 0) return;
    SMG_E_SWITCH(a.nxp / 64, allow_lds(k2_coarse<T, A, EE>, lds_bytes); allow_lds(k2_coarse_grp<T, A, EE>, lds_bytes);
                 allow_lds(k2_coarse_grp_e4<T, A>, lds_bytes);
                 SMG_LAUNCH_G(ev, (k2_coarse<T, A, EE>),
                              (grouped_e4<EE>(k2_coarse_grp_e4<T, A>, k2_coarse_grp<T, A, EE>)),
                              dim3(static_cast<unsigned>(nblk)), dim3(kThreads), lds_bytes, st, a));
}

// Points per thread of the 2D chain: tile_vec's width when every row, plane
// and right-hand-side offset is a multiple of it.
template <typename T, typename A>
int chain2_vec(const Chain2Args<T, A> &a)
{
    const int V = a.vmax == 1 ? 1 : tile_vec<T>(a.nx);
    if (V == 1) return 1;
    auto ok = [&](long long v) { return v % V == 0; };
    auto aligned = [&](const void *q) { return reinterpret_cast<uintptr_t>(q) % (V * sizeof(T)) == 0; };
    if (!ok(a.x0ps) || !ok(a.x0rs) || !ok(a.ops) || !ok(a.ors) || !aligned(a.x0) || !aligned(a.out)) return 1;
    for (int l = 1; l <= a.lc; ++l)
        if (!ok(a.cps[l]) || !ok(a.crs[l]) || !aligned(a.xc[l])) return 1;
    return V;
}

template <typename T, typename A, int V>
void launch_chain2_v(const Chain2Args<T, A> &a, hipStream_t st, const LaunchEv &ev)
{
    const long long ncol = (a.nx + kChainCols * V - 1) / (kChainCols * V);
    const long long nrun = (a.ny2[0] + kChainRun - 1) / kChainRun;
    const long long nblk = ncol * nrun * a.np * a.nrhs;
    if (nblk == 0) return;
    if (a.accumulate)
        SMG_LAUNCH_G(ev, (k2_chain<T, A, true, V>), (k2_chain_grp<T, A, true, V>), dim3(static_cast<unsigned>(nblk)),
                     dim3(256), 0, st, a);
    else
        SMG_LAUNCH_G(ev, (k2_chain<T, A, false, V>), (k2_chain_grp<T, A, false, V>),
                     dim3(static_cast<unsigned>(nblk)), dim3(256), 0, st, a);
}

template <typename T, typename A>
void launch_chain2(const Chain2Args<T, A> &a, hipStream_t st, const LaunchEv &ev)
{
    const int v = chain2_vec(a);
    if (v == 4) {
        if constexpr (stream_vec<T>() >= 4) launch_chain2_v<T, A, 4>(a, st, ev);
    } else if (v == 2) {
        if constexpr (stream_vec<T>() >= 2) launch_chain2_v<T, A, 2>(a, st, ev);
    } else {
        launch_chain2_v<T, A, 1>(a, st, ev);
    }
}

template <typename T, typename A>
void launch_up2(const Up2Args<T, A> &a, hipStream_t st, const LaunchEv &ev)
{
    const int nstrip = (a.ny + 2 * a.S - 1) / (2 * a.S);
    const long long nblk = static_cast<long long>(nstrip) * a.np * a.nrhs;
    if (nblk == 0) return;
    const size_t lds = static_cast<size_t>(2 * a.S + 4) * a.nxp * sizeof(A);
    SMG_E_SWITCH(a.nxp / 64, allow_lds(k2_up<T, A, EE>, lds); allow_lds(k2_up_grp<T, A, EE>, lds);
                 allow_lds(k2_up_grp_e4<T, A>, lds);
                 SMG_LAUNCH_G(ev, (k2_up<T, A, EE>), (grouped_e4<EE>(k2_up_grp_e4<T, A>, k2_up_grp<T, A, EE>)),
                              dim3(static_cast<unsigned>(nblk)), dim3(kThreads), lds, st, a));
}

template <typename T, typename A, int V>
void launch_chain3_v(const Chain3Args<T, A> &a, int nrhs, hipStream_t st, const LaunchEv &ev)
{
    const long long pl = static_cast<long long>(a.nx) * a.ny;
    const long long ncol = (pl + kChainCols * V - 1) / (kChainCols * V);
    const long long nrun = (a.nz[0] + kChainRun - 1) / kChainRun;
    SMG_LAUNCH_G(ev, (k3_chain<T, A, V>), (k3_chain_grp<T, A, V>), dim3(static_cast<unsigned>(ncol * nrun), nrhs),
                 dim3(256), 0, st, a);
}

long long chain3_blocks(int nx, int ny, int nz)
{
    const long long pl = static_cast<long long>(nx) * ny;
    return ((pl + kChainCols - 1) / kChainCols) * ((nz + kChainRun - 1) / kChainRun);
}

template <typename T, typename A>
void launch_chain3(const Chain3Args<T, A> &a, int nrhs, hipStream_t st, const LaunchEv &ev)
{
    constexpr int V = stream_vec<T>();
    bool vec = V > 1 && a.vmax != 1 && (static_cast<long long>(a.nx) * a.ny) % V == 0;
    for (int l = 0; l <= a.L && vec; ++l)
        vec = a.rs[l] % V == 0 && reinterpret_cast<uintptr_t>(a.x[l]) % (V * sizeof(T)) == 0;
    if (vec)
        launch_chain3_v<T, A, V>(a, nrhs, st, ev);
    else
        launch_chain3_v<T, A, 1>(a, nrhs, st, ev);
}

#define SMG_FUSED_INSTANTIATE(T, A)                                                                      \
    template void launch_down2<T, A>(const Down2Args<T, A> &, hipStream_t, const LaunchEv &);             \
    template void launch_coarse2<T, A>(const Coarse2Args<T, A> &, size_t, hipStream_t, const LaunchEv &); \
    template void launch_chain2<T, A>(const Chain2Args<T, A> &, hipStream_t, const LaunchEv &);           \
    template void launch_up2<T, A>(const Up2Args<T, A> &, hipStream_t, const LaunchEv &);                 \
    template void launch_chain3<T, A>(const Chain3Args<T, A> &, int, hipStream_t, const LaunchEv &);

SMG_FUSED_INSTANTIATE(double, double)
SMG_FUSED_INSTANTIATE(float, float)
SMG_FUSED_INSTANTIATE(bf16, float)

}  // namespace smg
