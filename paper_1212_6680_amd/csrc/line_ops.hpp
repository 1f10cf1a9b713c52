// Wave-level operations on one x-line held in the registers of a wave64:
// lane l owns points [l*E, l*E + E) (points >= nx are zero).
//
// The exact line solve evaluates the two first-order recurrences of the
// Thomas algorithm, y_i = g_i f_i + h_i y_{i-1} and u_i = y_i + h_i u_{i+1},
// as scans of affine maps x -> a x + b across the 64 lanes.  Within each
// 16-lane row the scan uses DPP row shifts (1, 2, 4, 8); the three row
// aggregates are read as uniform values with readlane and folded in, and the
// carry into each lane comes from a whole-wave DPP shift.  Everything stays in
// VGPRs: no LDS, no ds_bpermute.
#pragma once

#include "smg_internal.h"

namespace smg {
namespace lineops {

// DPP control codes (GFX9 encoding)
constexpr int kRowShl = 0x100;   // + n, n = 1..15: lane reads lane+n of its row
constexpr int kRowShr = 0x110;   // + n: lane reads lane-n of its row
constexpr int kWaveShl1 = 0x130; // lane reads lane+1 of the wave
constexpr int kWaveShr1 = 0x138; // lane reads lane-1 of the wave

// v from the DPP source lane, or `old` where the source is outside the row/wave
template <int CTRL>
__device__ inline float dpp(float old, float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ inline double dpp(double old, double v)
{
    const long long o = __double_as_longlong(old), s = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(static_cast<int>(o), static_cast<int>(s), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(static_cast<int>(o >> 32), static_cast<int>(s >> 32), CTRL, 0xf, 0xf,
                                               false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

__device__ inline float readlane(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }

__device__ inline double readlane(double v, int l)
{
    const long long s = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(s), l);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(s >> 32), l);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// (a, b) <- (a, b) o (pa, pb): first apply (pa, pb), then (a, b)
template <typename A>
__device__ inline void compose(A &a, A &b, A pa, A pb)
{
    b = a * pb + b;
    a = a * pa;
}

// Inclusive scan of lane maps in increasing lane order; on return b holds
// the composed map of lanes 0..l applied to 0.
template <typename A>
__device__ inline void scan_up(A &a, A &b, int lane)
{
    compose(a, b, dpp<kRowShr + 1>(A(1), a), dpp<kRowShr + 1>(A(0), b));
    compose(a, b, dpp<kRowShr + 2>(A(1), a), dpp<kRowShr + 2>(A(0), b));
    compose(a, b, dpp<kRowShr + 4>(A(1), a), dpp<kRowShr + 4>(A(0), b));
    compose(a, b, dpp<kRowShr + 8>(A(1), a), dpp<kRowShr + 8>(A(0), b));
    // row aggregates (uniform) and their prefixes
    const A a0 = readlane(a, 15), b0 = readlane(b, 15);
    const A a1 = readlane(a, 31), b1 = readlane(b, 31);
    const A a2 = readlane(a, 47), b2 = readlane(b, 47);
    A p1a = a0, p1b = b0;             // rows < 1
    A p2a = a1, p2b = b1;
    compose(p2a, p2b, p1a, p1b);      // rows < 2
    A p3a = a2, p3b = b2;
    compose(p3a, p3b, p2a, p2b);      // rows < 3
    const int row = lane >> 4;
    const A pa = row == 0 ? A(1) : row == 1 ? p1a : row == 2 ? p2a : p3a;
    const A pb = row == 0 ? A(0) : row == 1 ? p1b : row == 2 ? p2b : p3b;
    compose(a, b, pa, pb);
}

// Inclusive scan in decreasing lane order (lanes l..63).
template <typename A>
__device__ inline void scan_down(A &a, A &b, int lane)
{
    compose(a, b, dpp<kRowShl + 1>(A(1), a), dpp<kRowShl + 1>(A(0), b));
    compose(a, b, dpp<kRowShl + 2>(A(1), a), dpp<kRowShl + 2>(A(0), b));
    compose(a, b, dpp<kRowShl + 4>(A(1), a), dpp<kRowShl + 4>(A(0), b));
    compose(a, b, dpp<kRowShl + 8>(A(1), a), dpp<kRowShl + 8>(A(0), b));
    const A a3 = readlane(a, 48), b3 = readlane(b, 48);
    const A a2 = readlane(a, 32), b2 = readlane(b, 32);
    const A a1 = readlane(a, 16), b1 = readlane(b, 16);
    A q2a = a3, q2b = b3;             // rows > 2
    A q1a = a2, q1b = b2;
    compose(q1a, q1b, q2a, q2b);      // rows > 1
    A q0a = a1, q0b = b1;
    compose(q0a, q0b, q1a, q1b);      // rows > 0
    const int row = lane >> 4;
    const A qa = row == 3 ? A(1) : row == 2 ? q2a : row == 1 ? q1a : q0a;
    const A qb = row == 3 ? A(0) : row == 2 ? q2b : row == 1 ? q1b : q0b;
    compose(a, b, qa, qb);
}

// This lane's part of a Thomas table (g_i, h_i).
template <typename A, int E>
__device__ inline void load_fac(A (&g)[E], A (&h)[E], const Fac<A> *fac, int lane)
{
    const int i0 = lane * E;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const Fac<A> fe = fac[i0 + e];
        g[e] = fe.g;
        h[e] = fe.h;
    }
}

// Exact solve of one line in place with a Thomas table held in registers.
template <typename A, int E>
__device__ inline void thomas_gh(A (&f)[E], const A (&g)[E], const A (&h)[E], int lane)
{
    A pr[E];
    A acc = A(0), prod = A(1);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        acc = g[e] * f[e] + h[e] * acc;
        prod *= h[e];
        f[e] = acc;
        pr[e] = prod;
    }
    A sa = pr[E - 1], sb = f[E - 1];
    scan_up(sa, sb, lane);
    const A carry_in = dpp<kWaveShr1>(A(0), sb);   // y at the last point of lane l-1
#pragma unroll
    for (int e = 0; e < E; ++e) f[e] += pr[e] * carry_in;
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
    scan_down(sa, sb, lane);
    const A carry_up = dpp<kWaveShl1>(A(0), sb);   // u at the first point of lane l+1
#pragma unroll
    for (int e = 0; e < E; ++e) f[e] += pr[e] * carry_up;
}

// Exact solve of one line in place with the Thomas table fac (g_i, h_i).
template <typename A, int E>
__device__ inline void thomas(A (&f)[E], const Fac<A> *fac, int lane)
{
    A g[E], h[E];
    load_fac<A, E>(g, h, fac, lane);
    thomas_gh<A, E>(f, g, h, lane);
}

// f -= (a*Tx + b*I) w   (w zero beyond nx)
template <typename A, int E>
__device__ inline void sub_op(A (&f)[E], const A (&w)[E], A a, A b)
{
    if (a != A(0)) {
        const A left = dpp<kWaveShr1>(A(0), w[E - 1]);
        const A right = dpp<kWaveShl1>(A(0), w[0]);
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

// LDS lines are lane-interleaved: point e of lane l at [e*64 + l]
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

}  // namespace lineops
}  // namespace smg
