// Wave-level operations on one x-line held in the registers of a wave64:
// lane l owns points [l*E, l*E + E) (points >= nx are zero).
//
// The exact line solve evaluates the two first-order recurrences of the
// Thomas algorithm, y_i = g_i f_i + h_i y_{i-1} and u_i = y_i + h_i u_{i+1},
// as scans of affine maps x -> a x + b across the 64 lanes.  Within each
// 16-lane row the scan uses DPP row shifts (1, 2, 4, 8); across rows the
// forward scan uses DPP row broadcasts and the backward scan reads the row
// aggregates as uniform values with readlane; the carry into each lane comes
// from a whole-wave DPP shift.  Everything stays in VGPRs: no LDS, no
// ds_bpermute.
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

// DPP move with bound_ctrl: lanes whose source lies outside the row (or the
// wave) read 0, so no old value has to be set up.
template <int CTRL>
__device__ inline float dpp0(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}

template <int CTRL>
__device__ inline double dpp0(double v)
{
    const long long s = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(s), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(s >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Row broadcast (lane 15 or 31 of the wave into later rows) written only to
// the rows in ROWS; the other rows read 0.
constexpr int kRowBcast15 = 0x142;
constexpr int kRowBcast31 = 0x143;

template <int CTRL, int ROWS>
__device__ inline float dpp_rows(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, false));
}

template <int CTRL, int ROWS>
__device__ inline double dpp_rows(double v)
{
    const long long s = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(s), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(s >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// The exact line solve evaluates y_i = g_i f_i + h_i y_{i-1} (forward) and
// u_i = y_i + h_i u_{i+1} (backward).  Over a lane's E points each recurrence
// is an affine map x -> A_l x + B_l, where A_l (a product of h) depends on the
// table only and B_l on the data.  The lane scans combine the maps with
// B_l += M * B_{source}, where the multipliers M are products of A over
// lane ranges: a LinePlan holds them, built once per table, so that every
// solve with the table scans B alone (one DPP move and one FMA per step).
template <typename A, int E>
struct LinePlan {
    A g[E], h[E];
    A fm[4];          // forward row steps 1, 2, 4, 8: A over the lanes (l - s, l]
    A f15, f31;       // forward row broadcasts: A from the row start (and earlier rows) to l
    A bm[4];          // backward row steps: A over the lanes [l, l + s)
    A bq;             // backward: A from l to the end of its row
    A s16, s32;       // backward, uniform: A over all of row 1 and row 2
};

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

// Plan of the Thomas table fac: the products of h the lane scans multiply by.
template <typename A, int E>
__device__ inline void plan_products(LinePlan<A, E> &P, int lane);

template <typename A, int E>
__device__ inline void make_plan(LinePlan<A, E> &P, const Fac<A> *fac, int lane)
{
    load_fac<A, E>(P.g, P.h, fac, lane);
    plan_products<A, E>(P, lane);
}

// The scan multipliers of a plan whose rows P.g, P.h are in place.
template <typename A, int E>
__device__ inline void plan_products(LinePlan<A, E> &P, int lane)
{
    A a0 = A(1);
#pragma unroll
    for (int e = 0; e < E; ++e) a0 *= P.h[e];
    // forward: lanes without a source compose with the identity (A = 1)
    A a = a0;
    P.fm[0] = a;
    a *= dpp<kRowShr + 1>(A(1), a);
    P.fm[1] = a;
    a *= dpp<kRowShr + 2>(A(1), a);
    P.fm[2] = a;
    a *= dpp<kRowShr + 4>(A(1), a);
    P.fm[3] = a;
    a *= dpp<kRowShr + 8>(A(1), a);
    P.f15 = a;
    const int row = lane >> 4;
    const A a15 = dpp<kRowBcast15>(A(1), a);   // lane 15 of the previous row
    if (row == 1 || row == 3) a *= a15;
    P.f31 = a;
    // backward
    a = a0;
    P.bm[0] = a;
    a *= dpp<kRowShl + 1>(A(1), a);
    P.bm[1] = a;
    a *= dpp<kRowShl + 2>(A(1), a);
    P.bm[2] = a;
    a *= dpp<kRowShl + 4>(A(1), a);
    P.bm[3] = a;
    a *= dpp<kRowShl + 8>(A(1), a);
    P.bq = a;
    P.s16 = readlane(a, 16);
    P.s32 = readlane(a, 32);
}

// Exact solve of one line in place with a plan.
template <typename A, int E>
__device__ inline void solve_plan(A (&f)[E], const LinePlan<A, E> &P, int lane)
{
    A pr[E];
    A acc = A(0), prod = A(1);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        acc = P.g[e] * f[e] + P.h[e] * acc;
        prod *= P.h[e];
        f[e] = acc;
        pr[e] = prod;
    }
    // inclusive forward scan: rows by shifts, then rows 1, 3 from lane 15 of
    // the row before, rows 2, 3 from lane 31
    A b = f[E - 1];
    b = P.fm[0] * dpp0<kRowShr + 1>(b) + b;
    b = P.fm[1] * dpp0<kRowShr + 2>(b) + b;
    b = P.fm[2] * dpp0<kRowShr + 4>(b) + b;
    b = P.fm[3] * dpp0<kRowShr + 8>(b) + b;
    b = P.f15 * dpp_rows<kRowBcast15, 0xA>(b) + b;
    b = P.f31 * dpp_rows<kRowBcast31, 0xC>(b) + b;
    const A carry_in = dpp0<kWaveShr1>(b);   // y at the last point of lane l-1
#pragma unroll
    for (int e = 0; e < E; ++e) f[e] += pr[e] * carry_in;
    acc = A(0);
    prod = A(1);
#pragma unroll
    for (int e = E - 1; e >= 0; --e) {
        acc = f[e] + P.h[e] * acc;
        prod *= P.h[e];
        f[e] = acc;
        pr[e] = prod;
    }
    // inclusive backward scan: rows by shifts, then the later rows' totals
    // (first lanes of rows 1..3) composed as uniform values
    b = f[0];
    b = P.bm[0] * dpp0<kRowShl + 1>(b) + b;
    b = P.bm[1] * dpp0<kRowShl + 2>(b) + b;
    b = P.bm[2] * dpp0<kRowShl + 4>(b) + b;
    b = P.bm[3] * dpp0<kRowShl + 8>(b) + b;
    const A b1 = readlane(b, 16), b2 = readlane(b, 32), b3 = readlane(b, 48);
    const A q1 = P.s32 * b3 + b2;   // rows > 1
    const A q0 = P.s16 * q1 + b1;   // rows > 0
    const int row = lane >> 4;
    const A q = row == 3 ? A(0) : row == 2 ? b3 : row == 1 ? q1 : q0;
    b = P.bq * q + b;
    const A carry_up = dpp0<kWaveShl1>(b);   // u at the first point of lane l+1
#pragma unroll
    for (int e = 0; e < E; ++e) f[e] += pr[e] * carry_up;
}

// Exact solve of one line in place with the Thomas table fac (g_i, h_i).
template <typename A, int E>
__device__ inline void thomas(A (&f)[E], const Fac<A> *fac, int lane)
{
    LinePlan<A, E> P;
    make_plan<A, E>(P, fac, lane);
    solve_plan<A, E>(f, P, lane);
}

// f -= (a*Tx + b*I) w   (w zero beyond nx)
template <typename A, int E>
__device__ inline void sub_op(A (&f)[E], const A (&w)[E], A a, A b)
{
    if (a != A(0)) {
        const A left = dpp0<kWaveShr1>(w[E - 1]);
        const A right = dpp0<kWaveShl1>(w[0]);
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

// Widest access a lane's E consecutive values allow (bytes; 0: element by element).
template <typename T, int E>
constexpr int chunk_align()
{
    constexpr int cb = E * static_cast<int>(sizeof(T));
    return cb % 16 == 0 ? 16 : cb % 8 == 0 ? 8 : cb % 4 == 0 ? 4 : 0;
}

// A lane whose E points all lie inside the line reads them as one aligned
// chunk (16-byte loads for FP64 with E = 2 or 4, whole dwords for BF16) when
// the row is aligned;
// the lane holding the end of a ragged line goes point by point.
template <typename T, typename A, int E>
__device__ inline void gload(A (&v)[E], const T *row, int nx, int lane)
{
    constexpr int G = chunk_align<T, E>();
    if constexpr (G > 0) {
        if ((reinterpret_cast<uintptr_t>(row) % G) == 0 && (lane + 1) * E <= nx) {
            const T *p = static_cast<const T *>(__builtin_assume_aligned(row + lane * E, G));
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = static_cast<A>(ldv(p + e));
            return;
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = lane * E + e;
        v[e] = i < nx ? static_cast<A>(ldv(row + i)) : A(0);
    }
}

template <typename T, typename A, int E>
__device__ inline void gstore(T *row, const A (&v)[E], int nx, int lane)
{
    constexpr int G = chunk_align<T, E>();
    if constexpr (G > 0) {
        if ((reinterpret_cast<uintptr_t>(row) % G) == 0 && (lane + 1) * E <= nx) {
            T *p = static_cast<T *>(__builtin_assume_aligned(row + lane * E, G));
#pragma unroll
            for (int e = 0; e < E; ++e) stv(p + e, v[e]);
            return;
        }
    }
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
