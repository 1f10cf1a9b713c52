// Internal declarations of the SMG library (not part of the C ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/smg.h"

namespace smg {

// Optional dispatch-stamped start/stop events of one launch (hipExtLaunchKernel):
// the profiler times individual kernels with them; null events = plain launch.
struct LaunchEv {
    hipEvent_t e0 = nullptr;
    hipEvent_t e1 = nullptr;
};

// Launch recorder of the grouped (batched) path, see group.h.  A launch site
// without a grouped twin marks the recording unusable.
struct LaunchRec;
extern thread_local std::vector<LaunchRec> *g_rec;
extern thread_local int g_rec_unsupported;

#define SMG_LAUNCH(EV, K, G, B, L, S, ...)                                          \
    do {                                                                            \
        if (smg::g_rec)                                                             \
            smg::g_rec_unsupported = 1;                                             \
        else if ((EV).e0)                                                           \
            hipExtLaunchKernelGGL(K, G, B, L, S, (EV).e0, (EV).e1, 0, __VA_ARGS__); \
        else                                                                        \
            hipLaunchKernelGGL(K, G, B, L, S, __VA_ARGS__);                         \
    } while (0)

// bfloat16 storage: the upper half of an IEEE binary32, rounded to nearest even.
struct bf16 {
    uint16_t bits;
};

__host__ __device__ inline float bf16_to_f(bf16 v)
{
    union { uint32_t u; float f; } c;
    c.u = static_cast<uint32_t>(v.bits) << 16;
    return c.f;
}

__host__ __device__ inline bf16 f_to_bf16(float f)
{
    union { uint32_t u; float f; } c;
    c.f = f;
    uint32_t u = c.u;
    bf16 r;
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
        r.bits = static_cast<uint16_t>((u >> 16) | 0x40u);   // quiet NaN
    } else {
        u += 0x7fffu + ((u >> 16) & 1u);
        r.bits = static_cast<uint16_t>(u >> 16);
    }
    return r;
}

template <typename T> struct Arith { using type = T; };
template <> struct Arith<bf16> { using type = float; };

__device__ inline double ldv(const double *p) { return *p; }
__device__ inline float ldv(const float *p) { return *p; }
__device__ inline float ldv(const bf16 *p) { return bf16_to_f(*p); }
__device__ inline void stv(double *p, double v) { *p = v; }
__device__ inline void stv(float *p, float v) { *p = v; }
__device__ inline void stv(bf16 *p, float v) { *p = f_to_bf16(v); }

// a * b + c with one rounding, written out so that kernels instantiated for
// different widths round identically (the compiler's own contraction of
// a * b + c * d may pick either product)
__device__ inline double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// V consecutive stored values as one aligned access of V * sizeof(T) bytes.
// The caller guarantees that p is aligned to V elements; n_ok is the number
// of values from p that lie inside the row (or plane): when it is below V
// the values are read one by one, the missing ones as zero, and only the
// valid ones are written.
template <typename T, int V>
struct alignas(V * sizeof(T)) VecPack {
    T e[V];
};

template <typename T, typename A, int V>
__device__ inline void vld(A (&v)[V], const T *p, int n_ok)
{
    if constexpr (V == 1) {
        v[0] = n_ok > 0 ? static_cast<A>(ldv(p)) : A(0);
    } else if (n_ok >= V) {
        const VecPack<T, V> pk = *reinterpret_cast<const VecPack<T, V> *>(p);
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] = ldv(&pk.e[e]);
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] = e < n_ok ? static_cast<A>(ldv(p + e)) : A(0);
    }
}

template <typename T, typename A, int V>
__device__ inline void vst(T *p, const A (&v)[V], int n_ok)
{
    if constexpr (V == 1) {
        if (n_ok > 0) stv(p, v[0]);
    } else if (n_ok >= V) {
        VecPack<T, V> pk;
#pragma unroll
        for (int e = 0; e < V; ++e) stv(&pk.e[e], v[e]);
        *reinterpret_cast<VecPack<T, V> *>(p) = pk;
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e)
            if (e < n_ok) stv(p + e, v[e]);
    }
}

// V stored values held in registers as they were read (BF16 stays packed two
// to a register until it is used); zero bits read as zero in every type.
template <typename T, int V>
struct Held {
    VecPack<T, V> p;
};

template <typename T, int V>
__device__ inline void hld(Held<T, V> &h, const T *p, int n_ok)
{
    if (n_ok >= V) {
        h.p = *reinterpret_cast<const VecPack<T, V> *>(p);
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            if (e < n_ok)
                h.p.e[e] = p[e];
            else
                h.p.e[e] = T{};
        }
    }
}

template <typename T, typename A, int V>
__device__ inline void unpack(A (&v)[V], const Held<T, V> &h)
{
#pragma unroll
    for (int e = 0; e < V; ++e) v[e] = ldv(&h.p.e[e]);
}

// Points per thread of the streaming kernels: eight bytes of storage per lane
// and access in every precision.
template <typename T>
constexpr int stream_vec() { return static_cast<int>(8 / sizeof(T)); }

// Points per thread along x for the tiled streaming kernels (tiles of 64 V
// points): the widest power of two up to the storage type's vector width
// that divides nx and leaves at most an eighth of the tiles' points idle
// (wider tiles with idle lanes cost more in registers than they save).
template <typename T>
inline int tile_vec(int nx, int widest = stream_vec<T>())
{
    for (int v = widest; v > 1; v /= 2) {
        if (nx % v != 0) continue;
        const int w = 64 * v, waste = (nx + w - 1) / w * w - nx;
        if (8 * waste <= nx) return v;
    }
    return 1;
}

// Coefficients of one x-line of a 2D level: L_j = la*Tx + lb*I, coupling to
// line j+1 V_j = va*Tx + vb*I, Thomas table index fac.
template <typename A>
struct LineCoef {
    A la, lb, va, vb;
    int fac;
    int pad;
};

// Coefficients of one plane of a 3D level: C_K = ca*T2 + cb*I, coupling to
// plane K+1 U_K = ua*T2 + ub*I, plane type pt (index of its 2D hierarchy).
template <typename A>
struct PlaneCoef {
    A ca, cb, ua, ub;
    int pt;
    int pad;
};

// Thomas factors of one line operator: y_i = g_i f_i + h_i y_{i-1};
// u_i = y_i + h_i u_{i+1}; padded entries are zero.
template <typename A>
struct Fac {
    A g, h;
};

struct Level3 {
    int nz;
    size_t n;          // nx*ny*nz points
    size_t pcoef_off;  // offset of this level's PlaneCoef rows
};

// Kernel argument blocks --------------------------------------------------

template <typename T, typename A>
struct LineRelaxArgs {
    T *x;                    // 2D x of this level
    const T *b;              // 2D right-hand side
    long long xps, xrs;      // plane and rhs strides of x
    long long bps, brs;      // plane and rhs strides of b
    int nx, ny;              // line length, lines in this 2D level
    int colour, nq;          // lines j = 2q + colour (or j = q when ny == 1)
    int np, nrhs;            // planes in the batch, right-hand sides
    int kmul, koff;          // 3D plane of batch plane p: k = p*kmul + koff
    const PlaneCoef<A> *pc;  // this 3D level's plane rows
    const LineCoef<A> *lc;   // line rows of 2D level l of plane type 0
    int lines_total;         // line rows per plane type
    const Fac<A> *fac;       // Thomas tables
    int nxp;                 // padded table length
    int nbr_zero;            // neighbour lines are known to be zero
};

template <typename T, typename A>
struct Restrict2Args {
    const T *x; const T *b; T *bc;
    long long xps, xrs, bps, brs, cps, crs;
    int nx, ny, nyc, np, nrhs, kmul, koff;
    const PlaneCoef<A> *pc;
    const LineCoef<A> *lc;
    int lines_total;
    int x_zero;
};

template <typename T, typename A>
struct Prolong2Args {
    T *x; const T *xc;
    long long xps, xrs, cps, crs;
    int nx, ny, nyc, np, nrhs;
    int x_zero;
};

template <typename T, typename A>
struct Resid3Args {
    const T *x; const T *b; T *r;      // r: packed batch planes
    long long xrs, brs, rps, rrs;       // x and b: whole 3D level, packed planes
    int nx, ny, nz, np, nrhs, kmul, koff;
    A cx, cy;
    const PlaneCoef<A> *pc;
    int self_zero;
    int vmax;               // widest points per thread allowed (0: no limit)
};

template <typename T, typename A>
struct Correct3Args {
    T *x; const T *y;
    long long xrs, yps, yrs;
    int nx, ny, np, nrhs, kmul, koff;
};

template <typename T, typename A>
struct Restrict3Args {
    const T *x; const T *b; T *bc;
    long long xrs, brs, crs;
    int nx, ny, nz, nzc, nrhs;
    A cx, cy;
    const PlaneCoef<A> *pc;
    int x_zero;             // x is known to be zero: bc = P^T b
    int kchunk;             // coarse planes per block of the marching kernel (set by the launcher)
    int vmax;               // widest points per thread allowed (0: no limit)
};

template <typename T, typename A>
struct Prolong3Args {
    T *x; const T *xc;
    long long xrs, crs;
    int nx, ny, nz, nzc, nrhs;
    int x_zero;             // x is known to be zero: x = P xc
};

// Fused-schedule argument blocks (smg_fused.hip) ---------------------------
constexpr int kMaxLev = 16;     // 2D levels (ny <= 2^15) and 3D chain arrays
constexpr int kMaxLev3 = 24;

template <typename T, typename A>
struct Down2Args {
    const T *b; T *x; T *bc;
    long long bps, brs, xps, xrs, cps, crs;
    int nx, nxp, ny, nyc, S, np, nrhs, kmul, koff;
    const PlaneCoef<A> *pc;
    const LineCoef<A> *lc;      // rows of this 2D level, plane type 0
    int lines_total;
    const Fac<A> *fac;
    int march_waves;        // a launch marches runs of coarse lines while it keeps >= this many waves (0: never)
    int kr;                 // coarse lines per wave of the marching kernel (set by the launcher)
};

template <typename T, typename A>
struct Coarse2Args {
    const T *b; T *out;
    long long bps, brs, ops, ors;
    int nx, nxp, np, nrhs, kmul, koff;
    int l0, nlev;
    int ny2[kMaxLev], lev_off[kMaxLev];
    int ipre, ipost, accumulate;
    const PlaneCoef<A> *pc;
    const LineCoef<A> *lc;      // rows of 2D level 0, plane type 0
    int lines_total;
    const Fac<A> *fac;
    // down-only mode (one pre-smoothing sweep, no post-smoothing): the
    // kernel leaves every level's x (l0 .. nlev-1) in xl[l] (plane stride
    // nx*ny2[l], rhs stride P2 times that) for the prolongation chain
    int down_only, P2;
    T *xl[kMaxLev];
};

template <typename T, typename A>
struct Chain2Args {
    const T *x0; T *out;
    long long x0ps, x0rs, ops, ors;
    const T *xc[kMaxLev];
    long long cps[kMaxLev], crs[kMaxLev];
    int nx, np, nrhs, lc;
    int ny2[kMaxLev];
    int accumulate;
    int vmax;               // widest points per thread allowed (0: no limit)
};

template <typename T, typename A>
struct Up2Args {
    const T *xpre; const T *xc; const T *b; T *out;
    long long xps, xrs, cps, crs, bps, brs, ops, ors;
    int nx, nxp, ny, nyc, S, np, nrhs, kmul, koff;
    const PlaneCoef<A> *pc;
    const LineCoef<A> *lc;      // rows of this 2D level, plane type 0
    int lines_total;
    const Fac<A> *fac;
    int accumulate;
};

template <typename T, typename A>
struct Chain3Args {
    T *x[kMaxLev3];
    long long rs[kMaxLev3];
    int nz[kMaxLev3];
    int L, nx, ny;
    int vmax;               // widest points per thread allowed (0: no limit)
    // Optional Krylov dots taken while the fine level is stored (FP64, one
    // right-hand side): per block, (s, dr) into dpart[b] and (s, dq) (0 unless
    // want_sq) into dpart[chain3_blocks + b]; dpart null skips them.
    const double *dr, *dq;
    double *dpart;
    int want_sq;
};

template <typename T, typename A>
void launch_down2(const Down2Args<T, A> &a, hipStream_t st, const LaunchEv &ev = LaunchEv{});
template <typename T, typename A>
void launch_coarse2(const Coarse2Args<T, A> &a, size_t lds_bytes, hipStream_t st, const LaunchEv &ev = LaunchEv{});
template <typename T, typename A>
void launch_chain2(const Chain2Args<T, A> &a, hipStream_t st, const LaunchEv &ev = LaunchEv{});
template <typename T, typename A>
void launch_up2(const Up2Args<T, A> &a, hipStream_t st, const LaunchEv &ev = LaunchEv{});
template <typename T, typename A>
void launch_chain3(const Chain3Args<T, A> &a, int nrhs, hipStream_t st, const LaunchEv &ev = LaunchEv{});
// blocks of one FP64 3D chain launch over an nx x ny x nz level (one right-hand side)
long long chain3_blocks(int nx, int ny, int nz);
int fused_waves();   // waves per workgroup of the strip and coarse kernels

// Launchers (smg_kernels.hip) ---------------------------------------------
template <typename T, typename A>
void launch_line_relax(const LineRelaxArgs<T, A> &a, hipStream_t st, const LaunchEv &ev = LaunchEv{});
template <typename T, typename A>
void launch_restrict2(const Restrict2Args<T, A> &a, hipStream_t st, const LaunchEv &ev = LaunchEv{});
template <typename T, typename A>
void launch_prolong2(const Prolong2Args<T, A> &a, hipStream_t st, const LaunchEv &ev = LaunchEv{});
template <typename T, typename A>
void launch_resid3(const Resid3Args<T, A> &a, hipStream_t st, const LaunchEv &ev = LaunchEv{});
template <typename T, typename A>
void launch_correct3(const Correct3Args<T, A> &a, hipStream_t st, const LaunchEv &ev = LaunchEv{});
template <typename T, typename A>
void launch_restrict3(const Restrict3Args<T, A> &a, hipStream_t st, const LaunchEv &ev = LaunchEv{});
template <typename T, typename A>
void launch_prolong3(const Prolong3Args<T, A> &a, hipStream_t st, const LaunchEv &ev = LaunchEv{});
template <typename A>
void launch_thomas_tables(const LineCoef<double> *uniq_ab, int nfac, int nx, int nxp, Fac<A> *out, hipStream_t st);
template <typename T>
void launch_convert_in(const double *src, long long lds, T *dst, long long ldd, size_t n, int nrhs, hipStream_t st);
template <typename T>
void launch_convert_out(const T *src, long long lds, double *dst, long long ldd, size_t n, int nrhs, hipStream_t st);

// Krylov / vector kernels (krylov_kernels.hip) ----------------------------
struct KScalars {           // device-resident recurrence scalars
    double sr, sr_prev, sq, pq, alpha, alpha_prev, beta, rr, bb;
    int breakdown;
    int nonfinite;          // batched: non-finite start
    // batched solves: device-side iteration count and stopping test
    double rtol, bden, true_rr;
    int active, iters, max_iter, pad;
};

constexpr int kRedBlocks = 1024;   // fixed grid of the first reduction stage

// argument blocks of the Krylov kernels
struct ResidArgs {
    const double *b, *x;
    double *r;
    int nx, ny, nz;
    double cx, cy, cz;
    int kchunk, x_zero;
    double *partials;
};
struct DotsArgs {
    const double *s, *r, *q;
    int want_sq;
    long long n;
    double *partials;
};
struct UpdPQArgs {
    const double *s, *p_old;
    double *p_new, *q;
    const KScalars *sc;
    int nx, ny, nz;
    double cx, cy, cz;
    int kchunk;
    double *partials;
};
struct UpdXRArgs {
    double *x, *r;
    const double *p, *q;
    const KScalars *sc;
    long long n;
    double *partials;
};
struct FinArgs {
    int which, method, k, batched;
    const double *partials;
    KScalars *sc;
    double rtol;
    int max_iter;
    int nparts;             // partials per quantity (0: kRedBlocks)
};
struct CopyArgs {
    const double *src;
    double *dst;
    long long n;
};
struct FillArgs {
    double *dst;
    double v;
    long long n;
};

void launch_matvec7(const double *x, double *y, long long ld, int nrhs, int nx, int ny, int nz,
                    double cx, double cy, double cz, hipStream_t st);
void launch_init_resid(const double *b, const double *x, double *r, int x_zero, int nx, int ny, int nz,
                       double cx, double cy, double cz, double *partials, hipStream_t st);
void launch_dots_sr_sq(const double *s, const double *r, const double *q, int want_sq, size_t n,
                       double *partials, hipStream_t st);
void launch_update_p_q(const double *s, const double *p_old, double *p_new, double *q, const KScalars *sc,
                       int nx, int ny, int nz, double cx, double cy, double cz, double *partials, hipStream_t st);
void launch_update_xr(double *x, double *r, const double *p, const double *q, const KScalars *sc, size_t n,
                      double *partials, hipStream_t st);
// finalize: stage 2 of the reductions and the scalar recurrence.
// which: 0 = init (rr, bb), 1 = beta (sr, sq), 2 = alpha (pq), 3 = rr
// nparts: partials per quantity when they come from another grid (0: kRedBlocks)
void launch_finalize(int which, int method, int k, const double *partials, KScalars *sc, KScalars *host_copy,
                     hipStream_t st, int nparts = 0);
// batched mode of finalize: stopping test on the device (see KScalars)
void launch_finalize_batched(int which, int method, const double *partials, KScalars *sc, double rtol, int max_iter,
                             hipStream_t st, int nparts = 0);
void launch_copy(const double *src, double *dst, size_t n, hipStream_t st);
void launch_fill(double *dst, double v, size_t n, hipStream_t st);
void launch_true_resid(const double *b, const double *x, double *tmp, int nx, int ny, int nz, double cx,
                       double cy, double cz, double *partials, hipStream_t st);
// out = alpha a + beta b
void launch_axpby(double *out, const double *a, double alpha, const double *b, double beta, size_t n, hipStream_t st);
// (a1, b1) and (a2, b2) (a2, b2 may be null): fixed-grid partials on the
// device, summed on the host in a fixed order; synchronises st
int device_dot2(const double *a1, const double *b1, const double *a2, const double *b2, size_t n, double *partials,
                hipStream_t st, double *d1, double *d2);

}  // namespace smg

namespace smg {
// The Krylov buffers of a handle and its V-cycle, for the batched driver.
struct KrylovView {
    double *r, *s, *q, *pa, *pb, *part;
    KScalars *sc;
    smg_grid g;
    size_t n;
    int precision;
};
int krylov_view(smg_handle *h, KrylovView *v);
void vcycle_apply(smg_handle *h, const double *r, double *s, int nrhs, long long ld, hipStream_t st);
// s = B r for one right-hand side of length N, also taking the Krylov dots
// (s, r) and, with want_sq, (s, q) where the cycle ends in the FP64 3D chain:
// then returns true with the partials' array and count per quantity for the
// finalize step; false means s alone was computed.
bool vcycle_dots(smg_handle *h, const double *r, double *s, const double *q, int want_sq, hipStream_t st,
                 const double **part, int *nparts);
}  // namespace smg

// Handle queries shared by the library's translation units.
int smg_handle_size(const smg_handle *h, size_t *n);
const smg_grid *smg_handle_grid(const smg_handle *h);
namespace smg {
// the handle's reduction partials (2 * kRedBlocks doubles), free between solver steps
double *handle_partials(smg_handle *h);

// Variable-coefficient hierarchy (varcoef.hip): one per handle set up by smgv_setup
struct VarHier;
size_t var_workspace_bytes(int nx, int ny, int nz);
VarHier *var_create(int nx, int ny, int nz, const smg_opts *o, int interp, char *ws, const double *diag,
                    const double *ax, const double *ay, const double *az, hipStream_t st);
void var_destroy(VarHier *H);
void var_vcycle(VarHier *H, const double *r, double *s, int nrhs, long long ld, hipStream_t st);
void var_matvec(VarHier *H, const double *x, double *y, int nrhs, long long ld, hipStream_t st);
void var_init_resid(VarHier *H, const double *b, const double *x, double *r, int x_zero, double *partials,
                    hipStream_t st);
void var_update_p_q(VarHier *H, const double *s, const double *p_old, double *p_new, double *q, const KScalars *sc,
                    double *partials, hipStream_t st);
int var_levels(const VarHier *H, int *nlev3, int *nlev2);
int var_export(const VarHier *H, int l, int l2, double *out, hipStream_t st);
}  // namespace smg
// nonzero for a handle of smgv_setup (variable coefficients)
int smg_handle_is_var(const smg_handle *h);
int smg_handle_max_nrhs(const smg_handle *h, int32_t *max_nrhs);
