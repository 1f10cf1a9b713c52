// SMG for a variable-coefficient 7-point operator on gfx950.
//
// SMG was built for general structured-grid operators (Section 1, Schaffer's
// semicoarsening multigrid); the paper applies it to the constant Laplacian.
// This file carries the same V-cycle (z-semicoarsening, zebra plane
// relaxation whose plane solves are 2D y-semicoarsening cycles with zebra
// x-line relaxation, Galerkin coarse operators, correction form, pre F then
// C and post C then F) to a symmetric 7-point operator given per point,
//     (A x)_p = diag_p x_p - sum_e (a_e[p] x_{p+e} + a_e[p-e] x_{p-e}),
// where nothing is shared between points any more:
//   * every 3D level stores its operator per point: the in-plane block C_k
//     (5-point, symmetric: centre, east, north) and the coupling U_k from
//     plane k to plane k+1 (5-point: centre, east, west, north, south);
//   * prolongation has one weight per point of an even (F) plane for each of
//     its two C-plane neighbours: 1/2 (linear), or the F-point's collapsed
//     couplings to the two planes, a/(a+b) and b/(a+b) (operator-dependent);
//     an F-plane with one C-neighbour takes 1/2 from it;
//   * the Galerkin product P^T A P is formed per coarse point from the fine
//     blocks and the diagonal weight matrices; the products of diagonal
//     weights with 5-point blocks stay 5-point, so coarse 3D levels are
//     15-point (5 in-plane points on 3 planes);
//   * every plane of every 3D level has its own 2D hierarchy built the same
//     way in y: line blocks L_j (tridiagonal, symmetric) and couplings V_j
//     (tridiagonal) per point, 9-point coarse 2D operators;
//   * x-line solves use per-line LU factors of L_j.  One wave solves one line
//     of up to 512 points: each lane holds E consecutive points, composes the
//     affine maps of the forward (and then backward) Thomas recurrence over
//     them, and the 64 lanes combine their maps by DPP scans.
// Storage, all FP64, x fastest within a plane, planes (or lines) outermost.
// The hierarchy lives in the caller's workspace; the host schedules one
// launch per stage, looping over right-hand sides, except that without
// post-smoothing the upward half of each 2D cycle is one chain kernel.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "line_ops.hpp"
#include "smg_internal.h"

namespace smg {

struct VarLevel3 {
    int nz;                      // planes
    size_t cc, ce, cn;           // C_k: centre, (i,j)-(i+1,j), (i,j)-(i,j+1)
    size_t uc, ue, uw, un, us;   // U_k: (i,j) in plane k to (i,j), (i+1,j), (i-1,j), (i,j+1), (i,j-1) in k+1
    size_t wdn, wup;             // weights of even planes (to coarse K-1 below and K above)
    size_t x, b;                 // level vectors (levels >= 1)
    std::vector<size_t> lc, le, vc, ve, vw, ydn, yup, invm, g;   // per 2D level, all planes
};

struct VarHier {
    int nx, ny, nz, pre, post, ipre, ipost, order, interp;
    size_t N;
    char *ws;
    std::vector<int> ny2;        // lines per 2D level
    std::vector<VarLevel3> lev;
    std::vector<size_t> bx2, bb2;   // 2D batch buffers per 2D level
    size_t total;
    template <typename X> X *at(size_t off) const { return reinterpret_cast<X *>(ws + off); }
};

namespace {

constexpr int kB = 256;
constexpr int kVcMaxLev = 16;   // 2D levels of the chained kernel (ny <= 2^15)

inline unsigned nblk(long long n, int b) { return static_cast<unsigned>((n + b - 1) / b); }

size_t al(size_t v) { return (v + 255) / 256 * 256; }

// ---------------------------------------------------------------------------
// Setup kernels
// ---------------------------------------------------------------------------

// level 0 from the caller's operator: C = diag, -ax, -ay; U = -az at the centre
__global__ void k_var_fine(const double *diag, const double *ax, const double *ay, const double *az, int nx, int ny,
                           int nz, double *cc, double *ce, double *cn, double *uc, double *ue, double *uw, double *un,
                           double *us)
{
    const long long n = static_cast<long long>(nx) * ny * nz;
    const long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int i = static_cast<int>(p % nx), j = static_cast<int>((p / nx) % ny), k = static_cast<int>(p / nx / ny);
    cc[p] = diag[p];
    ce[p] = i + 1 < nx ? -ax[p] : 0.0;
    cn[p] = j + 1 < ny ? -ay[p] : 0.0;
    uc[p] = k + 1 < nz ? -az[p] : 0.0;
    ue[p] = uw[p] = un[p] = us[p] = 0.0;
}

// Interpolation weights of the even fine blocks f along the outer index of a
// level with nb blocks of nx x ny points (ns such operators stacked one after
// another): wdn (from the block below) and wup (from the block above).  The
// collapsed couplings of point p are a = -(column sum of the coupling from
// block f-1 into p) and b = -(row sum of the coupling from p into block
// f+1); with `op` and both positive the weights are a/(a+b) and b/(a+b), else
// 1/2.  A block with one neighbour takes 1/2.  Planes couple 5-point
// (E/W/N/S); lines are the case ny = 1 (3-point, un and us null).
__global__ void k_var_weights(const double *uc, const double *ue, const double *uw, const double *un,
                              const double *us, int nx, int ny, int nb, int ns, int op, double *wdn, double *wup)
{
    const long long m = static_cast<long long>(nx) * ny;
    const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= m * nb * ns) return;
    const int f = static_cast<int>((e / m) % nb);
    if (f % 2) return;
    const long long p = e % m;
    const int i = static_cast<int>(p % nx), j = static_cast<int>(p / nx);
    const bool has_dn = f >= 1, has_up = f + 1 < nb;
    double wd = has_dn ? 0.5 : 0.0, wu = has_up ? 0.5 : 0.0;
    if (op && has_dn && has_up) {
        const long long d = e - m, u = e;    // coupling blocks f-1 -> f and f -> f+1, at p
        double a = uc[d];
        if (i > 0) a += ue[d - 1];
        if (i + 1 < nx) a += uw[d + 1];
        if (j > 0) a += un[d - nx];
        if (j + 1 < ny) a += us[d + nx];
        a = -a;
        double b = uc[u] + ue[u] + uw[u];
        if (ny > 1) b += un[u] + us[u];
        b = -b;
        if (a > 0.0 && b > 0.0) {
            wd = a / (a + b);
            wu = b / (a + b);
        }
    }
    wdn[e] = wd;
    wup[e] = wu;
}

// Views of a block operator with nb blocks of nx x ny points: C (symmetric
// in-block: cc, ce, cn) and U (block f to f+1: uc, ue, uw, un, us).  Lines
// are the case ny = 1 (cn, un, us unused).
struct BlockOp {
    const double *cc, *ce, *cn, *uc, *ue, *uw, *un, *us;
    int nx, ny;
    // C_f[p][q], q = p + (di, dj) with |di| + |dj| <= 1, inside the block
    __device__ double C(long long base, int i, int j, int di, int dj) const
    {
        const long long p = base + static_cast<long long>(j) * nx + i;
        if (di == 0 && dj == 0) return cc[p];
        if (di == 1) return ce[p];
        if (di == -1) return ce[p - 1];
        if (dj == 1) return cn[p];
        return cn[p - nx];
    }
    // U_f[p][q]: p in block f, q = p' + (di, dj) in block f+1
    __device__ double U(long long base, int i, int j, int di, int dj) const
    {
        const long long p = base + static_cast<long long>(j) * nx + i;
        if (di == 0 && dj == 0) return uc[p];
        if (di == 1) return ue[p];
        if (di == -1) return uw[p];
        if (dj == 1) return un[p];
        return us[p];
    }
    // U_f[q][p]: q = p + (di, dj) in block f, p' in block f+1 (the transposed coupling)
    __device__ double Ut(long long base, int i, int j, int di, int dj) const
    {
        return U(base, i + di, j + dj, -di, -dj);
    }
};

// Galerkin P^T A P of a block-tridiagonal operator under the per-point
// semicoarsening prolongation: coarse block K sits on fine block f1 = 2K+1,
// fine f0 = 2K takes wup[f0] of coarse K, fine f2 = 2K+2 takes wdn[f2] of K
// (and wup[f2] of K+1).  With W the diagonal weight matrices:
//   C^c_K = W0 C_f0 W0 + C_f1 + W2 C_f2 W2 + W0 U_f0 + U_f0^T W0 + U_f1 W2 + W2 U_f1^T
//   U^c_K = U_f1 W2' + W2 C_f2 W2' + W2 U_f2            (W0 = wup[f0], W2 = wdn[f2], W2' = wup[f2])
// terms of missing fine blocks dropped.  One thread per coarse point.
__global__ void k_var_galerkin(BlockOp F, const double *wdn, const double *wup, int nb, int ns, double *cc,
                               double *ce, double *cn, double *uc, double *ue, double *uw, double *un, double *us)
{
    const int nx = F.nx, ny = F.ny;
    const long long m = static_cast<long long>(nx) * ny;
    const int nc = nb / 2;
    const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= m * nc * ns) return;
    const long long sbase = (e / (m * nc)) * m * nb;   // the stacked operator's fine blocks
    const int K = static_cast<int>((e / m) % nc);
    const long long p = e % m;
    const int i = static_cast<int>(p % nx), j = static_cast<int>(p / nx);
    const int f0 = 2 * K, f1 = 2 * K + 1, f2 = 2 * K + 2, f3 = 2 * K + 3;
    const bool h2 = f2 < nb, h3 = f3 < nb;
    const long long b0 = sbase + f0 * m, b1 = sbase + f1 * m, b2 = sbase + f2 * m;
    auto in = [&](int di, int dj) { return i + di >= 0 && i + di < nx && j + dj >= 0 && j + dj < ny; };
    auto w = [&](const double *wt, long long base, int di, int dj) {
        return wt[base + static_cast<long long>(j + dj) * nx + i + di];
    };
    // C^c at q = p, p+x, p+y
    const int dq[3][2] = {{0, 0}, {1, 0}, {0, 1}};
    double outc[3];
    for (int t = 0; t < 3; ++t) {
        const int di = dq[t][0], dj = dq[t][1];
        if (!in(di, dj)) {
            outc[t] = 0.0;
            continue;
        }
        const double w0p = w(wup, b0, 0, 0), w0q = w(wup, b0, di, dj);
        double v = w0p * F.C(b0, i, j, di, dj) * w0q + F.C(b1, i, j, di, dj);
        v += w0p * F.U(b0, i, j, di, dj) + F.Ut(b0, i, j, di, dj) * w0q;
        if (h2) {
            const double w2p = w(wdn, b2, 0, 0), w2q = w(wdn, b2, di, dj);
            v += w2p * F.C(b2, i, j, di, dj) * w2q;
            v += F.U(b1, i, j, di, dj) * w2q + w2p * F.Ut(b1, i, j, di, dj);
        }
        outc[t] = v;
    }
    cc[e] = outc[0];
    ce[e] = outc[1];
    if (cn) cn[e] = outc[2];
    // U^c at q = p', p'+x, p'-x, p'+y, p'-y
    const int du[5][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    double outu[5];
    for (int t = 0; t < 5; ++t) {
        const int di = du[t][0], dj = du[t][1];
        outu[t] = 0.0;
        if (!h3 || !in(di, dj)) continue;
        const double w2p = w(wdn, b2, 0, 0), wq = w(wup, b2, di, dj);
        outu[t] = F.U(b1, i, j, di, dj) * wq + w2p * F.C(b2, i, j, di, dj) * wq + w2p * F.U(b2, i, j, di, dj);
    }
    uc[e] = outu[0];
    ue[e] = outu[1];
    uw[e] = outu[2];
    if (un) {
        un[e] = outu[3];
        us[e] = outu[4];
    }
}

// 2D level 0 of every plane of a 3D level: L_j = the x-part of C_k on line j,
// V_j = C_k's coupling of line j to line j+1 (diagonal)
__global__ void k_var_plane0(const double *cc, const double *ce, const double *cn, long long n, double *lc, double *le,
                             double *vc, double *ve, double *vw)
{
    const long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    lc[p] = cc[p];
    le[p] = ce[p];
    vc[p] = cn[p];
    ve[p] = vw[p] = 0.0;
}

// LU factors of every line block: invm[i] = 1/m_i, g[i] = le_i / m_i with
// m_0 = lc_0, m_{i+1} = lc_{i+1} - le_i g_i (the blocks are SPD: no pivoting)
__global__ void k_var_factor(const double *lc, const double *le, long long nlines, int nx, double *invm, double *g)
{
    const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nlines) return;
    const long long b = t * nx;
    double m = lc[b];
    for (int i = 0; i < nx; ++i) {
        const double im = 1.0 / m;
        invm[b + i] = im;
        const double gi = i + 1 < nx ? le[b + i] * im : 0.0;
        g[b + i] = gi;
        if (i + 1 < nx) m = lc[b + i + 1] - le[b + i] * gi;
    }
}

// ---------------------------------------------------------------------------
// V-cycle kernels
// ---------------------------------------------------------------------------

struct Lines {                    // a 2D level of all planes of a 3D level
    const double *lc, *le, *vc, *ve, *vw, *invm, *g;
    int nx, ny;
};

// (Q x)_j[i] on line j of a plane's 2D level: L_j x_j + V_{j-1}^T x_{j-1} + V_j x_{j+1}
// (OWN false: without L_j x_j, for a line whose x is still zero)
template <bool OWN = true>
__device__ inline double q_line(const Lines &Q, long long cb, const double *x, long long xb, int j, int i)
{
    // Every operand is loaded at an index clamped into the plane, so all the
    // loads are in flight together; a term past an edge is then skipped, and
    // the sum keeps the stencil's order.
    const int nx = Q.nx;
    const long long c = cb + static_cast<long long>(j) * nx + i, xc = xb + static_cast<long long>(j) * nx + i;
    const bool hw = i > 0, he = i + 1 < nx, hs = j > 0, hn = j + 1 < Q.ny;
    const int dw = hw ? 1 : 0, de = he ? 1 : 0;
    const long long ds = hs ? nx : 0, dn = hn ? nx : 0;
    double v = 0.0;
    if constexpr (OWN) {
        const double l0 = Q.lc[c], lw = Q.le[c - dw], le = Q.le[c];
        const double x0 = x[xc], xw = x[xc - dw], xe = x[xc + de];
        v = l0 * x0;
        if (hw) v += lw * xw;
        if (he) v += le * xe;
    }
    const long long d = c - ds, xd = xc - ds, xu = xc + dn;
    const double sc = Q.vc[d], sw = Q.ve[d - dw], se = Q.vw[d + de];
    const double xs0 = x[xd], xsw = x[xd - dw], xse = x[xd + de];
    const double nc = Q.vc[c], ne = Q.ve[c], nw = Q.vw[c];
    const double xn0 = x[xu], xne = x[xu + de], xnw = x[xu - dw];
    if (hs) {
        v += sc * xs0;
        if (hw) v += sw * xsw;
        if (he) v += se * xse;
    }
    if (hn) {
        v += nc * xn0;
        if (he) v += ne * xne;
        if (hw) v += nw * xnw;
    }
    return v;
}

// Zebra half-sweep over the lines of one colour, for np planes at once:
// x_j += L_j^{-1} (b - Q x)_j.  One wave per line.  Plane pb of the batch is
// plane k0 + ks*pb of the level's coefficient arrays.
// Phase 1 (coalesced: lane handles points t*64 + lane): the residual r and
// the forward Thomas coefficients alpha_i = -le_{i-1}/m_i, beta_i = r_i/m_i and
// g_i go to LDS.  Phase 2 (lane l owns the E consecutive points l*E ..): the
// recurrence y_i = alpha_i y_{i-1} + beta_i and then u_i = y_i - g_i u_{i+1} as
// affine maps composed over the lane's points and combined across lanes by
// DPP scans (scan_fwd, scan_bwd); u overwrites beta.  Phase 3 (coalesced):
// x += u.  LDS rows are padded to an odd stride per chunk so that the chunk
// reads spread over the banks.
constexpr int kRelaxWaves = kB / 64;
__host__ __device__ constexpr int relax_stride(int E) { return E % 2 ? E : E + 1; }

// ordering of one wave's LDS writes and reads across its lanes
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Scans of affine maps x -> A x + B across the 64 lanes of a wave on DPP, for
// per-line coefficients (no precomputed products): within each 16-lane row
// by shifts 1, 2, 4, 8 (lanes without a source compose with the identity),
// then across rows.  Composition of a map with the one before it:
// (A, B) o (A', B') = (A A', A B' + B).
template <int CTRL, int ROWS>
__device__ inline double dpp_rows_id(double old, double v)
{
    const long long o = __double_as_longlong(old), s = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(static_cast<int>(o), static_cast<int>(s), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(static_cast<int>(o >> 32), static_cast<int>(s >> 32), CTRL, ROWS, 0xf,
                                               false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// inclusive prefix: lane l ends with the composition of lanes l, l-1, .., 0
__device__ inline void scan_fwd(double &A, double &B)
{
    using namespace lineops;
#define SMG_VSTEP(CTRL)                                  \
    {                                                    \
        const double Ap = dpp<CTRL>(1.0, A);             \
        const double Bp = dpp0<CTRL>(B);                 \
        B = A * Bp + B;                                  \
        A = A * Ap;                                      \
    }
    SMG_VSTEP(kRowShr + 1)
    SMG_VSTEP(kRowShr + 2)
    SMG_VSTEP(kRowShr + 4)
    SMG_VSTEP(kRowShr + 8)
#undef SMG_VSTEP
    {   // rows 1 and 3 from lane 15 of the row before
        const double Ap = dpp_rows_id<kRowBcast15, 0xA>(1.0, A), Bp = dpp_rows_id<kRowBcast15, 0xA>(0.0, B);
        B = A * Bp + B;
        A = A * Ap;
    }
    {   // rows 2 and 3 from lane 31
        const double Ap = dpp_rows_id<kRowBcast31, 0xC>(1.0, A), Bp = dpp_rows_id<kRowBcast31, 0xC>(0.0, B);
        B = A * Bp + B;
        A = A * Ap;
    }
}

// suffix: lane l ends with its map composed with those of lanes l+1 .. 63
// applied to zero beyond the last lane (only B is needed afterwards)
__device__ inline void scan_bwd(double &A, double &B, int lane)
{
    using namespace lineops;
#define SMG_VSTEP(CTRL)                                  \
    {                                                    \
        const double Ap = dpp<CTRL>(1.0, A);             \
        const double Bp = dpp0<CTRL>(B);                 \
        B = A * Bp + B;                                  \
        A = A * Ap;                                      \
    }
    SMG_VSTEP(kRowShl + 1)
    SMG_VSTEP(kRowShl + 2)
    SMG_VSTEP(kRowShl + 4)
    SMG_VSTEP(kRowShl + 8)
#undef SMG_VSTEP
    // each row's total map sits at its first lane; u entering row r from the
    // right is rows r+1 .. 3 applied to zero
    const double a1 = readlane(A, 16), b1 = readlane(B, 16);
    const double a2 = readlane(A, 32), b2 = readlane(B, 32);
    const double b3 = readlane(B, 48);
    const double u2 = b3, u1 = a2 * u2 + b2, u0 = a1 * u1 + b1;
    const int row = lane >> 4;
    const double u = row == 3 ? 0.0 : row == 2 ? u2 : row == 1 ? u1 : u0;
    B = A * u + B;
}

// Half-sweeps of a 2D level whose x starts at zero (no fill needed): the
// first colour's lines solve L_j x_j = b_j (MODE 1), the second colour's
// L_j x_j = b_j - V x of the neighbours (MODE 2); both assign x.  MODE 0 is
// the correction x_j += L_j^{-1} (b - Q x)_j.
// One line of a zebra half-sweep by one wave (the three phases above);
// lds: this wave's 3 * 64 * relax_stride(E) doubles.
template <int E, int MODE>
__device__ inline void relax_line(const Lines &Q, const double *b, double *x, long long cb, long long xb, int j,
                                  double *lds)
{
    constexpr int S = relax_stride(E);
    constexpr int ROW = 64 * S;
    const int lane = threadIdx.x & 63;
    double *Rb = lds, *Al = lds + ROW, *Gl = lds + 2 * ROW;
    auto pos = [](int i) { return (i / E) * S + i % E; };
    const int nx = Q.nx;
    const long long cl = cb + static_cast<long long>(j) * nx, xl = xb + static_cast<long long>(j) * nx;
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int i = t * 64 + lane;
        double al = 0.0, be = 0.0, gi = 0.0;
        if (i < nx) {
            const double im = Q.invm[cl + i];
            const double q = MODE == 1 ? 0.0 : MODE == 2 ? q_line<false>(Q, cb, x, xb, j, i) : q_line(Q, cb, x, xb, j, i);
            be = (b[xl + i] - q) * im;
            al = i > 0 ? -Q.le[cl + i - 1] * im : 0.0;
            gi = Q.g[cl + i];
        }
        Rb[pos(i)] = be;
        Al[pos(i)] = al;
        Gl[pos(i)] = gi;
    }
    wave_sync();
    // forward: y -> A y + B over the lane's points, then across lanes
    double A = 1.0, B = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = lane * S + e;
        B = Al[p] * B + Rb[p];
        A = Al[p] * A;
    }
    scan_fwd(A, B);
    double yin = lineops::dpp0<lineops::kWaveShr1>(B);   // y at the last point of lane - 1 (0 for lane 0)
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = lane * S + e;
        yin = Al[p] * yin + Rb[p];
        Rb[p] = yin;
    }
    // backward: u_i = y_i - g_i u_{i+1}, composed from the top
    A = 1.0;
    B = 0.0;
#pragma unroll
    for (int e = E - 1; e >= 0; --e) {
        const int p = lane * S + e;
        B = -Gl[p] * B + Rb[p];
        A = -Gl[p] * A;
    }
    scan_bwd(A, B, lane);
    double uin = lineops::dpp0<lineops::kWaveShl1>(B);   // u at the first point of lane + 1 (0 for lane 63)
#pragma unroll
    for (int e = E - 1; e >= 0; --e) {
        const int p = lane * S + e;
        uin = Rb[p] - Gl[p] * uin;
        Rb[p] = uin;
    }
    wave_sync();
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int i = t * 64 + lane;
        if (i < nx) {
            if (MODE == 0)
                x[xl + i] += Rb[pos(i)];
            else
                x[xl + i] = Rb[pos(i)];
        }
    }
    wave_sync();   // the next line of this wave reuses the LDS rows
}

template <int E, int MODE>
__global__ __launch_bounds__(kB) void k_var_relax(Lines Q, const double *b, double *x, int np, int colour, int k0,
                                                  int ks)
{
    extern __shared__ double lds[];
    const int w = threadIdx.x >> 6;
    const long long wv = static_cast<long long>(blockIdx.x) * kRelaxWaves + w;
    const int nlc = (Q.ny - colour + 1) / 2;
    if (wv >= static_cast<long long>(nlc) * np) return;   // whole waves exit together
    const int pb = static_cast<int>(wv / nlc);
    const int j = colour + 2 * static_cast<int>(wv % nlc);
    const long long cb = static_cast<long long>(k0 + ks * pb) * Q.ny * Q.nx;
    const long long xb = static_cast<long long>(pb) * Q.ny * Q.nx;
    relax_line<E, MODE>(Q, b, x, cb, xb, j, lds + w * 3 * 64 * relax_stride(E));
}

// b_c = P^T (b - Q x) for np planes: coarse line J takes fine line 2J+1,
// ydn[2J+2] of line 2J+2 and yup[2J] of line 2J.
// swept: 0, the residual as defined; 1 (2), x is one half-sweep pair from
// zero with the even (odd) lines solved first.  Then the lines solved second
// have zero residual (each was solved exactly against its final neighbours)
// and a line solved first has r_j = -(V_{j-1}^T x_{j-1} + V_j x_{j+1}) (it
// solved L_j x_j = b_j while its neighbours were zero), equal to the residual
// as defined up to rounding and with far fewer reads.
__global__ void k_var_restrict2(Lines Q, const double *ydn, const double *yup, const double *b, const double *x,
                                double *bc, int np, int k0, int ks, int swept)
{
    const int nx = Q.nx, ny = Q.ny, nyc = ny / 2;
    const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= static_cast<long long>(np) * nyc * nx) return;
    const int i = static_cast<int>(e % nx);
    const int J = static_cast<int>((e / nx) % nyc);
    const int pb = static_cast<int>(e / nx / nyc);
    const long long cb = static_cast<long long>(k0 + ks * pb) * ny * nx, xb = static_cast<long long>(pb) * ny * nx;
    auto r = [&](int j) { return b[xb + static_cast<long long>(j) * nx + i] - q_line(Q, cb, x, xb, j, i); };
    auto rn = [&](int j) { return -q_line<false>(Q, cb, x, xb, j, i); };
    const double wu = yup[cb + static_cast<long long>(2 * J) * nx + i];
    const bool up = 2 * J + 2 < ny;
    double v;
    if (swept == 1) {
        v = wu * rn(2 * J);
        if (up) v += ydn[cb + static_cast<long long>(2 * J + 2) * nx + i] * rn(2 * J + 2);
    } else if (swept == 2) {
        v = rn(2 * J + 1);
    } else {
        v = r(2 * J + 1) + wu * r(2 * J);
        if (up) v += ydn[cb + static_cast<long long>(2 * J + 2) * nx + i] * r(2 * J + 2);
    }
    bc[e] = v;
}

// x += P x_c for np planes
__global__ void k_var_prolong2(const double *ydn, const double *yup, int nx, int ny, const double *xc, double *x,
                               int np, int k0, int ks)
{
    const int nyc = ny / 2;
    const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= static_cast<long long>(np) * ny * nx) return;
    const int i = static_cast<int>(e % nx);
    const int j = static_cast<int>((e / nx) % ny);
    const int pb = static_cast<int>(e / nx / ny);
    const long long cb = static_cast<long long>(k0 + ks * pb) * ny * nx;
    const long long xcb = static_cast<long long>(pb) * nyc * nx;
    double v;
    if (j % 2) {
        v = xc[xcb + static_cast<long long>(j / 2) * nx + i];
    } else {
        const long long c = cb + static_cast<long long>(j) * nx + i;
        v = 0.0;
        if (j / 2 - 1 >= 0) v += ydn[c] * xc[xcb + static_cast<long long>(j / 2 - 1) * nx + i];
        if (j / 2 < nyc) v += yup[c] * xc[xcb + static_cast<long long>(j / 2) * nx + i];
    }
    x[e] += v;
}

// The upward half of a 2D cycle without post-smoothing in one pass: from the
// coarsest level, v_l = x_l + P_l v_{l+1} with the per-point weights of
// k_var_prolong2 (the same arithmetic per point), then the 3D correction of
// k_var_correct3 (x_k += v_0 on plane k = k0 + ks*pb; assign: x_k = v_0).
// A block owns 64 columns and a run of 32 fine lines of one plane; each
// coarser level's window of lines is staged in LDS.
constexpr int kVcCols = 64, kVcRun = 32, kVcWin = 24;

struct VChainArgs {
    const double *x[kVcMaxLev];                        // bx2 of each 2D level
    const double *ydn[kVcMaxLev], *yup[kVcMaxLev];      // weights of each 2D level
    int ny2[kVcMaxLev];
    int nl, nx, np, k0, ks, assign;
    double *x3;                                         // 3D x of the level
    long long m;                                        // points per plane
};

struct VWin {
    int lo, hi;
};

__device__ inline VWin vc_coarser(VWin f, int nc)
{
    VWin c;
    c.lo = f.lo - 1 < 0 ? 0 : (f.lo - 1) >> 1;
    c.hi = f.hi >> 1;
    if (c.hi > nc - 1) c.hi = nc - 1;
    return c;
}

// P v_c at fine line jj, column col, window wc of the coarse level, with the
// fine line's weights wd (ydn) and wu (yup) at this column
__device__ inline double vc_prolong(const double *vc, VWin wc, int jj, int nyc, int col, double wd, double wu)
{
    if (jj & 1) return vc[((jj - 1) / 2 - wc.lo) * kVcCols + col];
    double v = 0.0;
    if (jj / 2 - 1 >= 0) v += wd * vc[(jj / 2 - 1 - wc.lo) * kVcCols + col];
    if (jj / 2 < nyc) v += wu * vc[(jj / 2 - wc.lo) * kVcCols + col];
    return v;
}

__global__ __launch_bounds__(256) void k_var_chain2(VChainArgs a)
{
    __shared__ double vs[2][kVcWin * kVcCols];
    const int nx = a.nx;
    const int ncol = (nx + kVcCols - 1) / kVcCols;
    const int nrun = (a.ny2[0] + kVcRun - 1) / kVcRun;
    int bid = blockIdx.x;
    const int ct = bid % ncol;
    bid /= ncol;
    const int rt = bid % nrun;
    const int pb = bid / nrun;
    const int col = threadIdx.x & (kVcCols - 1), row0 = threadIdx.x >> 6;   // 4 rows of 64
    const int i = ct * kVcCols + col;
    const bool in = i < nx;
    const int k = a.k0 + a.ks * pb;
    const VWin w0{rt * kVcRun, min(a.ny2[0], rt * kVcRun + kVcRun) - 1};
    auto win = [&](int l) {
        VWin wv = w0;
        for (int q = 0; q < l; ++q) wv = vc_coarser(wv, a.ny2[q + 1]);
        return wv;
    };
    // x of level l at line jj of plane pb (batch-packed), weights at plane k
    auto xrow = [&](int l, int jj) {
        return in ? a.x[l][(static_cast<long long>(pb) * a.ny2[l] + jj) * nx + i] : 0.0;
    };
    auto wc_of = [&](int l, int jj) { return (static_cast<long long>(k) * a.ny2[l] + jj) * nx + i; };
    // A level's rows of x and of its weights are all loaded before any of
    // them is used, so their latencies overlap (a loop that loaded and used
    // one row at a time waited a round trip per row).
    constexpr int kRows = kVcWin / 4, kRows0 = kVcRun / 4;   // rows per thread
    int cur = 0;
    for (int l = a.nl - 1; l >= 1; --l) {
        const VWin wl = win(l);
        double xr[kRows], wd[kRows], wu[kRows];
#pragma unroll
        for (int t = 0; t < kRows; ++t) {
            const int jj = wl.lo + row0 + 4 * t;
            xr[t] = wd[t] = wu[t] = 0.0;
            if (jj <= wl.hi) {
                xr[t] = xrow(l, jj);
                if (in && l < a.nl - 1) {
                    wd[t] = a.ydn[l][wc_of(l, jj)];
                    wu[t] = a.yup[l][wc_of(l, jj)];
                }
            }
        }
        if (l == a.nl - 1) {   // the coarsest level as it is
#pragma unroll
            for (int t = 0; t < kRows; ++t) {
                const int jj = wl.lo + row0 + 4 * t;
                if (jj <= wl.hi) vs[cur][(jj - wl.lo) * kVcCols + col] = xr[t];
            }
        } else {
            const VWin wc = win(l + 1);
#pragma unroll
            for (int t = 0; t < kRows; ++t) {
                const int jj = wl.lo + row0 + 4 * t;
                if (jj <= wl.hi) {
                    const double s = in ? vc_prolong(vs[cur], wc, jj, a.ny2[l + 1], col, wd[t], wu[t]) : 0.0;
                    vs[cur ^ 1][(jj - wl.lo) * kVcCols + col] = xr[t] + s;
                }
            }
            cur ^= 1;
        }
        __syncthreads();
    }
    if (!in) return;   // after the last barrier
    const VWin wc = win(1);
    double xr[kRows0], wd[kRows0], wu[kRows0], old[kRows0];
#pragma unroll
    for (int t = 0; t < kRows0; ++t) {
        const int jj = w0.lo + row0 + 4 * t;
        xr[t] = wd[t] = wu[t] = old[t] = 0.0;
        if (jj <= w0.hi) {
            xr[t] = xrow(0, jj);
            wd[t] = a.ydn[0][wc_of(0, jj)];
            wu[t] = a.yup[0][wc_of(0, jj)];
            if (!a.assign) old[t] = a.x3[k * a.m + static_cast<long long>(jj) * nx + i];
        }
    }
#pragma unroll
    for (int t = 0; t < kRows0; ++t) {
        const int jj = w0.lo + row0 + 4 * t;
        if (jj > w0.hi) break;
        const double v = xr[t] + vc_prolong(vs[cur], wc, jj, a.ny2[1], col, wd[t], wu[t]);
        double *dst = a.x3 + k * a.m + static_cast<long long>(jj) * nx + i;
        if (a.assign)
            *dst = v;
        else
            *dst = old[t] + v;
    }
}

struct Planes {                   // a 3D level
    BlockOp op;
    int nz;
};

// (A_l x)_k at point p of plane k: C_k x_k + U_{k-1}^T x_{k-1} + U_k x_{k+1}
// (OWN false: without C_k x_k, for a plane whose x is still zero)
template <bool OWN = true>
__device__ inline double a_plane(const Planes &A, const double *x, int k, int i, int j)
{
    // loads at clamped indices, all in flight together; terms past an edge
    // skipped afterwards, in the stencil's order (as in q_line)
    const BlockOp &o = A.op;
    const int nx = o.nx, ny = o.ny;
    const long long m = static_cast<long long>(nx) * ny;
    const long long p = k * m + static_cast<long long>(j) * nx + i;
    const bool hw = i > 0, he = i + 1 < nx, hs = j > 0, hn = j + 1 < ny, hd = k > 0, hu = k + 1 < A.nz;
    const int dw = hw ? 1 : 0, de = he ? 1 : 0;
    const long long ds = hs ? nx : 0, dn = hn ? nx : 0;
    double v = 0.0;
    if constexpr (OWN) {
        const double c0 = o.cc[p], cw = o.ce[p - dw], ce = o.ce[p], cs = o.cn[p - ds], cn = o.cn[p];
        const double x0 = x[p], xw = x[p - dw], xe = x[p + de], xs = x[p - ds], xn = x[p + dn];
        v = c0 * x0;
        if (hw) v += cw * xw;
        if (he) v += ce * xe;
        if (hs) v += cs * xs;
        if (hn) v += cn * xn;
    }
    // U_{k-1}^T: entries of the rows of plane k-1 that reach p
    const long long d = p - (hd ? m : 0);
    const double dc = o.uc[d], de_ = o.ue[d - dw], dw_ = o.uw[d + de], ds_ = o.un[d - ds], dn_ = o.us[d + dn];
    const double yd0 = x[d], ydw = x[d - dw], yde = x[d + de], yds = x[d - ds], ydn = x[d + dn];
    const long long u = p + (hu ? m : 0);
    const double uc = o.uc[p], ue = o.ue[p], uw = o.uw[p], un = o.un[p], us = o.us[p];
    const double yu0 = x[u], yue = x[u + de], yuw = x[u - dw], yun = x[u + dn], yus = x[u - ds];
    if (hd) {
        v += dc * yd0;
        if (hw) v += de_ * ydw;
        if (he) v += dw_ * yde;
        if (hs) v += ds_ * yds;
        if (hn) v += dn_ * ydn;
    }
    if (hu) {
        v += uc * yu0;
        if (he) v += ue * yue;
        if (hw) v += uw * yuw;
        if (hn) v += un * yun;
        if (hs) v += us * yus;
    }
    return v;
}

// residual of the planes of one colour into the 2D batch buffer; OWN false:
// the colour's own planes of x are zero (not read)
template <bool OWN>
__global__ void k_var_resid3(Planes A, const double *b, const double *x, int colour, double *r)
{
    const int nx = A.op.nx, ny = A.op.ny;
    const long long m = static_cast<long long>(nx) * ny;
    const int npl = (A.nz - colour + 1) / 2;
    const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= npl * m) return;
    const int pb = static_cast<int>(e / m);
    const int k = colour + 2 * pb;
    const int i = static_cast<int>(e % nx), j = static_cast<int>((e % m) / nx);
    r[e] = b[k * m + e % m] - a_plane<OWN>(A, x, k, i, j);
}

// the planes of one colour of b into the 2D batch buffer (the residual of a zero x)
__global__ void k_var_gather3(const double *b, long long m, int nz, int colour, double *r)
{
    const int npl = (nz - colour + 1) / 2;
    const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= npl * m) return;
    r[e] = b[(colour + 2 * (e / m)) * m + e % m];
}

// x_k += y_pb for the planes of one colour (assign: x_k = y_pb)
__global__ void k_var_correct3(double *x, const double *y, long long m, int nz, int colour, int assign)
{
    const int npl = (nz - colour + 1) / 2;
    const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= npl * m) return;
    const int k = colour + 2 * static_cast<int>(e / m);
    if (assign)
        x[k * m + e % m] = y[e];
    else
        x[k * m + e % m] += y[e];
}

// b_c = P^T (b - A x): coarse plane K takes fine plane 2K+1, wup of plane 2K
// and wdn of plane 2K+2.  A thread owns one point of the plane and marches
// through kRestrictRun coarse planes, so the residual of fine plane 2K+2 also
// serves coarse plane K+1.
constexpr int kRestrictRun = 8;

__global__ void k_var_restrict3(Planes A, const double *wdn, const double *wup, const double *b, const double *x,
                                double *bc)
{
    const int nx = A.op.nx, ny = A.op.ny, nzc = A.nz / 2;
    const long long m = static_cast<long long>(nx) * ny;
    const long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= m) return;
    const int K0 = static_cast<int>(blockIdx.y) * kRestrictRun, K1 = min(K0 + kRestrictRun, nzc);
    const int i = static_cast<int>(p % nx), j = static_cast<int>(p / nx);
    auto r = [&](int k) { return b[k * m + p] - a_plane(A, x, k, i, j); };
    double r0 = r(2 * K0);
    for (int K = K0; K < K1; ++K) {
        const double r1 = r(2 * K + 1);
        double v = r1 + wup[2 * K * m + p] * r0;
        double r2 = 0.0;
        if (2 * K + 2 < A.nz) {
            r2 = r(2 * K + 2);
            v += wdn[(2 * K + 2) * m + p] * r2;
        }
        bc[K * m + p] = v;
        r0 = r2;
    }
}

__global__ void k_var_prolong3(const double *wdn, const double *wup, long long m, int nz, const double *xc, double *x)
{
    const int nzc = nz / 2;
    const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nz * m) return;
    const int k = static_cast<int>(e / m);
    const long long p = e % m;
    double v;
    if (k % 2) {
        v = xc[(k / 2) * m + p];
    } else {
        v = 0.0;
        if (k / 2 - 1 >= 0) v += wdn[e] * xc[(k / 2 - 1) * m + p];
        if (k / 2 < nzc) v += wup[e] * xc[(k / 2) * m + p];
    }
    x[e] += v;
}

__global__ void k_var_copy(const double *src, double *dst, long long n)
{
    const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < n) dst[e] = src[e];
}

// ---------------------------------------------------------------------------
// Krylov passes with the fine operator (the same partial-sum layout and
// fixed reduction grid as the constant-coefficient passes)
// ---------------------------------------------------------------------------

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ inline double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) s += lds[i];
    __syncthreads();
    return s;
}

// (A v)_c of the fine operator with v given pointwise by vf(c)
template <typename F>
__device__ inline double a_fine(const Planes &A, F vf, long long c)
{
    const BlockOp &o = A.op;
    const int nx = o.nx, ny = o.ny;
    const long long m = static_cast<long long>(nx) * ny;
    const int i = static_cast<int>(c % nx), j = static_cast<int>((c / nx) % ny), k = static_cast<int>(c / m);
    double v = o.cc[c] * vf(c);
    if (i > 0) v += o.ce[c - 1] * vf(c - 1);
    if (i + 1 < nx) v += o.ce[c] * vf(c + 1);
    if (j > 0) v += o.cn[c - nx] * vf(c - nx);
    if (j + 1 < ny) v += o.cn[c] * vf(c + nx);
    if (k > 0) v += o.uc[c - m] * vf(c - m);
    if (k + 1 < A.nz) v += o.uc[c] * vf(c + m);
    return v;
}

__global__ __launch_bounds__(kB) void k_var_matvec(Planes A, const double *x, double *y, long long n, long long ld)
{
    const int r = blockIdx.y;
    const double *xr = x + r * ld;
    double *yr = y + r * ld;
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(gridDim.x) * blockDim.x)
        yr[c] = a_fine(A, [&](long long q) { return xr[q]; }, c);
}

__global__ __launch_bounds__(kB) void k_var_init_resid(Planes A, const double *b, const double *x, double *r,
                                                       int x_zero, long long n, double *partials)
{
    __shared__ double lds[kB / 64];
    double rr = 0.0, bb = 0.0;
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(gridDim.x) * blockDim.x) {
        const double bv = b[c];
        const double rv = x_zero ? bv : bv - a_fine(A, [&](long long q) { return x[q]; }, c);
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

__global__ __launch_bounds__(kB) void k_var_update_p_q(Planes A, const double *s, const double *p_old, double *p_new,
                                                       double *q, const KScalars *sc, long long n, double *partials)
{
    __shared__ double lds[kB / 64];
    const double beta = sc->beta;
    auto pv = [&](long long c) { return beta == 0.0 ? s[c] : s[c] + beta * p_old[c]; };
    double pq = 0.0;
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(gridDim.x) * blockDim.x) {
        const double p0 = pv(c);
        const double qv = a_fine(A, pv, c);
        p_new[c] = p0;
        q[c] = qv;
        pq += p0 * qv;
    }
    pq = block_sum(pq, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = pq;
}

// The same update with p staged per plane in an LDS tile (64 x 8 points and
// their in-plane halo) while each block marches through a run of planes, so
// every p value is formed once instead of once per neighbour that reads it.
// q adds the operator's terms in a_fine's order (bitwise a_fine's q); the
// partial (p, q) is per block, at most kRedBlocks blocks (block 0 zeroes the
// unused slots).
constexpr int kPTX = 64, kPTY = 8, kPThreads = kPTX * kPTY;

__global__ __launch_bounds__(kPThreads) void k_var_update_p_q_tiled(Planes A, const double *s, const double *p_old,
                                                                    double *p_new, double *q, const KScalars *sc,
                                                                    int kchunk, double *partials)
{
    __shared__ double tile[(kPTY + 2) * (kPTX + 2)];
    __shared__ double lds[kPThreads / 64];
    const BlockOp &o = A.op;
    const double beta = sc->beta;
    const int nx = o.nx, ny = o.ny, nz = A.nz;
    const int tx = threadIdx.x % kPTX, ty = threadIdx.x / kPTX;
    const int i = blockIdx.x * kPTX + tx, j = blockIdx.y * kPTY + ty;
    const bool in = i < nx && j < ny;
    const long long m = static_cast<long long>(nx) * ny;
    const long long c2 = static_cast<long long>(j) * nx + i;
    const int k0 = blockIdx.z * kchunk, k1 = min(nz, k0 + kchunk);
    auto pv = [&](long long c) { return beta == 0.0 ? s[c] : s[c] + beta * p_old[c]; };
    // halo cell of this thread: the rows above and below the tile, then the
    // columns left and right of it (no corners: the in-plane stencil has none)
    const int t = threadIdx.x;
    int hy = -1, hx = -1;
    if (t < kPTX) {
        hy = 0; hx = t + 1;
    } else if (t < 2 * kPTX) {
        hy = kPTY + 1; hx = t - kPTX + 1;
    } else if (t < 2 * kPTX + kPTY) {
        hy = t - 2 * kPTX + 1; hx = 0;
    } else if (t < 2 * kPTX + 2 * kPTY) {
        hy = t - 2 * kPTX - kPTY + 1; hx = kPTX + 1;
    }
    const int hi = blockIdx.x * kPTX + hx - 1, hj = blockIdx.y * kPTY + hy - 1;
    const bool hin = hy >= 0 && hi >= 0 && hi < nx && hj >= 0 && hj < ny;
    const long long hc2 = static_cast<long long>(hj) * nx + hi;
    const bool hw = i > 0, he = i + 1 < nx, hs = j > 0, hn = j + 1 < ny;
    const long long dw = hw ? 1 : 0, ds = hs ? nx : 0;
    double pm = (in && k0 > 0 && k0 < nz) ? pv((k0 - 1) * m + c2) : 0.0;
    double pc = (in && k0 < nz) ? pv(k0 * m + c2) : 0.0;
    double pq = 0.0;
    constexpr int RW = kPTX + 2;
    for (int k = k0; k < k1; ++k) {
        const double pn = (in && k + 1 < nz) ? pv((k + 1) * m + c2) : 0.0;
        tile[(ty + 1) * RW + tx + 1] = pc;
        if (hy >= 0) tile[hy * RW + hx] = hin ? pv(k * m + hc2) : 0.0;
        __syncthreads();
        if (in) {
            const long long c = k * m + c2, dd = k > 0 ? m : 0;
            const int cc = (ty + 1) * RW + tx + 1;
            const double c0 = o.cc[c], cw = o.ce[c - dw], ce = o.ce[c], cs = o.cn[c - ds], cn = o.cn[c],
                         cd = o.uc[c - dd], cu = o.uc[c];
            double v = c0 * pc;
            if (hw) v += cw * tile[cc - 1];
            if (he) v += ce * tile[cc + 1];
            if (hs) v += cs * tile[cc - RW];
            if (hn) v += cn * tile[cc + RW];
            if (k > 0) v += cd * pm;
            if (k + 1 < nz) v += cu * pn;
            p_new[c] = pc;
            q[c] = v;
            pq += pc * v;
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

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

int levels_of(int n)
{
    int L = 1;
    while (n > 1) {
        n /= 2;
        ++L;
    }
    return L;
}

// Offsets of the hierarchy inside the workspace (from byte 0)
void layout(VarHier &H)
{
    size_t off = 0;
    auto take = [&](size_t count) {
        const size_t r = off;
        off = al(off + count * 8);
        return r;
    };
    const size_t m = static_cast<size_t>(H.nx) * H.ny;
    H.ny2.clear();
    for (int v = H.ny;; v /= 2) {
        H.ny2.push_back(v);
        if (v == 1) break;
    }
    H.lev.assign(levels_of(H.nz), VarLevel3{});
    int nzl = H.nz;
    for (size_t l = 0; l < H.lev.size(); ++l, nzl /= 2) {
        VarLevel3 &L = H.lev[l];
        L.nz = nzl;
        const size_t n = m * nzl;
        L.cc = take(n);
        L.ce = take(n);
        L.cn = take(n);
        L.uc = take(n);
        L.ue = take(n);
        L.uw = take(n);
        L.un = take(n);
        L.us = take(n);
        L.wdn = take(n);
        L.wup = take(n);
        L.x = l > 0 ? take(n) : 0;
        L.b = l > 0 ? take(n) : 0;
        for (int v : H.ny2) {
            const size_t n2 = static_cast<size_t>(nzl) * v * H.nx;
            L.lc.push_back(take(n2));
            L.le.push_back(take(n2));
            L.vc.push_back(take(n2));
            L.ve.push_back(take(n2));
            L.vw.push_back(take(n2));
            L.ydn.push_back(take(n2));
            L.yup.push_back(take(n2));
            L.invm.push_back(take(n2));
            L.g.push_back(take(n2));
        }
    }
    // batch buffers: the planes of one colour of the finest level
    const size_t npmax = static_cast<size_t>((H.nz + 1) / 2);
    H.bx2.clear();
    H.bb2.clear();
    for (int v : H.ny2) {
        H.bx2.push_back(take(npmax * v * H.nx));
        H.bb2.push_back(take(npmax * v * H.nx));
    }
    H.total = off;
}

BlockOp block_op(const VarHier &H, const VarLevel3 &L)
{
    return BlockOp{H.at<double>(L.cc), H.at<double>(L.ce), H.at<double>(L.cn), H.at<double>(L.uc),
                   H.at<double>(L.ue), H.at<double>(L.uw), H.at<double>(L.un), H.at<double>(L.us),
                   H.nx,                H.ny};
}

Planes planes_of(const VarHier &H, int l) { return Planes{block_op(H, H.lev[l]), H.lev[l].nz}; }

Lines lines_of(const VarHier &H, int l, int l2)
{
    const VarLevel3 &L = H.lev[l];
    return Lines{H.at<double>(L.lc[l2]), H.at<double>(L.le[l2]),   H.at<double>(L.vc[l2]), H.at<double>(L.ve[l2]),
                 H.at<double>(L.vw[l2]), H.at<double>(L.invm[l2]), H.at<double>(L.g[l2]),  H.nx,
                 H.ny2[l2]};
}

void build(VarHier &H, const double *diag, const double *ax, const double *ay, const double *az, hipStream_t st)
{
    const long long m = static_cast<long long>(H.nx) * H.ny;
    {
        VarLevel3 &L = H.lev[0];
        hipLaunchKernelGGL(k_var_fine, dim3(nblk(m * H.nz, kB)), dim3(kB), 0, st, diag, ax, ay, az, H.nx, H.ny, H.nz,
                           H.at<double>(L.cc), H.at<double>(L.ce), H.at<double>(L.cn), H.at<double>(L.uc),
                           H.at<double>(L.ue), H.at<double>(L.uw), H.at<double>(L.un), H.at<double>(L.us));
    }
    for (size_t l = 0; l + 1 < H.lev.size(); ++l) {
        VarLevel3 &F = H.lev[l], &Cl = H.lev[l + 1];
        const BlockOp o = block_op(H, F);
        hipLaunchKernelGGL(k_var_weights, dim3(nblk(m * F.nz, kB)), dim3(kB), 0, st, o.uc, o.ue, o.uw, o.un, o.us,
                           H.nx, H.ny, F.nz, 1, H.interp, H.at<double>(F.wdn), H.at<double>(F.wup));
        hipLaunchKernelGGL(k_var_galerkin, dim3(nblk(m * Cl.nz, kB)), dim3(kB), 0, st, o, H.at<double>(F.wdn),
                           H.at<double>(F.wup), F.nz, 1, H.at<double>(Cl.cc), H.at<double>(Cl.ce), H.at<double>(Cl.cn),
                           H.at<double>(Cl.uc), H.at<double>(Cl.ue), H.at<double>(Cl.uw), H.at<double>(Cl.un),
                           H.at<double>(Cl.us));
    }
    // 2D hierarchies of every plane of every 3D level.  A plane's 2D level is
    // a block-tridiagonal operator over lines (blocks of nx points: the line
    // blocks L_j in the centre/east slots, the couplings V_j in the
    // centre/east/west slots); the planes of a 3D level are stacked.
    for (size_t l = 0; l < H.lev.size(); ++l) {
        VarLevel3 &L = H.lev[l];
        const long long n = m * L.nz;
        hipLaunchKernelGGL(k_var_plane0, dim3(nblk(n, kB)), dim3(kB), 0, st, H.at<double>(L.cc), H.at<double>(L.ce),
                           H.at<double>(L.cn), n, H.at<double>(L.lc[0]), H.at<double>(L.le[0]), H.at<double>(L.vc[0]),
                           H.at<double>(L.ve[0]), H.at<double>(L.vw[0]));
        for (size_t l2 = 0; l2 < H.ny2.size(); ++l2) {
            const int nyl = H.ny2[l2];
            const long long nlines = static_cast<long long>(L.nz) * nyl;
            hipLaunchKernelGGL(k_var_factor, dim3(nblk(nlines, 64)), dim3(64), 0, st, H.at<double>(L.lc[l2]),
                               H.at<double>(L.le[l2]), nlines, H.nx, H.at<double>(L.invm[l2]), H.at<double>(L.g[l2]));
            if (l2 + 1 == H.ny2.size()) break;
            const int nyc = H.ny2[l2 + 1];
            const BlockOp o{H.at<double>(L.lc[l2]), H.at<double>(L.le[l2]), nullptr, H.at<double>(L.vc[l2]),
                            H.at<double>(L.ve[l2]), H.at<double>(L.vw[l2]), nullptr,   nullptr, H.nx, 1};
            hipLaunchKernelGGL(k_var_weights, dim3(nblk(nlines * H.nx, kB)), dim3(kB), 0, st, o.uc, o.ue, o.uw,
                               nullptr, nullptr, H.nx, 1, nyl, L.nz, H.interp, H.at<double>(L.ydn[l2]),
                               H.at<double>(L.yup[l2]));
            hipLaunchKernelGGL(k_var_galerkin, dim3(nblk(static_cast<long long>(L.nz) * nyc * H.nx, kB)), dim3(kB), 0,
                               st, o, H.at<double>(L.ydn[l2]), H.at<double>(L.yup[l2]), nyl, L.nz,
                               H.at<double>(L.lc[l2 + 1]), H.at<double>(L.le[l2 + 1]), nullptr,
                               H.at<double>(L.vc[l2 + 1]), H.at<double>(L.ve[l2 + 1]), H.at<double>(L.vw[l2 + 1]),
                               nullptr, nullptr);
        }
    }
}

// ---------------------------------------------------------------------------
// V-cycle schedule (host)
// ---------------------------------------------------------------------------

template <int MODE>
void relax_mode(const VarHier &H, int l, int l2, int np, int colour, int k0, int ks, hipStream_t st)
{
    const Lines Q = lines_of(H, l, l2);
    const long long waves = static_cast<long long>((Q.ny - colour + 1) / 2) * np;
    if (waves <= 0) return;
    const dim3 grid(nblk(waves, kRelaxWaves)), block(kB);
    const double *b = H.at<double>(H.bb2[l2]);
    double *x = H.at<double>(H.bx2[l2]);
    const int E = (H.nx + 63) / 64;
    const size_t lds = static_cast<size_t>(kRelaxWaves) * 3 * 64 * relax_stride(E) * sizeof(double);
    switch (E) {
    case 1: hipLaunchKernelGGL((k_var_relax<1, MODE>), grid, block, lds, st, Q, b, x, np, colour, k0, ks); break;
    case 2: hipLaunchKernelGGL((k_var_relax<2, MODE>), grid, block, lds, st, Q, b, x, np, colour, k0, ks); break;
    case 3: hipLaunchKernelGGL((k_var_relax<3, MODE>), grid, block, lds, st, Q, b, x, np, colour, k0, ks); break;
    case 4: hipLaunchKernelGGL((k_var_relax<4, MODE>), grid, block, lds, st, Q, b, x, np, colour, k0, ks); break;
    case 5: hipLaunchKernelGGL((k_var_relax<5, MODE>), grid, block, lds, st, Q, b, x, np, colour, k0, ks); break;
    case 6: hipLaunchKernelGGL((k_var_relax<6, MODE>), grid, block, lds, st, Q, b, x, np, colour, k0, ks); break;
    case 7: hipLaunchKernelGGL((k_var_relax<7, MODE>), grid, block, lds, st, Q, b, x, np, colour, k0, ks); break;
    default: hipLaunchKernelGGL((k_var_relax<8, MODE>), grid, block, lds, st, Q, b, x, np, colour, k0, ks); break;
    }
}

// mode: 0 correction; 1, 2 the two half-sweeps from a zero x (see relax_line)
void relax(const VarHier &H, int l, int l2, int np, int colour, int k0, int ks, hipStream_t st, int mode = 0)
{
    if (mode == 1)
        relax_mode<1>(H, l, l2, np, colour, k0, ks, st);
    else if (mode == 2)
        relax_mode<2>(H, l, l2, np, colour, k0, ks, st);
    else
        relax_mode<0>(H, l, l2, np, colour, k0, ks, st);
}

// the chain replaces the per-level prolongations when nothing follows them
bool chained(const VarHier &H) { return H.ipost == 0 && H.ny2.size() > 1 && H.ny2.size() <= kVcMaxLev; }

// One 2D V-cycle, for np planes at once (plane pb of the batch is plane
// k0 + ks*pb of 3D level l): right-hand sides in bb2[l2], result in bx2[l2].
// down_only: the downward half only (pre-smoothing, restriction, coarsest
// solve); the prolongations are left to chain_up.
void vcycle2(const VarHier &H, int l, int l2, int np, int k0, int ks, hipStream_t st, bool down_only = false)
{
    const int ny = H.ny2[l2];
    const long long n2 = static_cast<long long>(np) * ny * H.nx;
    double *x = H.at<double>(H.bx2[l2]);
    if (ny == 1) {   // coarsest 2D level: one exact line solve
        relax(H, l, l2, np, 0, k0, ks, st, 1);
        return;
    }
    // x starts at zero: the first sweep assigns it (without pre-smoothing
    // the prolongation adds to a zeroed x)
    if (H.ipre == 0) launch_fill(x, 0.0, static_cast<size_t>(n2), st);
    const int first = H.order == 0 ? 0 : 1, second = 1 - first;
    for (int t = 0; t < H.ipre; ++t) {
        relax(H, l, l2, np, first, k0, ks, st, t == 0 ? 1 : 0);
        relax(H, l, l2, np, second, k0, ks, st, t == 0 ? 2 : 0);
    }
    const VarLevel3 &L = H.lev[l];
    const Lines Q = lines_of(H, l, l2);
    const long long nc = static_cast<long long>(np) * H.ny2[l2 + 1] * H.nx;
    // one pre-smoothing pair from zero: the restriction needs the lines solved first only
    const int swept = H.ipre == 1 ? (first == 0 ? 1 : 2) : 0;
    hipLaunchKernelGGL(k_var_restrict2, dim3(nblk(nc, kB)), dim3(kB), 0, st, Q, H.at<double>(L.ydn[l2]),
                       H.at<double>(L.yup[l2]), H.at<double>(H.bb2[l2]), x, H.at<double>(H.bb2[l2 + 1]), np, k0, ks,
                       swept);
    vcycle2(H, l, l2 + 1, np, k0, ks, st, down_only);
    if (down_only) return;
    hipLaunchKernelGGL(k_var_prolong2, dim3(nblk(n2, kB)), dim3(kB), 0, st, H.at<double>(L.ydn[l2]),
                       H.at<double>(L.yup[l2]), H.nx, ny, H.at<double>(H.bx2[l2 + 1]), x, np, k0, ks);
    for (int t = 0; t < H.ipost; ++t) {
        relax(H, l, l2, np, second, k0, ks, st);
        relax(H, l, l2, np, first, k0, ks, st);
    }
}

// The upward half of the 2D cycles of np planes (after vcycle2 down_only)
// and their 3D correction: x_k += v_0 (assign: x_k = v_0), k = k0 + ks*pb.
void chain_up(const VarHier &H, int l, int np, int k0, int ks, double *x, int assign, hipStream_t st)
{
    const VarLevel3 &L = H.lev[l];
    VChainArgs a{};
    a.nl = static_cast<int>(H.ny2.size());
    for (int l2 = 0; l2 < a.nl; ++l2) {
        a.x[l2] = H.at<double>(H.bx2[l2]);
        a.ny2[l2] = H.ny2[l2];
        if (l2 + 1 < a.nl) {
            a.ydn[l2] = H.at<double>(L.ydn[l2]);
            a.yup[l2] = H.at<double>(L.yup[l2]);
        }
    }
    a.nx = H.nx;
    a.np = np;
    a.k0 = k0;
    a.ks = ks;
    a.assign = assign;
    a.x3 = x;
    a.m = static_cast<long long>(H.nx) * H.ny;
    const int ncol = (H.nx + kVcCols - 1) / kVcCols, nrun = (H.ny2[0] + kVcRun - 1) / kVcRun;
    hipLaunchKernelGGL(k_var_chain2, dim3(static_cast<unsigned>(ncol) * nrun * np), dim3(256), 0, st, a);
}

// zebra half-sweep over the planes of one colour: x_k += V2_k((b - A x)_k).
// zero: 0 general; 1 x is zero (its planes are not read: the right-hand sides
// are b); 2 the colour's own planes of x are zero (not read).  With zero > 0
// the colour's planes of x are assigned, so x needs no clearing beforehand.
void sweep3(const VarHier &H, int l, int colour, const double *b, double *x, hipStream_t st, int zero = 0)
{
    const VarLevel3 &L = H.lev[l];
    const int np = (L.nz - colour + 1) / 2;
    if (np <= 0) return;
    const long long m = static_cast<long long>(H.nx) * H.ny;
    double *r = H.at<double>(H.bb2[0]);
    const dim3 grid(nblk(np * m, kB));
    if (zero == 1)
        hipLaunchKernelGGL(k_var_gather3, grid, dim3(kB), 0, st, b, m, L.nz, colour, r);
    else if (zero == 2)
        hipLaunchKernelGGL(k_var_resid3<false>, grid, dim3(kB), 0, st, planes_of(H, l), b, x, colour, r);
    else
        hipLaunchKernelGGL(k_var_resid3<true>, grid, dim3(kB), 0, st, planes_of(H, l), b, x, colour, r);
    const int assign = zero > 0 ? 1 : 0;
    if (chained(H)) {
        vcycle2(H, l, 0, np, colour, 2, st, true);
        chain_up(H, l, np, colour, 2, x, assign, st);
        return;
    }
    vcycle2(H, l, 0, np, colour, 2, st);
    hipLaunchKernelGGL(k_var_correct3, grid, dim3(kB), 0, st, x, H.at<double>(H.bx2[0]), m, L.nz, colour, assign);
}

void vcycle3(const VarHier &H, int l, const double *b, double *x, hipStream_t st)
{
    const VarLevel3 &L = H.lev[l];
    const long long m = static_cast<long long>(H.nx) * H.ny;
    if (L.nz == 1) {   // coarsest 3D level: one plane solve
        hipLaunchKernelGGL(k_var_copy, dim3(nblk(m, kB)), dim3(kB), 0, st, b, H.at<double>(H.bb2[0]), m);
        if (chained(H)) {
            vcycle2(H, l, 0, 1, 0, 1, st, true);
            chain_up(H, l, 1, 0, 1, x, 1, st);
            return;
        }
        vcycle2(H, l, 0, 1, 0, 1, st);
        hipLaunchKernelGGL(k_var_copy, dim3(nblk(m, kB)), dim3(kB), 0, st, H.at<double>(H.bx2[0]), x, m);
        return;
    }
    // x starts at zero: the first sweep assigns every plane (without
    // pre-smoothing the restriction reads a cleared x)
    if (H.pre == 0) launch_fill(x, 0.0, static_cast<size_t>(m * L.nz), st);
    const int first = H.order == 0 ? 0 : 1, second = 1 - first;
    for (int t = 0; t < H.pre; ++t) {
        sweep3(H, l, first, b, x, st, t == 0 ? 1 : 0);
        sweep3(H, l, second, b, x, st, t == 0 ? 2 : 0);
    }
    const VarLevel3 &C = H.lev[l + 1];
    hipLaunchKernelGGL(k_var_restrict3, dim3(nblk(m, kB), (C.nz + kRestrictRun - 1) / kRestrictRun), dim3(kB), 0,
                       st, planes_of(H, l),
                       H.at<double>(L.wdn), H.at<double>(L.wup), b, x, H.at<double>(C.b));
    vcycle3(H, l + 1, H.at<double>(C.b), H.at<double>(C.x), st);
    hipLaunchKernelGGL(k_var_prolong3, dim3(nblk(m * L.nz, kB)), dim3(kB), 0, st, H.at<double>(L.wdn),
                       H.at<double>(L.wup), m, L.nz, H.at<double>(C.x), x);
    for (int t = 0; t < H.post; ++t) {
        sweep3(H, l, second, b, x, st);
        sweep3(H, l, first, b, x, st);
    }
}

}  // namespace

size_t var_workspace_bytes(int nx, int ny, int nz)
{
    VarHier H{};
    H.nx = nx;
    H.ny = ny;
    H.nz = nz;
    layout(H);
    return H.total;
}

VarHier *var_create(int nx, int ny, int nz, const smg_opts *o, int interp, char *ws, const double *diag,
                    const double *ax, const double *ay, const double *az, hipStream_t st)
{
    VarHier *H = new (std::nothrow) VarHier();
    if (!H) return nullptr;
    H->nx = nx;
    H->ny = ny;
    H->nz = nz;
    H->N = static_cast<size_t>(nx) * ny * nz;
    H->pre = o->pre;
    H->post = o->post;
    H->ipre = o->inner_pre < 0 ? o->pre : o->inner_pre;
    H->ipost = o->inner_post < 0 ? o->post : o->inner_post;
    H->order = o->order;
    H->interp = interp;
    H->ws = ws;
    layout(*H);
    build(*H, diag, ax, ay, az, st);
    return H;
}

void var_destroy(VarHier *H) { delete H; }

void var_vcycle(VarHier *H, const double *r, double *s, int nrhs, long long ld, hipStream_t st)
{
    for (int c = 0; c < nrhs; ++c) vcycle3(*H, 0, r + c * ld, s + c * ld, st);
}

void var_matvec(VarHier *H, const double *x, double *y, int nrhs, long long ld, hipStream_t st)
{
    const long long n = static_cast<long long>(H->N);
    const unsigned gx = std::min<unsigned>(nblk(n, kB), 2048);
    hipLaunchKernelGGL(k_var_matvec, dim3(gx, nrhs), dim3(kB), 0, st, planes_of(*H, 0), x, y, n, ld);
}

void var_init_resid(VarHier *H, const double *b, const double *x, double *r, int x_zero, double *partials,
                    hipStream_t st)
{
    hipLaunchKernelGGL(k_var_init_resid, dim3(kRedBlocks), dim3(kB), 0, st, planes_of(*H, 0), b, x, r, x_zero,
                       static_cast<long long>(H->N), partials);
}

void var_update_p_q(VarHier *H, const double *s, const double *p_old, double *p_new, double *q, const KScalars *sc,
                    double *partials, hipStream_t st)
{
    const int gx = (H->nx + kPTX - 1) / kPTX, gy = (H->ny + kPTY - 1) / kPTY;
    if (static_cast<long long>(gx) * gy <= kRedBlocks) {   // planes tiled, runs of planes per block
        const int gz0 = std::max(1, std::min(H->nz, kRedBlocks / (gx * gy)));
        const int kchunk = (H->nz + gz0 - 1) / gz0, gz = (H->nz + kchunk - 1) / kchunk;
        hipLaunchKernelGGL(k_var_update_p_q_tiled, dim3(gx, gy, gz), dim3(kPThreads), 0, st, planes_of(*H, 0), s,
                           p_old, p_new, q, sc, kchunk, partials);
        return;
    }
    hipLaunchKernelGGL(k_var_update_p_q, dim3(kRedBlocks), dim3(kB), 0, st, planes_of(*H, 0), s, p_old, p_new, q, sc,
                       static_cast<long long>(H->N), partials);
}

int var_levels(const VarHier *H, int *nlev3, int *nlev2)
{
    *nlev3 = static_cast<int>(H->lev.size());
    *nlev2 = static_cast<int>(H->ny2.size());
    return SMG_OK;
}

// copies of the stored operators: 3D level l (8 arrays of nz_l*nx*ny: cc, ce,
// cn, uc, ue, uw, un, us) or the 2D level l2 of every plane of it (5 arrays of
// nz_l*ny_l2*nx: lc, le, vc, ve, vw), into a device buffer
int var_export(const VarHier *H, int l, int l2, double *out, hipStream_t st)
{
    if (l < 0 || l >= static_cast<int>(H->lev.size()) || l2 < -1 || l2 >= static_cast<int>(H->ny2.size()))
        return SMG_EINVAL;
    const VarLevel3 &L = H->lev[l];
    std::vector<size_t> src;
    size_t n;
    if (l2 < 0) {
        src = {L.cc, L.ce, L.cn, L.uc, L.ue, L.uw, L.un, L.us};
        n = static_cast<size_t>(L.nz) * H->nx * H->ny;
    } else {
        src = {L.lc[l2], L.le[l2], L.vc[l2], L.ve[l2], L.vw[l2]};
        n = static_cast<size_t>(L.nz) * H->ny2[l2] * H->nx;
    }
    for (size_t a = 0; a < src.size(); ++a)
        if (hipMemcpyAsync(out + a * n, H->at<double>(src[a]), n * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return SMG_EHIP;
    return SMG_OK;
}

}  // namespace smg
