// Host side of the SMG library: setup, V-cycle schedule, Krylov loops, C ABI.
//
// Setup follows the Section 3 reading of SMG: z-semicoarsening with Galerkin
// coarse operators.  Because the prolongation acts on the plane index only,
// every level stays block-tridiagonal with blocks in span{T2, I}, so a level
// is four scalars per plane (C_K = ca*T2 + cb*I, U_K = ua*T2 + ub*I).  The
// same construction in y turns every plane operator alpha*T2 + beta*I into a
// 2D hierarchy of x-line blocks in span{Tx, I}.  Planes with equal (ca, cb)
// share one 2D hierarchy ("plane type") and lines with equal (la, lb) share
// one Thomas factor table, so the tables are a few hundred KB even at 384^3.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <utility>

#include "net_internal.h"
#include "smg_internal.h"

using namespace smg;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxSmooth = 8;
constexpr int kMaxNx = 512;
constexpr int kProfAll = -1;      // profile every kernel family at once

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Galerkin coarsening of a block-tridiagonal operator with diagonal blocks
// D_f = da[f]*S + db[f]*I and couplings O_f = oa[f]*S + ob[f]*I (f <-> f+1)
// under linear interpolation from the odd points:
//   D^c_K = 1/4 D_{2K} + D_{2K+1} + 1/4 D_{2K+2} + O_{2K} + O_{2K+1}
//   O^c_K = 1/2 O_{2K+1} + 1/4 D_{2K+2} + 1/2 O_{2K+2}
// (terms naming a block past the end are absent).
struct BlockTri {
    std::vector<double> da, db, oa, ob;   // oa/ob have size n (last entry unused)
    int n() const { return static_cast<int>(da.size()); }
};

BlockTri galerkin(const BlockTri &f)
{
    const int n = f.n(), nc = n / 2;
    BlockTri c;
    c.da.assign(nc, 0.0);
    c.db.assign(nc, 0.0);
    c.oa.assign(nc, 0.0);
    c.ob.assign(nc, 0.0);
    for (int K = 0; K < nc; ++K) {
        const int f0 = 2 * K, f1 = 2 * K + 1, f2 = 2 * K + 2;
        double a = 0.25 * f.da[f0] + f.da[f1] + f.oa[f0];
        double b = 0.25 * f.db[f0] + f.db[f1] + f.ob[f0];
        if (f2 < n) {
            a += 0.25 * f.da[f2] + f.oa[f1];
            b += 0.25 * f.db[f2] + f.ob[f1];
        }
        c.da[K] = a;
        c.db[K] = b;
        if (K + 1 < nc) {
            c.oa[K] = 0.5 * f.oa[f1] + 0.25 * f.da[f2] + 0.5 * f.oa[f2];
            c.ob[K] = 0.5 * f.ob[f1] + 0.25 * f.db[f2] + 0.5 * f.ob[f2];
        }
    }
    return c;
}

struct Layout {
    size_t pcoef, lcoef, uniq, fac;        // tables
    std::vector<size_t> xl, bl;             // 3D levels >= 1
    std::vector<size_t> x2, b2, y2;         // 2D batch buffers per 2D level
    size_t rlo, slo;                        // low-precision level-0 in/out
    size_t kr, ks, kp0, kp1, kq, part, sc;  // Krylov
    size_t part3;                           // Krylov dots taken by the FP64 3D chain
    size_t total;
};

}  // namespace

struct smg_handle {
    smg_grid g;
    smg_opts o;
    int ipre, ipost;
    int max_nrhs;
    size_t N;
    int E, nxp;
    std::vector<int> nz;          // 3D level sizes
    std::vector<size_t> pc_off;   // PlaneCoef row offset per 3D level
    std::vector<int> ny2;         // 2D level sizes (shared by every plane)
    std::vector<int> lev2_off;    // line row offset per 2D level
    int lines_total;
    int nptypes, nfac, P2;
    size_t elem;                  // bytes per stored value
    // fused schedule: first LDS-resident 2D level, its LDS bytes, strip sizes
    bool fused;
    int l0;
    size_t coarse_lds;
    int S_down, S_up;
    int march_waves;              // down2 launches march runs of coarse lines while they keep this many waves
    size_t coarse_budget, strip_budget;   // LDS budgets the schedule was built for
    char *ws;
    Layout L;
    KScalars *host_sc;            // pinned host mirror of the device scalars
    smg::VarHier *var = nullptr;  // variable-coefficient hierarchy (smgv_setup), else null
    // per-kernel profiling: launches of family prof_family (every family when
    // it is kProfAll) get dispatch-stamped events and their algorithmic bytes
    // are summed; ev_lev / ev_bytes tag each stamped launch with its 3D level
    bool prof;
    int prof_family;
    std::vector<hipEvent_t> ev;
    int ev_used;
    double prof_bytes;
    std::vector<int> ev_lev;
    std::vector<double> ev_bytes;
    template <typename X> X *at(size_t off) const { return reinterpret_cast<X *>(ws + off); }
};

namespace {

int check_grid(const smg_grid *g, const smg_opts *o)
{
    if (!g || !o) return SMG_EINVAL;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nx > kMaxNx) return SMG_EINVAL;
    if (!(g->cx > 0.0) || !(g->cy > 0.0) || !(g->cz > 0.0)) return SMG_EINVAL;
    if (!std::isfinite(g->cx) || !std::isfinite(g->cy) || !std::isfinite(g->cz)) return SMG_EINVAL;
    if (o->pre < 0 || o->post < 0 || o->pre > kMaxSmooth || o->post > kMaxSmooth) return SMG_EINVAL;
    if (o->inner_pre < -1 || o->inner_post < -1 || o->inner_pre > kMaxSmooth || o->inner_post > kMaxSmooth)
        return SMG_EINVAL;
    if (o->order != 0 && o->order != 1) return SMG_EINVAL;
    if (o->precision < SMG_PREC_F64 || o->precision > SMG_PREC_BF16) return SMG_EINVAL;
    if (o->kernel_mode < 0 || o->kernel_mode > 2) return SMG_EINVAL;
    return SMG_OK;
}

size_t elem_size(int prec) { return prec == SMG_PREC_F64 ? 8 : prec == SMG_PREC_F32 ? 4 : 2; }
size_t arith_size(int prec) { return prec == SMG_PREC_F64 ? 8 : 4; }

// LDS budgets of the fused kernels (bytes per workgroup).  The coarse kernel
// is latency-bound (one workgroup per plane), so it may take most of a CU's
// 160 KB: every extra 2D level it absorbs removes one launch per 2D cycle.
constexpr size_t kCoarseLds = 160 * 1024;
constexpr size_t kStripLds = 48 * 1024;
// Register-only pre-smoothing: a launch with at least twice this many
// coarse-line waves gives each wave a run of 2, 4 or 8 coarse lines (fewer
// redundant line solves, fewer waves); below it every wave takes one line.
constexpr int kMarchWaves = 2048;

// Schedule of the fused 2D cycle for given LDS budgets: the coarse kernel
// takes every 2D level from l0 down whose lines fit coarse_budget; the strip
// kernels size their strips to strip_budget.
void apply_fused_schedule(smg_handle *h, size_t coarse_budget, size_t strip_budget)
{
    const size_t line = static_cast<size_t>(h->nxp) * arith_size(h->o.precision);
    const size_t row = h->o.precision == SMG_PREC_F64 ? sizeof(LineCoef<double>) : sizeof(LineCoef<float>);
    const int nl = static_cast<int>(h->ny2.size());
    h->l0 = nl - 1;
    h->coarse_lds = 0;
    // without post-smoothing the coarse kernel runs the downward half only and
    // holds one level's b and x at a time (down-only mode, from level 1 up)
    const bool down_only = h->ipre == 1 && h->ipost == 0 && h->o.order == 0;
    for (int l = nl - 1; l >= 0; --l) {
        size_t lines = 0;
        for (int m = l; m < nl; ++m) lines += h->ny2[m];
        // x and b of every line (down-only: of the first level), then the line rows
        const size_t xb = down_only && l >= 1 ? 2 * static_cast<size_t>(h->ny2[l]) : 2 * lines;
        const size_t bytes = xb * line + lines * row;
        if (bytes > coarse_budget) break;
        h->l0 = l;
        h->coarse_lds = bytes;
    }
    // k2_down handles one F line, one C line and one coarse line per wave
    const long long sl = static_cast<long long>(strip_budget / line);
    long long S = (sl - 5) / 2;
    const int smax = fused_waves() - 3;
    h->S_down = S < 1 ? 1 : (S > smax ? smax : static_cast<int>(S));
    S = (sl - 4) / 2;
    h->S_up = S < 1 ? 1 : (S > 16 ? 16 : static_cast<int>(S));
    h->coarse_budget = coarse_budget;
    h->strip_budget = strip_budget;
    h->fused = h->o.kernel_mode != 1 && nl <= kMaxLev && h->nz.size() <= static_cast<size_t>(kMaxLev3) &&
               h->coarse_lds > 0;
}

void choose_fused_schedule(smg_handle *h) { apply_fused_schedule(h, kCoarseLds, kStripLds); }

// Table sizes need the dedup counts, which depend only on the grid; the
// host part of the setup is cheap, so sizing runs it too.
struct Tables {
    std::vector<int> nz;
    std::vector<BlockTri> lev3;
    std::vector<std::pair<double, double>> ptypes;   // (ca, cb) per plane type
    std::vector<std::vector<int>> ptype_of;          // per level, per plane
    std::vector<int> ny2, lev2_off;
    int lines_total = 0;
    // per plane type: concatenated 2D level rows (la, lb, va, vb, fac)
    std::vector<double> line_rows;                    // 4 doubles per row
    std::vector<int> line_fac;
    std::vector<std::pair<double, double>> uniq;      // (la, lb) per Thomas table
};

Tables build_tables(const smg_grid &g)
{
    Tables t;
    BlockTri f;
    f.da.assign(g.nz, 1.0);
    f.db.assign(g.nz, 2.0 * g.cz);
    f.oa.assign(g.nz, 0.0);
    f.ob.assign(g.nz, -g.cz);
    t.lev3.push_back(f);
    while (t.lev3.back().n() > 1) t.lev3.push_back(galerkin(t.lev3.back()));
    for (auto &L : t.lev3) t.nz.push_back(L.n());

    std::map<std::pair<double, double>, int> pmap;
    for (auto &L : t.lev3) {
        std::vector<int> pt(L.n());
        for (int k = 0; k < L.n(); ++k) {
            auto key = std::make_pair(L.da[k], L.db[k]);
            auto it = pmap.find(key);
            if (it == pmap.end()) {
                it = pmap.emplace(key, static_cast<int>(t.ptypes.size())).first;
                t.ptypes.push_back(key);
            }
            pt[k] = it->second;
        }
        t.ptype_of.push_back(pt);
    }

    int n = g.ny;
    t.ny2.push_back(n);
    while (n > 1) {
        n /= 2;
        t.ny2.push_back(n);
    }
    t.lines_total = 0;
    for (int v : t.ny2) {
        t.lev2_off.push_back(t.lines_total);
        t.lines_total += v;
    }

    std::map<std::pair<double, double>, int> fmap;
    for (auto &pt : t.ptypes) {
        const double alpha = pt.first, beta = pt.second;
        BlockTri l0;
        l0.da.assign(g.ny, alpha * g.cx);
        l0.db.assign(g.ny, 2.0 * alpha * g.cy + beta);
        l0.oa.assign(g.ny, 0.0);
        l0.ob.assign(g.ny, -alpha * g.cy);
        BlockTri cur = l0;
        for (size_t l = 0; l < t.ny2.size(); ++l) {
            if (l > 0) cur = galerkin(cur);
            for (int j = 0; j < cur.n(); ++j) {
                const bool last = j == cur.n() - 1;
                t.line_rows.push_back(cur.da[j]);
                t.line_rows.push_back(cur.db[j]);
                t.line_rows.push_back(last ? 0.0 : cur.oa[j]);
                t.line_rows.push_back(last ? 0.0 : cur.ob[j]);
                auto key = std::make_pair(cur.da[j], cur.db[j]);
                auto it = fmap.find(key);
                if (it == fmap.end()) {
                    it = fmap.emplace(key, static_cast<int>(t.uniq.size())).first;
                    t.uniq.push_back(key);
                }
                t.line_fac.push_back(it->second);
            }
        }
    }
    return t;
}

Layout make_layout(const smg_grid &g, const smg_opts &o, int max_nrhs, const Tables &t, int nxp)
{
    Layout L{};
    const size_t es = elem_size(o.precision), as = arith_size(o.precision);
    const size_t N = static_cast<size_t>(g.nx) * g.ny * g.nz;
    const size_t pl = static_cast<size_t>(g.nx) * g.ny;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t r = off;
        off = align_up(off + bytes);
        return r;
    };
    size_t nplanes = 0;
    for (int v : t.nz) nplanes += v;
    const size_t pcsz = as == 8 ? sizeof(PlaneCoef<double>) : sizeof(PlaneCoef<float>);
    const size_t lcsz = as == 8 ? sizeof(LineCoef<double>) : sizeof(LineCoef<float>);
    const size_t fsz = as == 8 ? sizeof(Fac<double>) : sizeof(Fac<float>);
    L.pcoef = take(nplanes * pcsz);
    L.lcoef = take(t.ptypes.size() * t.lines_total * lcsz);
    L.uniq = take(t.uniq.size() * lcsz);
    L.fac = take(t.uniq.size() * nxp * fsz);
    L.xl.assign(t.nz.size(), 0);
    L.bl.assign(t.nz.size(), 0);
    for (size_t l = 1; l < t.nz.size(); ++l) {
        L.xl[l] = take(static_cast<size_t>(max_nrhs) * pl * t.nz[l] * es);
        L.bl[l] = take(static_cast<size_t>(max_nrhs) * pl * t.nz[l] * es);
    }
    const size_t P2 = (g.nz + 1) / 2;
    for (size_t l = 0; l < t.ny2.size(); ++l) {
        const size_t sz = static_cast<size_t>(max_nrhs) * P2 * g.nx * t.ny2[l] * es;
        L.x2.push_back(take(sz));
        L.b2.push_back(take(sz));
        L.y2.push_back(take(sz));
    }
    if (o.precision != SMG_PREC_F64) {
        L.rlo = take(static_cast<size_t>(max_nrhs) * N * es);
        L.slo = take(static_cast<size_t>(max_nrhs) * N * es);
    }
    L.kr = take(N * 8);
    L.ks = take(N * 8);
    L.kp0 = take(N * 8);
    L.kp1 = take(N * 8);
    L.kq = take(N * 8);
    L.part = take(2 * kRedBlocks * 8);
    L.part3 = o.precision == SMG_PREC_F64 ? take(2 * static_cast<size_t>(chain3_blocks(g.nx, g.ny, g.nz)) * 8) : 0;
    L.sc = take(sizeof(KScalars));
    L.total = off;
    return L;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------------------
// V-cycle
// ---------------------------------------------------------------------------

// Krylov inner products (s, r) and, with want_sq, (s, q) that a cycle ending in
// the FP64 3D chain takes while it stores s (one right-hand side).
struct VcDots {
    const double *r, *q;
    int want_sq;
};

template <typename T, typename A>
struct VCycle {
    smg_handle *h;
    hipStream_t st;
    int nrhs;
    T *x0;
    const T *b0;
    long long ld0;
    const VcDots *dots = nullptr;   // Krylov dots to take with the output, if the schedule can
    bool dots_done = false;

    struct Batch {          // a set of planes handled by one batched 2D cycle
        int np, kmul, koff;
        const PlaneCoef<A> *pc;
        T *x;
        long long xps, xrs;
        const T *b;
        long long bps, brs;
    };

    long long pl() const { return static_cast<long long>(h->g.nx) * h->g.ny; }
    long long nl(int l) const { return pl() * h->nz[l]; }
    T *X(int l) const { return l == 0 ? x0 : h->at<T>(h->L.xl[l]); }
    T *B(int l) const { return l == 0 ? const_cast<T *>(b0) : h->at<T>(h->L.bl[l]); }
    long long LD(int l) const { return l == 0 ? ld0 : nl(l); }
    const PlaneCoef<A> *PC(int l) const { return h->at<PlaneCoef<A>>(h->L.pcoef) + h->pc_off[l]; }
    const LineCoef<A> *LC(int l2) const { return h->at<LineCoef<A>>(h->L.lcoef) + h->lev2_off[l2]; }
    long long ps2(int l2) const { return static_cast<long long>(h->g.nx) * h->ny2[l2]; }
    long long rs2(int l2) const { return static_cast<long long>(h->P2) * ps2(l2); }

    int cur_lev = 0;        // 3D level whose work is being launched (profiling tag)

    // widest points-per-thread the streaming kernels may take (0: their own choice)
    int vmax() const { return h->o.kernel_mode == 2 ? 1 : 0; }

    // Events for this launch when its family is being profiled; `values` is the
    // launch's algorithmic traffic in stored values (each read or written once).
    LaunchEv ev_for(int family, double values)
    {
        if (!h->prof || (h->prof_family != kProfAll && family != h->prof_family) ||
            h->ev_used + 2 > static_cast<int>(h->ev.size()))
            return LaunchEv{};
        LaunchEv e{h->ev[h->ev_used], h->ev[h->ev_used + 1]};
        h->ev_lev[h->ev_used / 2] = cur_lev;
        h->ev_bytes[h->ev_used / 2] = values * sizeof(T);
        h->ev_used += 2;
        h->prof_bytes += values * sizeof(T);
        return e;
    }

    // colour residual: b and the result on the colour's planes, the other
    // colour's planes once, and the own planes unless they are still zero
    double resid3_values(int nz, int np, bool self_zero) const
    {
        return (2.0 * np + (nz - np) + (self_zero ? 0.0 : np)) * pl() * nrhs;
    }

    void line_relax(const Batch &bt, int l2, T *x, long long xps, long long xrs, const T *b, long long bps,
                    long long brs, int colour, int nbr_zero)
    {
        LineRelaxArgs<T, A> a{};
        a.x = x; a.b = b;
        a.xps = xps; a.xrs = xrs; a.bps = bps; a.brs = brs;
        a.nx = h->g.nx;
        a.ny = h->ny2[l2];
        a.colour = colour;
        a.nq = a.ny == 1 ? 1 : (colour == 0 ? (a.ny + 1) / 2 : a.ny / 2);
        a.np = bt.np; a.nrhs = nrhs; a.kmul = bt.kmul; a.koff = bt.koff;
        a.pc = bt.pc;
        a.lc = LC(l2);
        a.lines_total = h->lines_total;
        a.fac = h->at<Fac<A>>(h->L.fac);
        a.nxp = h->nxp;
        a.nbr_zero = nbr_zero || a.ny == 1;
        const double lines = a.nbr_zero ? 2.0 * a.nq : static_cast<double>(a.nq + a.ny);
        launch_line_relax<T, A>(a, st, ev_for(SMG_KERNEL_LINE_RELAX, lines * a.nx * a.np * a.nrhs));
    }

    void v2(const Batch &bt, int l2)
    {
        const int ny = h->ny2[l2];
        T *x = l2 == 0 ? bt.x : h->at<T>(h->L.x2[l2]);
        const T *b = l2 == 0 ? bt.b : h->at<T>(h->L.b2[l2]);
        const long long xps = l2 == 0 ? bt.xps : ps2(l2), xrs = l2 == 0 ? bt.xrs : rs2(l2);
        const long long bps = l2 == 0 ? bt.bps : ps2(l2), brs = l2 == 0 ? bt.brs : rs2(l2);
        if (ny == 1) {
            line_relax(bt, l2, x, xps, xrs, b, bps, brs, 0, 1);
            return;
        }
        const int first = h->o.order == 0 ? 0 : 1, second = 1 - first;
        for (int s = 0; s < h->ipre; ++s) {
            line_relax(bt, l2, x, xps, xrs, b, bps, brs, first, s == 0);
            line_relax(bt, l2, x, xps, xrs, b, bps, brs, second, 0);
        }
        const int x_zero = h->ipre == 0;
        Restrict2Args<T, A> ra{};
        ra.x = x; ra.b = b; ra.bc = h->at<T>(h->L.b2[l2 + 1]);
        ra.xps = xps; ra.xrs = xrs; ra.bps = bps; ra.brs = brs;
        ra.cps = ps2(l2 + 1); ra.crs = rs2(l2 + 1);
        ra.nx = h->g.nx; ra.ny = ny; ra.nyc = h->ny2[l2 + 1];
        ra.np = bt.np; ra.nrhs = nrhs; ra.kmul = bt.kmul; ra.koff = bt.koff;
        ra.pc = bt.pc; ra.lc = LC(l2); ra.lines_total = h->lines_total;
        ra.x_zero = x_zero;
        launch_restrict2<T, A>(ra, st, ev_for(SMG_KERNEL_RESTRICT2,
                                             (x_zero ? 1.0 : 2.0) * ny * h->g.nx * bt.np * nrhs +
                                                 1.0 * ra.nyc * h->g.nx * bt.np * nrhs));
        v2(bt, l2 + 1);
        Prolong2Args<T, A> pa{};
        pa.x = x; pa.xc = h->at<T>(h->L.x2[l2 + 1]);
        pa.xps = xps; pa.xrs = xrs; pa.cps = ps2(l2 + 1); pa.crs = rs2(l2 + 1);
        pa.nx = h->g.nx; pa.ny = ny; pa.nyc = h->ny2[l2 + 1];
        pa.np = bt.np; pa.nrhs = nrhs; pa.x_zero = x_zero;
        launch_prolong2<T, A>(pa, st, ev_for(SMG_KERNEL_PROLONG2,
                                            ((x_zero ? 1.0 : 2.0) * ny + pa.nyc) * h->g.nx * bt.np * nrhs));
        for (int s = 0; s < h->ipost; ++s) {
            line_relax(bt, l2, x, xps, xrs, b, bps, brs, second, 0);
            line_relax(bt, l2, x, xps, xrs, b, bps, brs, first, 0);
        }
    }

    // lines the coarse kernel reads and writes: b and x of level l0 (plus the
    // output read back when accumulating); down-only: b of l0, x of every level
    double coarse_values(const Coarse2Args<T, A> &c) const
    {
        if (!c.down_only) return (2.0 + c.accumulate) * c.ny2[c.l0];
        double v = c.ny2[c.l0];
        for (int l = c.l0; l < c.nlev; ++l) v += c.ny2[l];
        return v;
    }

    bool fused2() const { return h->fused && h->o.order == 0 && h->ipre == 1 && h->ipost <= 1; }
    bool chain3() const { return h->fused && h->o.post == 0 && h->o.pre >= 1; }

    // One batched 2D cycle on the fused schedule; the result is written to
    // out (plane stride ops, rhs stride ors), assigned or accumulated.
    void v2_fused(const Batch &bt, T *out, long long ops, long long ors, bool accumulate)
    {
        const int l0 = h->l0, nl = static_cast<int>(h->ny2.size());
        const int nx = h->g.nx;
        // where x_0 after pre-smoothing goes: in place in out when nothing is
        // accumulated and no post-smoothing reads it back across strips
        const bool in_place = h->ipost == 0 && !accumulate;
        T *x0pre = in_place ? out : h->at<T>(h->L.x2[0]);
        const long long x0ps = in_place ? ops : ps2(0), x0rs = in_place ? ors : rs2(0);
        auto Bp = [&](int l) { return l == 0 ? bt.b : h->at<T>(h->L.b2[l]); };
        auto Bps = [&](int l) { return l == 0 ? bt.bps : ps2(l); };
        auto Brs = [&](int l) { return l == 0 ? bt.brs : rs2(l); };
        for (int l = 0; l < l0; ++l) {
            Down2Args<T, A> d{};
            d.b = Bp(l); d.bps = Bps(l); d.brs = Brs(l);
            d.x = l == 0 ? x0pre : h->at<T>(h->L.x2[l]);
            d.xps = l == 0 ? x0ps : ps2(l); d.xrs = l == 0 ? x0rs : rs2(l);
            d.bc = h->at<T>(h->L.b2[l + 1]); d.cps = ps2(l + 1); d.crs = rs2(l + 1);
            d.nx = nx; d.nxp = h->nxp; d.ny = h->ny2[l]; d.nyc = h->ny2[l + 1]; d.S = h->S_down;
            d.np = bt.np; d.nrhs = nrhs; d.kmul = bt.kmul; d.koff = bt.koff;
            d.pc = bt.pc; d.lc = LC(l); d.lines_total = h->lines_total; d.fac = h->at<Fac<A>>(h->L.fac);
            d.march_waves = h->march_waves;
            launch_down2<T, A>(d, st, ev_for(SMG_KERNEL_DOWN2,
                                             (2.0 * d.ny + d.nyc) * nx * bt.np * static_cast<double>(nrhs)));
        }
        Coarse2Args<T, A> c{};
        c.b = Bp(l0); c.bps = Bps(l0); c.brs = Brs(l0);
        if (l0 == 0) {
            c.out = out; c.ops = ops; c.ors = ors; c.accumulate = accumulate;
        } else {
            c.out = h->at<T>(h->L.x2[l0]); c.ops = ps2(l0); c.ors = rs2(l0); c.accumulate = 0;
        }
        c.nx = nx; c.nxp = h->nxp; c.np = bt.np; c.nrhs = nrhs; c.kmul = bt.kmul; c.koff = bt.koff;
        c.l0 = l0; c.nlev = nl;
        for (int l = 0; l < nl; ++l) {
            c.ny2[l] = h->ny2[l];
            c.lev_off[l] = h->lev2_off[l];
        }
        c.ipre = h->ipre; c.ipost = h->ipost;
        c.pc = bt.pc; c.lc = LC(0); c.lines_total = h->lines_total; c.fac = h->at<Fac<A>>(h->L.fac);
        // down-only: every level's x in the level arrays, the chain from the coarsest
        const bool down_only = h->ipost == 0 && h->ipre == 1 && l0 >= 1;
        c.down_only = down_only;
        c.P2 = static_cast<int>(h->P2);
        for (int l = l0; l < nl; ++l) c.xl[l] = h->at<T>(h->L.x2[l]);
        launch_coarse2<T, A>(c, h->coarse_lds, st,
                             ev_for(SMG_KERNEL_COARSE2, coarse_values(c) * nx * bt.np * static_cast<double>(nrhs)));
        if (l0 == 0) return;
        if (h->ipost == 0) {
            Chain2Args<T, A> ch{};
            ch.x0 = x0pre; ch.x0ps = x0ps; ch.x0rs = x0rs;
            ch.out = out; ch.ops = ops; ch.ors = ors; ch.accumulate = accumulate;
            const int lc = down_only ? nl - 1 : l0;
            for (int l = 1; l <= lc; ++l) {
                ch.xc[l] = h->at<T>(h->L.x2[l]);
                ch.cps[l] = ps2(l);
                ch.crs[l] = rs2(l);
            }
            for (int l = 0; l <= lc; ++l) ch.ny2[l] = h->ny2[l];
            ch.nx = nx; ch.np = bt.np; ch.nrhs = nrhs; ch.lc = lc;
            ch.vmax = vmax();
            double lines = (2.0 + accumulate) * h->ny2[0];
            for (int l = 1; l <= lc; ++l) lines += h->ny2[l];
            launch_chain2<T, A>(ch, st, ev_for(SMG_KERNEL_CHAIN2, lines * nx * bt.np * static_cast<double>(nrhs)));
            return;
        }
        for (int l = l0 - 1; l >= 0; --l) {
            Up2Args<T, A> u{};
            u.xpre = l == 0 ? x0pre : h->at<T>(h->L.x2[l]);
            u.xps = l == 0 ? x0ps : ps2(l); u.xrs = l == 0 ? x0rs : rs2(l);
            u.xc = l + 1 == l0 ? h->at<T>(h->L.x2[l0]) : h->at<T>(h->L.y2[l + 1]);
            u.cps = ps2(l + 1); u.crs = rs2(l + 1);
            u.b = Bp(l); u.bps = Bps(l); u.brs = Brs(l);
            if (l == 0) {
                u.out = out; u.ops = ops; u.ors = ors; u.accumulate = accumulate;
            } else {
                u.out = h->at<T>(h->L.y2[l]); u.ops = ps2(l); u.ors = rs2(l); u.accumulate = 0;
            }
            u.nx = nx; u.nxp = h->nxp; u.ny = h->ny2[l]; u.nyc = h->ny2[l + 1]; u.S = h->S_up;
            u.np = bt.np; u.nrhs = nrhs; u.kmul = bt.kmul; u.koff = bt.koff;
            u.pc = bt.pc; u.lc = LC(l); u.lines_total = h->lines_total; u.fac = h->at<Fac<A>>(h->L.fac);
            launch_up2<T, A>(u, st, ev_for(SMG_KERNEL_UP2, ((3.0 + u.accumulate) * u.ny + u.nyc) * nx * bt.np *
                                                                static_cast<double>(nrhs)));
        }
    }

    // one zebra half-sweep over the planes of one colour at 3D level l
    void sweep3(int l, int colour, bool all_zero, bool self_zero)
    {
        if (fused2()) {
            sweep3_fused(l, colour, all_zero, self_zero);
            return;
        }
        const int nz = h->nz[l];
        const int np = colour == 0 ? (nz + 1) / 2 : nz / 2;
        if (np == 0) return;
        T *X0 = X(l);
        const T *B0 = B(l);
        const long long p = pl(), ld = LD(l);
        Batch bt{np, 2, colour, PC(l), nullptr, 0, 0, nullptr, 0, 0};
        if (all_zero) {            // x = 0: the plane right-hand sides are b itself
            bt.x = X0 + colour * p; bt.xps = 2 * p; bt.xrs = ld;
            bt.b = B0 + colour * p; bt.bps = 2 * p; bt.brs = ld;
            v2(bt, 0);
            return;
        }
        Resid3Args<T, A> ra{};
        ra.x = X0; ra.b = B0; ra.r = h->at<T>(h->L.b2[0]);
        ra.xrs = ld; ra.brs = ld; ra.rps = p; ra.rrs = rs2(0);
        ra.nx = h->g.nx; ra.ny = h->g.ny; ra.nz = nz; ra.np = np; ra.nrhs = nrhs;
        ra.kmul = 2; ra.koff = colour;
        ra.cx = static_cast<A>(h->g.cx); ra.cy = static_cast<A>(h->g.cy);
        ra.pc = PC(l);
        ra.self_zero = self_zero;
        ra.vmax = vmax();
        launch_resid3<T, A>(ra, st, ev_for(SMG_KERNEL_RESID3, resid3_values(nz, np, self_zero)));
        bt.b = ra.r; bt.bps = p; bt.brs = rs2(0);
        if (self_zero) {           // own planes still zero: write the solve in place
            bt.x = X0 + colour * p; bt.xps = 2 * p; bt.xrs = ld;
            v2(bt, 0);
            return;
        }
        bt.x = h->at<T>(h->L.x2[0]); bt.xps = p; bt.xrs = rs2(0);
        v2(bt, 0);
        Correct3Args<T, A> ca{};
        ca.x = X0; ca.y = bt.x; ca.xrs = ld; ca.yps = p; ca.yrs = rs2(0);
        ca.nx = h->g.nx; ca.ny = h->g.ny; ca.np = np; ca.nrhs = nrhs; ca.kmul = 2; ca.koff = colour;
        launch_correct3<T, A>(ca, st, ev_for(SMG_KERNEL_CORRECT3, 3.0 * np * p * nrhs));
    }

    void sweep3_fused(int l, int colour, bool all_zero, bool self_zero)
    {
        const int nz = h->nz[l];
        const int np = colour == 0 ? (nz + 1) / 2 : nz / 2;
        if (np == 0) return;
        T *X0 = X(l);
        const long long p = pl(), ld = LD(l);
        Batch bt{np, 2, colour, PC(l), nullptr, 0, 0, nullptr, 0, 0};
        if (all_zero) {
            bt.b = B(l) + colour * p; bt.bps = 2 * p; bt.brs = ld;
        } else {
            Resid3Args<T, A> ra{};
            ra.x = X0; ra.b = B(l); ra.r = h->at<T>(h->L.b2[0]);
            ra.xrs = ld; ra.brs = ld; ra.rps = p; ra.rrs = rs2(0);
            ra.nx = h->g.nx; ra.ny = h->g.ny; ra.nz = nz; ra.np = np; ra.nrhs = nrhs;
            ra.kmul = 2; ra.koff = colour;
            ra.cx = static_cast<A>(h->g.cx); ra.cy = static_cast<A>(h->g.cy);
            ra.pc = PC(l);
            ra.self_zero = self_zero;
            ra.vmax = vmax();
            launch_resid3<T, A>(ra, st, ev_for(SMG_KERNEL_RESID3, resid3_values(nz, np, self_zero)));
            bt.b = ra.r; bt.bps = p; bt.brs = rs2(0);
        }
        v2_fused(bt, X0 + colour * p, 2 * p, ld, !self_zero);
    }

    void chain3_all()
    {
        Chain3Args<T, A> a{};
        const int L = static_cast<int>(h->nz.size()) - 1;
        for (int l = 0; l <= L; ++l) {
            a.x[l] = X(l);
            a.rs[l] = LD(l);
            a.nz[l] = h->nz[l];
        }
        a.L = L; a.nx = h->g.nx; a.ny = h->g.ny;
        a.vmax = vmax();
        if constexpr (sizeof(T) == 8) {
            if (dots && nrhs == 1) {
                a.dr = dots->r; a.dq = dots->q; a.want_sq = dots->want_sq;
                a.dpart = h->at<double>(h->L.part3);
                dots_done = true;
            }
        }
        double planes = h->nz[0];
        for (int l = 0; l <= L; ++l) planes += h->nz[l];
        launch_chain3<T, A>(a, nrhs, st, ev_for(SMG_KERNEL_CHAIN3, planes * pl() * nrhs));
    }

    void v3(int l)
    {
        cur_lev = l;
        const int nz = h->nz[l];
        if (nz == 1) {
            Batch bt{1, 1, 0, PC(l), X(l), pl(), LD(l), B(l), pl(), LD(l)};
            if (fused2())
                v2_fused(bt, X(l), pl(), LD(l), false);
            else
                v2(bt, 0);
            return;
        }
        const int first = h->o.order == 0 ? 0 : 1, second = 1 - first;
        for (int s = 0; s < h->o.pre; ++s) {
            sweep3(l, first, s == 0, s == 0);
            sweep3(l, second, false, s == 0);
        }
        const int x_zero = h->o.pre == 0;
        Restrict3Args<T, A> ra{};
        ra.x = X(l); ra.b = B(l); ra.bc = B(l + 1);
        ra.xrs = LD(l); ra.brs = LD(l); ra.crs = nl(l + 1);
        ra.nx = h->g.nx; ra.ny = h->g.ny; ra.nz = nz; ra.nzc = h->nz[l + 1]; ra.nrhs = nrhs;
        ra.cx = static_cast<A>(h->g.cx); ra.cy = static_cast<A>(h->g.cy);
        ra.pc = PC(l);
        ra.x_zero = x_zero;
        ra.vmax = vmax();
        launch_restrict3<T, A>(ra, st, ev_for(SMG_KERNEL_RESTRICT3,
                                             ((x_zero ? 1.0 : 2.0) * nz + h->nz[l + 1]) * pl() * nrhs));
        v3(l + 1);
        cur_lev = l;
        if (chain3()) {          // no post-smoothing: all prolongations in one pass
            if (l == 0) {
                cur_lev = static_cast<int>(h->nz.size());   // spans every level
                chain3_all();
            }
            return;
        }
        Prolong3Args<T, A> pa{};
        pa.x = X(l); pa.xc = X(l + 1); pa.xrs = LD(l); pa.crs = nl(l + 1);
        pa.nx = h->g.nx; pa.ny = h->g.ny; pa.nz = nz; pa.nzc = h->nz[l + 1]; pa.nrhs = nrhs;
        pa.x_zero = x_zero;
        launch_prolong3<T, A>(pa, st, ev_for(SMG_KERNEL_PROLONG3,
                                            ((x_zero ? 1.0 : 2.0) * nz + h->nz[l + 1]) * pl() * nrhs));
        for (int s = 0; s < h->o.post; ++s) {
            sweep3(l, second, false, false);
            sweep3(l, first, false, false);
        }
    }
};

template <typename T, typename A>
bool run_vcycle(smg_handle *h, const double *r, double *s, int nrhs, long long ld, hipStream_t st,
                const VcDots *dots)
{
    VCycle<T, A> vc{h, st, nrhs, nullptr, nullptr, 0};
    if constexpr (sizeof(T) == 8) {
        vc.x0 = reinterpret_cast<T *>(s);
        vc.b0 = reinterpret_cast<const T *>(r);
        vc.ld0 = ld;
        vc.dots = dots;
        vc.v3(0);
        return vc.dots_done;
    } else {
        T *rlo = h->at<T>(h->L.rlo), *slo = h->at<T>(h->L.slo);
        launch_convert_in<T>(r, ld, rlo, static_cast<long long>(h->N), h->N, nrhs, st);
        vc.x0 = slo;
        vc.b0 = rlo;
        vc.ld0 = static_cast<long long>(h->N);
        vc.v3(0);
        launch_convert_out<T>(slo, static_cast<long long>(h->N), s, ld, h->N, nrhs, st);
        return false;
    }
}

// s = B r.  With dots, the cycle may also leave the Krylov partials (s, r) and
// (s, q) for the finalize step; it returns whether it did (they are then in
// part3, chain3_blocks per quantity), else the caller takes them itself.
bool vcycle(smg_handle *h, const double *r, double *s, int nrhs, long long ld, hipStream_t st,
            const VcDots *dots = nullptr)
{
    if (h->var) {
        var_vcycle(h->var, r, s, nrhs, ld, st);
        return false;
    }
    switch (h->o.precision) {
    case SMG_PREC_F64: return run_vcycle<double, double>(h, r, s, nrhs, ld, st, dots);
    case SMG_PREC_F32: return run_vcycle<float, float>(h, r, s, nrhs, ld, st, dots);
    default: return run_vcycle<bf16, float>(h, r, s, nrhs, ld, st, dots);
    }
}

template <typename A>
int upload_tables(smg_handle *h, const Tables &t, hipStream_t st)
{
    std::vector<PlaneCoef<A>> pc;
    for (size_t l = 0; l < t.lev3.size(); ++l) {
        const BlockTri &L = t.lev3[l];
        for (int k = 0; k < L.n(); ++k) {
            PlaneCoef<A> c{};
            c.ca = static_cast<A>(L.da[k]);
            c.cb = static_cast<A>(L.db[k]);
            c.ua = k + 1 < L.n() ? static_cast<A>(L.oa[k]) : A(0);
            c.ub = k + 1 < L.n() ? static_cast<A>(L.ob[k]) : A(0);
            c.pt = t.ptype_of[l][k];
            pc.push_back(c);
        }
    }
    std::vector<LineCoef<A>> lc(t.line_fac.size());
    for (size_t i = 0; i < lc.size(); ++i) {
        lc[i].la = static_cast<A>(t.line_rows[4 * i + 0]);
        lc[i].lb = static_cast<A>(t.line_rows[4 * i + 1]);
        lc[i].va = static_cast<A>(t.line_rows[4 * i + 2]);
        lc[i].vb = static_cast<A>(t.line_rows[4 * i + 3]);
        lc[i].fac = t.line_fac[i];
    }
    // Thomas tables are built on the device from FP64 (la, lb) pairs.
    std::vector<LineCoef<double>> uq(t.uniq.size());
    for (size_t i = 0; i < uq.size(); ++i) {
        uq[i] = LineCoef<double>{};
        uq[i].la = t.uniq[i].first;
        uq[i].lb = t.uniq[i].second;
    }
    if (hipMemcpyAsync(h->ws + h->L.pcoef, pc.data(), pc.size() * sizeof(pc[0]), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(h->ws + h->L.lcoef, lc.data(), lc.size() * sizeof(lc[0]), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(h->ws + h->L.uniq, uq.data(), uq.size() * sizeof(uq[0]), hipMemcpyHostToDevice, st) !=
            hipSuccess)
        return SMG_EHIP;
    launch_thomas_tables<A>(h->at<LineCoef<double>>(h->L.uniq), h->nfac, h->g.nx, h->nxp, h->at<Fac<A>>(h->L.fac),
                            st);
    if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) return SMG_EHIP;
    return SMG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Krylov (Algorithm 1)
// ---------------------------------------------------------------------------
int smg::krylov_run(smg_handle *h, int method, const double *b, double *x, const krylov_opts *o,
                    krylov_info *info, void *stream, PrecondHook *hook)
{
    if (!h || !b || !x || !o) return SMG_EINVAL;
    if (o->max_iter < 0 || !(o->rtol >= 0.0)) return SMG_EINVAL;
    if (o->precond != SMG_PRECOND_SMG && o->precond != SMG_PRECOND_NONE) return SMG_EINVAL;
    if (o->stop_norm != SMG_STOP_2NORM && o->stop_norm != SMG_STOP_CNORM) return SMG_EINVAL;
    if ((o->err_a || o->sin_angle) && !o->xstar) return SMG_EINVAL;
    if (o->xstar && !o->diag_work) return SMG_EINVAL;
    hipStream_t st = as_stream(stream);
    const auto t0 = std::chrono::steady_clock::now();
    const smg_grid &g = h->g;
    const size_t n = h->N;
    double *r = h->at<double>(h->L.kr), *s = h->at<double>(h->L.ks), *q = h->at<double>(h->L.kq);
    double *pa = h->at<double>(h->L.kp0), *pb = h->at<double>(h->L.kp1);
    double *part = h->at<double>(h->L.part);
    KScalars *sc = h->at<KScalars>(h->L.sc);
    KScalars *hs = h->host_sc;
    const bool cstop = o->stop_norm == SMG_STOP_CNORM;
    const bool want_c = cstop || o->history_c;
    const bool diag = o->xstar != nullptr;
    krylov_info inf{};
    inf.rel_res_c = std::numeric_limits<double>::quiet_NaN();
    auto finish = [&](int status) {
        inf.status = status;
        inf.solve_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (info) *info = inf;
        return status;
    };
    auto sync = [&]() { return hipStreamSynchronize(st) == hipSuccess && hipGetLastError() == hipSuccess; };
    auto precond = [&](const double *in, double *out) {
        if (o->precond == SMG_PRECOND_SMG)
            vcycle(h, in, out, 1, static_cast<long long>(n), st);
        else
            launch_copy(in, out, n, st);
    };
    // s_k = B r_k for iteration kk.  Without a correction hook the cycle may
    // take the iteration's (s, r) and (s, q) as it stores s; returns whether it
    // did (the partials are then in part3, nparts3 per quantity).
    const double *part3 = nullptr;
    int nparts3 = 0;
    auto precond_k = [&](int kk) {
        if (o->precond != SMG_PRECOND_SMG || (hook && hook->active)) {
            precond(r, s);
            return false;
        }
        return vcycle_dots(h, r, s, q, method == 1 && kk > 0, st, &part3, &nparts3);
    };
    // ||x* - x||_A^2 with the diagnostic scratch (e = x* - x, then A e)
    double *de = diag ? o->diag_work : nullptr, *dw = diag ? o->diag_work + n : nullptr;
    // the operator's passes: the 7-point model stencil, or the handle's
    // variable-coefficient operator
    auto op_matvec = [&](const double *in, double *out) {
        if (h->var)
            var_matvec(h->var, in, out, 1, static_cast<long long>(n), st);
        else
            launch_matvec7(in, out, static_cast<long long>(n), 1, g.nx, g.ny, g.nz, g.cx, g.cy, g.cz, st);
    };
    auto op_resid = [&](const double *bb, const double *xx, double *rr, int x_zero) {
        if (h->var)
            var_init_resid(h->var, bb, xx, rr, x_zero, part, st);
        else
            launch_init_resid(bb, xx, rr, x_zero, g.nx, g.ny, g.nz, g.cx, g.cy, g.cz, part, st);
    };
    auto op_update_p_q = [&](const double *su, double *p_old, double *p_new) {
        if (h->var)
            var_update_p_q(h->var, su, p_old, p_new, q, sc, part, st);
        else
            launch_update_p_q(su, p_old, p_new, q, sc, g.nx, g.ny, g.nz, g.cx, g.cy, g.cz, part, st);
    };
    auto err_a2 = [&](double *out) {
        launch_axpby(de, o->xstar, 1.0, x, -1.0, n, st);
        op_matvec(de, dw);
        return device_dot2(de, dw, nullptr, nullptr, n, part, st, out, nullptr);
    };
    // End of an iteration's work on the stream (its scalars are in hs once it
    // completes), so that the next iteration's V-cycle can be queued before
    // the host waits; see the loop.
    struct Event {
        hipEvent_t e = nullptr;
        ~Event()
        {
            if (e) (void)hipEventDestroy(e);
        }
    } done;
    if (hipEventCreateWithFlags(&done.e, hipEventDisableTiming) != hipSuccess) return finish(SMG_EHIP);
    auto fall_back = [&](int k, int reason) {
        hook->active = 0;
        hook->fallback_iter = k;
        hook->fallback_reason = reason;
    };

    if (o->x0_zero) launch_fill(x, 0.0, n, st);
    op_resid(b, x, r, o->x0_zero ? 1 : 0);
    launch_finalize(0, method, 0, part, sc, hs, st);
    if (!sync()) return finish(SMG_EHIP);
    if (!std::isfinite(hs->rr) || !std::isfinite(hs->bb)) return finish(SMG_ENONFINITE);
    const double bnorm = std::sqrt(hs->bb);
    const double bden = bnorm > 0.0 ? bnorm : 1.0;
    double rel = std::sqrt(hs->rr) / bden;
    std::vector<double> rels{rel};
    if (o->history) o->history[0] = rel;
    // Denominator of the C-norm ratio, sqrt|(T b, b)|.  With x0 = 0 it is the
    // first iteration's sqrt|(s_0, r_0)|; otherwise T b costs one V-cycle here.
    double cden = 0.0;
    bool cden_pending = false;
    if (want_c) {
        if (o->precond == SMG_PRECOND_NONE) {
            cden = bnorm;
        } else if (o->x0_zero) {
            cden_pending = true;
        } else {
            double tbb = 0.0;
            precond(b, s);
            if (device_dot2(s, b, nullptr, nullptr, n, part, st, &tbb, nullptr) != SMG_OK) return finish(SMG_EHIP);
            cden = std::sqrt(std::fabs(tbb));
        }
    }
    double ea0 = 0.0;
    if (diag) {
        if (err_a2(&ea0) != SMG_OK) return finish(SMG_EHIP);
        if (o->err_a) o->err_a[0] = ea0 > 0.0 ? 1.0 : 0.0;
    }
    int k = 0, status = SMG_NOT_CONVERGED;
    bool queued = false;        // this iteration's V-cycle is already on the stream
    bool queued_dots = false;   // ... and it took the iteration's dots
    bool cconv = false;         // C-norm test met
    for (; k < o->max_iter; ++k) {
        if (!cstop && !(rel > o->rtol)) break;
        bool fused_dots;
        if (queued) {
            queued = false;
            fused_dots = queued_dots;
        } else {
            fused_dots = precond_k(k);
        }
        const double *su = s;
        bool dots_done = false;
        if (hook && hook->active) {
            // learned correction of s_k; the policy falls back to plain s_k
            const double *sl = hook->apply(hook->ctx, r, s, st);
            if (!sl) return finish(SMG_EHIP);
            launch_dots_sr_sq(sl, r, q, method == 1 && k > 0, n, part, st);
            launch_finalize(1, method, k, part, sc, hs, st);
            if (!sync()) return finish(SMG_EHIP);
            if (!std::isfinite(hs->sr) || !std::isfinite(hs->sq))
                fall_back(k, NET_FALLBACK_NONFINITE);
            else if (!(hs->sr > 0.0))
                fall_back(k, NET_FALLBACK_SR);
            else {
                su = sl;
                dots_done = true;
            }
        }
        if (!dots_done) {
            if (fused_dots) {
                launch_finalize(1, method, k, part3, sc, want_c ? hs : nullptr, st, nparts3);
            } else {
                launch_dots_sr_sq(s, r, q, method == 1 && k > 0, n, part, st);
                launch_finalize(1, method, k, part, sc, want_c ? hs : nullptr, st);
            }
        }
        if (want_c) {
            // (s_k, r_k) on the host: the C-norm ratio and its stopping test
            if (!sync()) return finish(SMG_EHIP);
            const double crk = std::sqrt(std::fabs(hs->sr));
            if (cden_pending) {
                cden = crk;
                cden_pending = false;
            }
            const double relc = crk / (cden > 0.0 ? cden : 1.0);
            inf.rel_res_c = relc;
            if (o->history_c) o->history_c[k] = relc;
            if (cstop && !(relc > o->rtol)) {
                cconv = true;
                break;
            }
        }
        if (diag) {
            // Theorem 1: cos = |(r_k, s_k)| / (||r_k||_{A^{-1}} ||A s_k||_{A^{-1}}), with
            // ||r_k||_{A^{-1}} = ||x* - x_k||_A and ||A s_k||_{A^{-1}}^2 = (s_k, A s_k)
            double ea = 0.0, sas = 0.0, sr = 0.0;
            if (err_a2(&ea) != SMG_OK) return finish(SMG_EHIP);
            op_matvec(su, dw);
            if (device_dot2(su, dw, su, r, n, part, st, &sas, &sr) != SMG_OK) return finish(SMG_EHIP);
            if (o->sin_angle) {
                const double c2 = (ea > 0.0 && sas > 0.0) ? sr * sr / (ea * sas) : 1.0;
                o->sin_angle[k] = std::sqrt(std::max(0.0, 1.0 - c2));
            }
        }
        op_update_p_q(su, pa, pb);
        launch_finalize(2, method, k, part, sc, nullptr, st);
        launch_update_xr(x, r, pb, q, sc, n, part, st);
        launch_finalize(3, method, k, part, sc, hs, st);
        // When the residual history says the next iteration will run (the
        // rate of the last two steps, with a margin of 4 over rtol), its
        // V-cycle s = B r_{k+1} goes on the stream before the host waits for
        // this iteration's scalars, so the GPU does not idle meanwhile.  The
        // V-cycle writes s and its own level buffers only, which nothing reads
        // after a stop (the true residual below uses s as scratch).
        const double pred = k == 0 ? 0.5 * rels[0] : rels[k] * (rels[k] / rels[k - 1]);
        const bool ahead = o->precond == SMG_PRECOND_SMG && !(hook && hook->active) && !diag && !cstop &&
                           k + 1 < o->max_iter && pred > 4.0 * o->rtol;
        if (ahead) {
            if (hipEventRecord(done.e, st) != hipSuccess) return finish(SMG_EHIP);
            queued_dots = precond_k(k + 1);
            queued = true;
            if (hipEventSynchronize(done.e) != hipSuccess || hipGetLastError() != hipSuccess)
                return finish(SMG_EHIP);
        } else if (!sync()) {
            return finish(SMG_EHIP);
        }
        std::swap(pa, pb);
        if (hs->breakdown) {
            inf.iters = k;
            status = SMG_EBREAKDOWN;
            break;
        }
        rel = std::sqrt(hs->rr) / bden;
        rels.push_back(rel);
        if (o->history) o->history[k + 1] = rel;
        if (diag && o->err_a) {
            double ea = 0.0;
            if (err_a2(&ea) != SMG_OK) return finish(SMG_EHIP);
            o->err_a[k + 1] = ea0 > 0.0 ? std::sqrt(ea / ea0) : 0.0;
        }
        if (!std::isfinite(rel)) {
            status = SMG_EBREAKDOWN;
            ++k;
            break;
        }
        if (hook && hook->active && k >= 1 && rel > 0.9 * rels[k - 1]) fall_back(k + 1, NET_FALLBACK_STAGNATION);
    }
    inf.iters = k;
    if (status != SMG_EBREAKDOWN) status = (cstop ? cconv : rel <= o->rtol) ? SMG_OK : SMG_NOT_CONVERGED;
    inf.rel_res = rel;
    op_resid(b, x, s, 0);
    launch_finalize(0, method, 0, part, sc, hs, st);
    if (!sync()) return finish(SMG_EHIP);
    inf.true_rel_res = std::sqrt(hs->rr) / bden;
    return finish(status);
}

int smg_handle_size(const smg_handle *h, size_t *n)
{
    if (!h || !n) return SMG_EINVAL;
    *n = h->N;
    return SMG_OK;
}

const smg_grid *smg_handle_grid(const smg_handle *h) { return h ? &h->g : nullptr; }

double *smg::handle_partials(smg_handle *h) { return h->at<double>(h->L.part); }

int smg_handle_is_var(const smg_handle *h) { return h && h->var ? 1 : 0; }

int smg::krylov_view(smg_handle *h, KrylovView *v)
{
    if (!h || !v) return SMG_EINVAL;
    v->r = h->at<double>(h->L.kr);
    v->s = h->at<double>(h->L.ks);
    v->q = h->at<double>(h->L.kq);
    v->pa = h->at<double>(h->L.kp0);
    v->pb = h->at<double>(h->L.kp1);
    v->part = h->at<double>(h->L.part);
    v->sc = h->at<KScalars>(h->L.sc);
    v->g = h->g;
    v->n = h->N;
    v->precision = h->o.precision;
    return SMG_OK;
}

void smg::vcycle_apply(smg_handle *h, const double *r, double *s, int nrhs, long long ld, hipStream_t st)
{
    vcycle(h, r, s, nrhs, ld, st);
}

bool smg::vcycle_dots(smg_handle *h, const double *r, double *s, const double *q, int want_sq, hipStream_t st,
                      const double **part, int *nparts)
{
    const VcDots d{r, q, want_sq};
    if (!vcycle(h, r, s, 1, static_cast<long long>(h->N), st, h->L.part3 ? &d : nullptr)) return false;
    *part = h->at<double>(h->L.part3);
    *nparts = static_cast<int>(chain3_blocks(h->g.nx, h->g.ny, h->g.nz));
    return true;
}

int smg_handle_max_nrhs(const smg_handle *h, int32_t *max_nrhs)
{
    if (!h || !max_nrhs) return SMG_EINVAL;
    *max_nrhs = h->max_nrhs;
    return SMG_OK;
}

namespace {

// Everything smg_setup does except creating the handle: Galerkin tables,
// schedule, workspace layout and the upload of the tables into ws (which
// synchronises the stream).  With pinned, the handle also gets the pinned host
// mirror of the Krylov scalars that the solvers read.
int fill_handle(smg_handle *h, const smg_grid *g, const smg_opts *o, int32_t max_nrhs, char *ws, size_t ws_bytes,
                hipStream_t st, bool pinned)
{
    const Tables t = build_tables(*g);
    h->g = *g;
    h->o = *o;
    h->ipre = o->inner_pre < 0 ? o->pre : o->inner_pre;
    h->ipost = o->inner_post < 0 ? o->post : o->inner_post;
    h->max_nrhs = max_nrhs;
    h->N = static_cast<size_t>(g->nx) * g->ny * g->nz;
    h->E = (g->nx + 63) / 64;
    h->nxp = 64 * h->E;
    h->nz = t.nz;
    size_t acc = 0;
    for (int v : t.nz) {
        h->pc_off.push_back(acc);
        acc += v;
    }
    h->ny2 = t.ny2;
    h->lev2_off = t.lev2_off;
    h->lines_total = t.lines_total;
    h->nptypes = static_cast<int>(t.ptypes.size());
    h->nfac = static_cast<int>(t.uniq.size());
    h->P2 = (g->nz + 1) / 2;
    h->elem = elem_size(o->precision);
    choose_fused_schedule(h);
    h->march_waves = kMarchWaves;
    h->L = make_layout(*g, *o, max_nrhs, t, h->nxp);
    h->host_sc = nullptr;
    if (ws_bytes < h->L.total) return SMG_EWORKSPACE;
    h->ws = ws;
    h->prof = false;
    h->ev_used = 0;
    h->prof_bytes = 0;
    if (pinned && hipHostMalloc(reinterpret_cast<void **>(&h->host_sc), sizeof(KScalars), hipHostMallocDefault) !=
                      hipSuccess) {
        h->host_sc = nullptr;
        return SMG_EHIP;
    }
    return arith_size(o->precision) == 8 ? upload_tables<double>(h, t, st) : upload_tables<float>(h, t, st);
}

// Device scratch of smg_apply_static: one copy per GPU, held until the
// process ends.  Host code never uses the array's name as an address; it uses
// the per-device address from hipGetSymbolAddress, looked up once per device
// with that device current.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

int static_scratch(char **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SMG_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SMG_EHIP;
        g_scratch_ptr[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return SMG_OK;
}

}  // namespace

namespace {

// Runs `reps` single-vector V-cycles with the launches of `family` (or every
// launch, kProfAll) stamped by events; per V-cycle, sums the launches, their
// durations and their algorithmic bytes into row 0, or with by_level into the
// row of the launch's 3D level (nrows = levels + 1).
int profile_run(smg_handle *h, int family, bool by_level, const double *r, double *s, int reps, hipStream_t st,
                int nrows, int32_t *launches, double *kernel_ms, double *bytes)
{
    if (h->ev.empty()) {
        h->ev.resize(2 * 4096);
        for (auto &e : h->ev)
            if (hipEventCreate(&e) != hipSuccess) return SMG_EHIP;
    }
    h->ev_lev.assign(h->ev.size() / 2, 0);
    h->ev_bytes.assign(h->ev.size() / 2, 0.0);
    for (int i = 0; i < nrows; ++i) {
        launches[i] = 0;
        kernel_ms[i] = 0.0;
        bytes[i] = 0.0;
    }
    h->prof = true;
    h->prof_family = family;
    for (int rep = 0; rep < reps; ++rep) {
        h->ev_used = 0;
        h->prof_bytes = 0;
        vcycle(h, r, s, 1, static_cast<long long>(h->N), st);
        if (hipStreamSynchronize(st) != hipSuccess) {
            h->prof = false;
            return SMG_EHIP;
        }
        for (int i = 0; i < h->ev_used; i += 2) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]) != hipSuccess) {
                h->prof = false;
                return SMG_EHIP;
            }
            const int row = by_level ? std::min(h->ev_lev[i / 2], nrows - 1) : 0;
            if (rep == 0) ++launches[row];
            kernel_ms[row] += ms / reps;
            bytes[row] += h->ev_bytes[i / 2] / reps;
        }
    }
    h->prof = false;
    return SMG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int smg_workspace_bytes(const smg_grid *g, const smg_opts *o, int32_t max_nrhs, size_t *bytes)
{
    if (check_grid(g, o) != SMG_OK || max_nrhs < 1 || !bytes) return SMG_EINVAL;
    try {
        const Tables t = build_tables(*g);
        const int E = (g->nx + 63) / 64;
        *bytes = make_layout(*g, *o, max_nrhs, t, 64 * E).total;
    } catch (...) {
        return SMG_EINVAL;
    }
    return SMG_OK;
}

int smg_setup(const smg_grid *g, const smg_opts *o, int32_t max_nrhs, void *ws, size_t ws_bytes, void *stream,
              smg_handle **out)
{
    if (!out) return SMG_EINVAL;
    *out = nullptr;
    if (check_grid(g, o) != SMG_OK || max_nrhs < 1 || !ws) return SMG_EINVAL;
    smg_handle *h = nullptr;
    try {
        h = new smg_handle();
        const int rc = fill_handle(h, g, o, max_nrhs, static_cast<char *>(ws), ws_bytes, as_stream(stream), true);
        if (rc != SMG_OK) {
            if (h->host_sc) (void)hipHostFree(h->host_sc);
            delete h;
            return rc;
        }
    } catch (const std::bad_alloc &) {
        delete h;
        return SMG_EINVAL;
    }
    *out = h;
    return SMG_OK;
}

int smg_apply_static(const smg_grid *g, const smg_opts *o, const double *r, double *s, int32_t nrhs, int64_t ld,
                     void *stream)
{
    if (check_grid(g, o) != SMG_OK || !r || !s || nrhs < 1) return SMG_EINVAL;
    if (ld < static_cast<int64_t>(g->nx) * g->ny * g->nz) return SMG_EINVAL;
    char *ws = nullptr;
    const int rc0 = static_scratch(&ws);
    if (rc0 != SMG_OK) return rc0;
    hipStream_t st = as_stream(stream);
    try {
        smg_handle h{};
        const int rc = fill_handle(&h, g, o, nrhs, ws, kStaticScratchBytes, st, false);
        if (rc != SMG_OK) return rc;
        vcycle(&h, r, s, nrhs, ld, st);
    } catch (const std::bad_alloc &) {
        return SMG_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? SMG_OK : SMG_EHIP;
}

int smg_apply(smg_handle *h, const double *r, double *s, int32_t nrhs, int64_t ld, void *stream)
{
    if (!h || !r || !s || nrhs < 1 || nrhs > h->max_nrhs || ld < static_cast<int64_t>(h->N)) return SMG_EINVAL;
    vcycle(h, r, s, nrhs, ld, as_stream(stream));
    return hipGetLastError() == hipSuccess ? SMG_OK : SMG_EHIP;
}

int smg_matvec(smg_handle *h, const double *x, double *y, int32_t nrhs, int64_t ld, void *stream)
{
    if (!h || !x || !y || nrhs < 1 || ld < static_cast<int64_t>(h->N) || nrhs > 65535) return SMG_EINVAL;
    if (h->var) {
        var_matvec(h->var, x, y, nrhs, ld, as_stream(stream));
        return hipGetLastError() == hipSuccess ? SMG_OK : SMG_EHIP;
    }
    launch_matvec7(x, y, ld, nrhs, h->g.nx, h->g.ny, h->g.nz, h->g.cx, h->g.cy, h->g.cz, as_stream(stream));
    return hipGetLastError() == hipSuccess ? SMG_OK : SMG_EHIP;
}

int pcg_solve(smg_handle *h, const double *b, double *x, const krylov_opts *o, krylov_info *info, void *stream)
{
    return krylov_run(h, 0, b, x, o, info, stream, nullptr);
}

int fpcg_solve(smg_handle *h, const double *b, double *x, const krylov_opts *o, krylov_info *info, void *stream)
{
    return krylov_run(h, 1, b, x, o, info, stream, nullptr);
}

int psd_solve(smg_handle *h, const double *b, double *x, const krylov_opts *o, krylov_info *info, void *stream)
{
    return krylov_run(h, 2, b, x, o, info, stream, nullptr);
}

// ---------------------------------------------------------------------------
// Variable coefficients
// ---------------------------------------------------------------------------
namespace {

int check_var(int32_t nx, int32_t ny, int32_t nz, const smg_opts *o, int32_t interp)
{
    if (!o || nx < 1 || ny < 1 || nz < 1 || nx > kMaxNx) return SMG_EINVAL;
    if (o->pre < 0 || o->post < 0 || o->pre > kMaxSmooth || o->post > kMaxSmooth) return SMG_EINVAL;
    if (o->inner_pre < -1 || o->inner_post < -1 || o->inner_pre > kMaxSmooth || o->inner_post > kMaxSmooth)
        return SMG_EINVAL;
    if (o->order != 0 && o->order != 1) return SMG_EINVAL;
    if (o->precision != SMG_PREC_F64) return SMG_EINVAL;
    if (interp != SMG_INTERP_LINEAR && interp != SMG_INTERP_OPERATOR) return SMG_EINVAL;
    return SMG_OK;
}

// Krylov vectors and scalars after the hierarchy
Layout var_krylov_layout(size_t base, size_t N)
{
    Layout L{};
    size_t off = base;
    auto take = [&](size_t b) {
        const size_t r = off;
        off = (off + b + 255) / 256 * 256;
        return r;
    };
    L.kr = take(N * 8);
    L.ks = take(N * 8);
    L.kp0 = take(N * 8);
    L.kp1 = take(N * 8);
    L.kq = take(N * 8);
    L.part = take(2 * kRedBlocks * 8);
    L.sc = take(sizeof(KScalars));
    L.total = off;
    return L;
}

}  // namespace

int smgv_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, const smg_opts *o, int32_t interp, int32_t max_nrhs,
                         size_t *bytes)
{
    if (check_var(nx, ny, nz, o, interp) != SMG_OK || max_nrhs < 1 || !bytes) return SMG_EINVAL;
    const size_t N = static_cast<size_t>(nx) * ny * nz;
    *bytes = var_krylov_layout(var_workspace_bytes(nx, ny, nz), N).total;
    return SMG_OK;
}

int smgv_setup(int32_t nx, int32_t ny, int32_t nz, const double *diag, const double *ax, const double *ay,
               const double *az, int32_t interp, const smg_opts *o, int32_t max_nrhs, void *ws, size_t ws_bytes,
               void *stream, smg_handle **out)
{
    if (!out) return SMG_EINVAL;
    *out = nullptr;
    if (check_var(nx, ny, nz, o, interp) != SMG_OK || max_nrhs < 1 || !ws || !diag || !ax || !ay || !az)
        return SMG_EINVAL;
    const size_t N = static_cast<size_t>(nx) * ny * nz;
    const Layout L = var_krylov_layout(var_workspace_bytes(nx, ny, nz), N);
    if (ws_bytes < L.total) return SMG_EWORKSPACE;
    hipStream_t st = as_stream(stream);
    smg_handle *h = new (std::nothrow) smg_handle();
    if (!h) return SMG_EINVAL;
    h->g = smg_grid{nx, ny, nz, 1.0, 1.0, 1.0};
    h->o = *o;
    h->ipre = o->inner_pre < 0 ? o->pre : o->inner_pre;
    h->ipost = o->inner_post < 0 ? o->post : o->inner_post;
    h->max_nrhs = max_nrhs;
    h->N = N;
    h->E = (nx + 63) / 64;
    h->nxp = 64 * h->E;
    h->fused = false;
    h->L = L;
    h->ws = static_cast<char *>(ws);
    h->prof = false;
    h->ev_used = 0;
    h->prof_bytes = 0;
    h->host_sc = nullptr;
    if (hipHostMalloc(reinterpret_cast<void **>(&h->host_sc), sizeof(KScalars), hipHostMallocDefault) != hipSuccess) {
        delete h;
        return SMG_EHIP;
    }
    h->var = var_create(nx, ny, nz, o, interp, h->ws, diag, ax, ay, az, st);
    if (!h->var || hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) {
        smg_destroy(h);
        return SMG_EHIP;
    }
    *out = h;
    return SMG_OK;
}

int smgv_levels(const smg_handle *h, int32_t *nlev3, int32_t *nlev2)
{
    if (!h || !h->var || !nlev3 || !nlev2) return SMG_EINVAL;
    int a = 0, b = 0;
    var_levels(h->var, &a, &b);
    *nlev3 = a;
    *nlev2 = b;
    return SMG_OK;
}

int smgv_export(smg_handle *h, int32_t level, int32_t level2, double *out, void *stream)
{
    if (!h || !h->var || !out) return SMG_EINVAL;
    const int rc = var_export(h->var, level, level2, out, as_stream(stream));
    if (rc != SMG_OK) return rc;
    return hipStreamSynchronize(as_stream(stream)) == hipSuccess ? SMG_OK : SMG_EHIP;
}

int smg_destroy(smg_handle *h)
{
    if (!h) return SMG_EINVAL;
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    if (h->host_sc) (void)hipHostFree(h->host_sc);
    if (h->var) var_destroy(h->var);
    delete h;
    return SMG_OK;
}

const char *smg_strerror(int status)
{
    switch (status) {
    case SMG_OK: return "ok";
    case SMG_NOT_CONVERGED: return "maximum number of iterations reached";
    case SMG_EINVAL: return "invalid argument";
    case SMG_EWORKSPACE: return "workspace too small";
    case SMG_EHIP: return "HIP runtime error";
    case SMG_EBREAKDOWN: return "breakdown: zero or non-finite denominator";
    case SMG_ENONFINITE: return "non-finite input";
    default: return "unknown status";
    }
}

int smg_set_march(smg_handle *h, int32_t march_waves)
{
    if (!h || march_waves < 0) return SMG_EINVAL;
    h->march_waves = march_waves;
    return SMG_OK;
}

int smg_get_schedule(const smg_handle *h, smg_tune_info *info)
{
    if (!h || !info) return SMG_EINVAL;
    *info = smg_tune_info{};
    info->l0 = h->l0;
    info->coarse_lds = static_cast<int64_t>(h->coarse_lds);
    info->s_down = h->S_down;
    info->s_up = h->S_up;
    info->march_waves = h->march_waves;
    return SMG_OK;
}

int smg_autotune(smg_handle *h, const double *r, double *s, int32_t reps, void *stream, smg_tune_info *info)
{
    if (!h || !r || !s || reps < 1 || h->var) return SMG_EINVAL;
    hipStream_t st = as_stream(stream);
    smg_tune_info inf{};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SMG_EHIP;
    // a schedule whose launches the device rejects (e.g. too much LDS) is not a candidate
    auto time_cycle = [&](double *ms) {
        (void)hipGetLastError();
        vcycle(h, r, s, 1, static_cast<long long>(h->N), st);   // warm-up (and LDS attributes)
        if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) return false;
        if (hipEventRecord(e0, st) != hipSuccess) return false;
        for (int i = 0; i < reps; ++i) vcycle(h, r, s, 1, static_cast<long long>(h->N), st);
        float t = 0.f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess)
            return false;
        *ms = t / reps;
        return true;
    };
    int rc = SMG_OK;
    double best = 0.0;
    size_t best_c = h->coarse_budget, best_s = h->strip_budget;
    if (!time_cycle(&best)) rc = SMG_EHIP;
    inf.default_ms = best;
    inf.candidates = 1;
    if (rc == SMG_OK && h->fused) {
        // candidate LDS budgets; budgets giving the same schedule are timed once
        const size_t cb[] = {16 << 10, 32 << 10, 64 << 10, 96 << 10, 128 << 10, 160 << 10};
        const size_t sb[] = {32 << 10, 48 << 10, 64 << 10, 96 << 10};
        const bool strips = h->nxp / 64 > 4;   // strip kernels only run on wide lines
        int dev = 0, max_lds = 64 << 10;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&max_lds, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess ||
            max_lds <= 0)
            max_lds = 64 << 10;
        std::vector<std::tuple<int, size_t, int, int>> seen;
        seen.emplace_back(h->l0, h->coarse_lds, h->S_down, h->S_up);
        for (size_t c : cb)
            for (size_t sbud : sb) {
                if (!strips && sbud != h->strip_budget) continue;
                if (c > static_cast<size_t>(max_lds) || sbud > static_cast<size_t>(max_lds)) continue;
                const size_t keep_c = h->coarse_budget, keep_s = h->strip_budget;
                apply_fused_schedule(h, c, sbud);
                const auto key = std::make_tuple(h->l0, h->coarse_lds, h->S_down, h->S_up);
                bool dup = !h->fused;
                for (const auto &k : seen) dup = dup || k == key;
                if (dup) {
                    apply_fused_schedule(h, keep_c, keep_s);
                    continue;
                }
                seen.push_back(key);
                double ms = 0.0;
                if (!time_cycle(&ms)) {
                    apply_fused_schedule(h, keep_c, keep_s);
                    continue;
                }
                ++inf.candidates;
                // a schedule replaces the current choice only if clearly faster (timing noise)
                if (ms < 0.98 * best) {
                    best = ms;
                    best_c = c;
                    best_s = sbud;
                }
                apply_fused_schedule(h, keep_c, keep_s);
            }
        apply_fused_schedule(h, best_c, best_s);
        // then the marching threshold of the register-only pre-smoothing
        // kernels (0: one wave per coarse line everywhere)
        const int cand_mw[] = {0, 1024, 2048, 4096, 8192};
        int best_mw = h->march_waves;
        const int keep_mw = h->march_waves;
        for (int mw : cand_mw) {
            if (mw == keep_mw) continue;
            h->march_waves = mw;
            double ms = 0.0;
            if (time_cycle(&ms)) {
                ++inf.candidates;
                if (ms < 0.98 * best) {
                    best = ms;
                    best_mw = mw;
                }
            }
        }
        h->march_waves = best_mw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    inf.best_ms = best;
    inf.l0 = h->l0;
    inf.coarse_lds = static_cast<int64_t>(h->coarse_lds);
    inf.s_down = h->S_down;
    inf.s_up = h->S_up;
    inf.march_waves = h->march_waves;
    if (info) *info = inf;
    return rc;
}

int smg_profile_kernel(smg_handle *h, int32_t family, const double *r, double *s, int32_t reps, void *stream,
                       int32_t *launches, double *kernel_ms, double *bytes)
{
    if (!h || !r || !s || reps < 1 || !launches || !kernel_ms || !bytes || h->var) return SMG_EINVAL;
    if (family < 0 || family >= SMG_KERNEL_COUNT) return SMG_EINVAL;
    const int nrows = 1;
    std::vector<int> cnt(nrows);
    std::vector<double> ms(nrows), by(nrows);
    const int rc =
        profile_run(h, family, false, r, s, reps, as_stream(stream), nrows, cnt.data(), ms.data(), by.data());
    if (rc != SMG_OK) return rc;
    *launches = cnt[0];
    *kernel_ms = ms[0];
    *bytes = by[0];
    return SMG_OK;
}

int smg_profile_levels(smg_handle *h, int32_t family, const double *r, double *s, int32_t reps, void *stream,
                       int32_t max_rows, int32_t *nrows, int32_t *launches, double *kernel_ms, double *bytes)
{
    if (!h || !r || !s || reps < 1 || !nrows || !launches || !kernel_ms || !bytes || h->var) return SMG_EINVAL;
    if (family < -1 || family >= SMG_KERNEL_COUNT) return SMG_EINVAL;
    const int rows = static_cast<int>(h->nz.size()) + 1;
    if (max_rows < rows) return SMG_EINVAL;
    *nrows = rows;
    return profile_run(h, family < 0 ? kProfAll : family, true, r, s, reps, as_stream(stream), rows, launches,
                       kernel_ms, bytes);
}

}  // extern "C"
