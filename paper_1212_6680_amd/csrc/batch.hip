// Batched flexible PCG (equation (2)) over many independent boxes.
//
// Each box keeps its own handle (hierarchy, Krylov vectors, scalars).  The
// launch sequence of one FPCG iteration is recorded per box with the same
// launch sites the single-box solver uses, the per-box sequences are merged
// into steps (a step runs one kernel for every box whose next launch is that
// kernel), and every step becomes ONE grouped launch over all its boxes (see
// group.h).  The stopping test runs on the device: a box that has converged
// clears its flag and its blocks return at once, so the iteration is a fixed
// launch sequence and is captured once as a HIP graph (two graphs: the two p
// buffers alternate between iterations) and replayed.  Per box, the kernels,
// their arguments and their order are those of fpcg_solve, so each box's
// iterates are bitwise those of its own single-box solve.
#include <limits>
#include <chrono>
#include <climits>
#include <cmath>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "group.h"
#include "smg_internal.h"

namespace smg {
thread_local std::vector<LaunchRec> *g_rec = nullptr;
thread_local int g_rec_unsupported = 0;
}  // namespace smg

using namespace smg;

namespace {

__global__ void k_count_active(KScalars *const *scs, int n, int *out)
{
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (scs[i]->active) atomicAdd(&cnt, 1);
    __syncthreads();
    if (threadIdx.x == 0) *out = cnt;
}

__global__ void k_gather_scalars(KScalars *const *scs, int n, KScalars *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = *scs[i];
}

struct Step {
    const void *kg;
    dim3 block;
    unsigned lds;
    int nent;
    int total;
    size_t tab;     // index of the first GroupEntry in the table buffer
};

struct Program {
    std::vector<Step> steps;
    std::vector<GroupEntry> entries;
};

// Greedy merge of per-box launch sequences into steps; a box's own order is
// kept.  Each step takes the kernel with the largest vote among the boxes'
// next launches, a box voting with weight (remaining launches)^power: power
// 0 is a plain majority, higher powers favour the longest remaining
// sequences (the critical path).  Launches of one kernel with different
// dynamic LDS sizes share a step, which requests the largest (every kernel
// derives its LDS layout from its own arguments).
bool merge_with(const std::vector<std::vector<LaunchRec>> &seqs, int power, Program &prog)
{
    const size_t nb = seqs.size();
    std::vector<size_t> pos(nb, 0);
    auto key = [](const LaunchRec &r) { return std::make_tuple(r.kg, r.block.x, r.block.y, r.block.z); };
    using Key = decltype(key(LaunchRec{}));
    for (;;) {
        std::map<Key, double> votes;
        Key first{};
        bool any = false;
        for (size_t i = 0; i < nb; ++i) {
            if (pos[i] >= seqs[i].size()) continue;
            const Key k = key(seqs[i][pos[i]]);
            if (!any) first = k;
            any = true;
            votes[k] += std::pow(static_cast<double>(seqs[i].size() - pos[i]), power);
        }
        if (!any) break;
        Key best = first;   // ties: the first box's next launch (deterministic)
        for (const auto &kv : votes)
            if (kv.second > votes[best]) best = kv.first;
        Step st{};
        st.tab = prog.entries.size();
        long long total = 0;
        for (size_t i = 0; i < nb; ++i) {
            if (pos[i] >= seqs[i].size() || key(seqs[i][pos[i]]) != best) continue;
            const LaunchRec &r = seqs[i][pos[i]++];
            const long long nblk = static_cast<long long>(r.grid.x) * r.grid.y * r.grid.z;
            if (nblk == 0) continue;
            GroupEntry e{};
            e.start = static_cast<int>(total);
            e.gx = static_cast<int>(r.grid.x);
            e.gy = static_cast<int>(r.grid.y);
            e.gz = static_cast<int>(r.grid.z);
            e.active = r.active;
            std::memcpy(e.args, r.args.data(), kGroupArgBytes);
            prog.entries.push_back(e);
            st.kg = r.kg;
            st.block = r.block;
            st.lds = r.lds > st.lds ? r.lds : st.lds;
            total += nblk;
            if (total > INT_MAX) return false;
        }
        st.nent = static_cast<int>(prog.entries.size() - st.tab);
        st.total = static_cast<int>(total);
        if (st.nent > 0) prog.steps.push_back(st);
    }
    return true;
}

// The merge with the fewest steps over a few vote weightings.
bool merge(const std::vector<std::vector<LaunchRec>> &seqs, Program &prog)
{
    bool found = false;
    for (int power = 0; power <= 3; ++power) {
        Program p;
        if (!merge_with(seqs, power, p)) continue;
        if (!found || p.steps.size() < prog.steps.size()) prog = std::move(p);
        found = true;
    }
    return found;
}

}  // namespace

struct smg_batch {
    int nbox = 0;
    std::vector<smg_handle *> hs;
    std::vector<KrylovView> kv;
    std::vector<const double *> b;
    std::vector<double *> x;
    Program iter[2];            // FPCG iteration with p buffers (pa -> pb) and (pb -> pa)
    size_t iter_off[2] = {0, 0};
    char *ws = nullptr;
    size_t ws_bytes = 0;
    size_t tab_off = 0, tab_bytes = 0;      // iteration tables
    size_t aux_off = 0, aux_bytes = 0;      // per-solve tables (start, end)
    size_t scs_off = 0, cnt_off = 0, gath_off = 0;
    hipStream_t pst = nullptr;  // private stream: graphs cannot capture the legacy default stream
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int use_graph = 0;
    int *host_cnt = nullptr;
    KScalars *host_sc = nullptr;
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

// Records fn(i) for every box with the recorder installed.
template <typename F>
bool record_boxes(int nbox, std::vector<std::vector<LaunchRec>> &seqs, F &&fn)
{
    seqs.assign(nbox, {});
    g_rec_unsupported = 0;
    for (int i = 0; i < nbox; ++i) {
        g_rec = &seqs[i];
        fn(i);
        g_rec = nullptr;
    }
    return g_rec_unsupported == 0;
}

int check_boxes(smg_handle *const *hs, int nbox, std::vector<KrylovView> &kv)
{
    if (!hs || nbox < 1) return SMG_EINVAL;
    kv.resize(nbox);
    for (int i = 0; i < nbox; ++i) {
        if (!hs[i] || smg_handle_is_var(hs[i]) || krylov_view(hs[i], &kv[i]) != SMG_OK) return SMG_EINVAL;
        if (kv[i].precision != SMG_PREC_F64) return SMG_EINVAL;
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return SMG_EINVAL;
    }
    return SMG_OK;
}

// Per-box launch sequence of one FPCG iteration (fpcg_solve's loop body).
void iteration_launches(smg_handle *h, const KrylovView &v, double *x, int parity, hipStream_t st)
{
    double *pa = parity ? v.pb : v.pa, *pb = parity ? v.pa : v.pb;
    const smg_grid &g = v.g;
    const double *dp = v.part;
    int np = 0;
    if (!vcycle_dots(h, v.r, v.s, v.q, 1, st, &dp, &np)) {
        dp = v.part;
        np = 0;
        launch_dots_sr_sq(v.s, v.r, v.q, 1, v.n, v.part, st);
    }
    launch_finalize_batched(1, 1, dp, v.sc, 0.0, 0, st, np);
    launch_update_p_q(v.s, pa, pb, v.q, v.sc, g.nx, g.ny, g.nz, g.cx, g.cy, g.cz, v.part, st);
    launch_finalize_batched(2, 1, v.part, v.sc, 0.0, 0, st);
    launch_update_xr(x, v.r, pb, v.q, v.sc, v.n, v.part, st);
    launch_finalize_batched(3, 1, v.part, v.sc, 0.0, 0, st);
}

bool build_iteration(smg_batch *bt, int parity, Program &prog)
{
    std::vector<std::vector<LaunchRec>> seqs;
    if (!record_boxes(bt->nbox, seqs, [&](int i) { iteration_launches(bt->hs[i], bt->kv[i], bt->x[i], parity, nullptr); }))
        return false;
    for (int i = 0; i < bt->nbox; ++i)
        for (auto &r : seqs[i]) r.active = &bt->kv[i].sc->active;
    prog = Program{};
    return merge(seqs, prog);
}

hipError_t launch_program(const Program &prog, const GroupEntry *dtab, hipStream_t st)
{
    for (const Step &s : prog.steps) {
        const GroupEntry *tab = dtab + s.tab;
        int n = s.nent;
        void *args[] = {&tab, &n};
        const hipError_t e = hipLaunchKernel(s.kg, dim3(static_cast<unsigned>(s.total)), s.block, args, s.lds, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int smg_batch_workspace_bytes(smg_handle *const *hs, int32_t nbox, size_t *bytes)
{
    if (!bytes) return SMG_EINVAL;
    smg_batch tmp;
    if (check_boxes(hs, nbox, tmp.kv) != SMG_OK) return SMG_EINVAL;
    tmp.nbox = nbox;
    tmp.hs.assign(hs, hs + nbox);
    tmp.x.assign(nbox, nullptr);
    size_t tab = 0, maxe = 0;
    for (int p = 0; p < 2; ++p) {
        if (!build_iteration(&tmp, p, tmp.iter[p])) return SMG_EINVAL;
        tab += align256(tmp.iter[p].entries.size() * sizeof(GroupEntry));
    }
    // start and end sequences: at most 4 launches per box each
    maxe = static_cast<size_t>(nbox) * 8;
    *bytes = tab + align256(maxe * sizeof(GroupEntry)) + align256(nbox * sizeof(KScalars *)) + 256 +
             align256(nbox * sizeof(KScalars));
    return SMG_OK;
}

int smg_batch_create(smg_handle *const *hs, int32_t nbox, const double *const *b, double *const *x, void *ws,
                     size_t ws_bytes, int32_t use_graph, void *stream, smg_batch **out)
{
    if (!out) return SMG_EINVAL;
    *out = nullptr;
    if (!b || !x || !ws || (use_graph != 0 && use_graph != 1)) return SMG_EINVAL;
    size_t need = 0;
    const int rc = smg_batch_workspace_bytes(hs, nbox, &need);
    if (rc != SMG_OK) return rc;
    if (ws_bytes < need) return SMG_EWORKSPACE;
    for (int i = 0; i < nbox; ++i)
        if (!b[i] || !x[i]) return SMG_EINVAL;
    smg_batch *bt = new (std::nothrow) smg_batch();
    if (!bt) return SMG_EHIP;
    bt->nbox = nbox;
    bt->hs.assign(hs, hs + nbox);
    check_boxes(hs, nbox, bt->kv);
    bt->b.assign(b, b + nbox);
    bt->x.assign(x, x + nbox);
    bt->ws = static_cast<char *>(ws);
    bt->ws_bytes = ws_bytes;
    bt->use_graph = use_graph;
    auto fail = [&](int code) {
        smg_batch_destroy(bt);
        return code;
    };
    size_t off = 0;
    for (int p = 0; p < 2; ++p) {
        if (!build_iteration(bt, p, bt->iter[p])) return fail(SMG_EINVAL);
        bt->iter_off[p] = off;
        off += align256(bt->iter[p].entries.size() * sizeof(GroupEntry));
    }
    bt->aux_off = off;
    bt->aux_bytes = align256(static_cast<size_t>(nbox) * 8 * sizeof(GroupEntry));
    off += bt->aux_bytes;
    bt->scs_off = off;
    off += align256(nbox * sizeof(KScalars *));
    bt->cnt_off = off;
    off += 256;
    bt->gath_off = off;
    off += align256(nbox * sizeof(KScalars));
    if (off > ws_bytes) return fail(SMG_EWORKSPACE);

    hipStream_t cst = static_cast<hipStream_t>(stream);
    if (hipStreamCreateWithFlags(&bt->pst, hipStreamNonBlocking) != hipSuccess) return fail(SMG_EHIP);
    if (hipEventCreateWithFlags(&bt->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&bt->ev_out, hipEventDisableTiming) != hipSuccess)
        return fail(SMG_EHIP);
    if (hipHostMalloc(reinterpret_cast<void **>(&bt->host_cnt), sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&bt->host_sc), nbox * sizeof(KScalars), hipHostMallocDefault) !=
            hipSuccess)
        return fail(SMG_EHIP);
    // tables and the per-box scalar pointers
    std::vector<KScalars *> scs(nbox);
    for (int i = 0; i < nbox; ++i) scs[i] = bt->kv[i].sc;
    if (hipEventRecord(bt->ev_in, cst) != hipSuccess || hipStreamWaitEvent(bt->pst, bt->ev_in, 0) != hipSuccess)
        return fail(SMG_EHIP);
    for (int p = 0; p < 2; ++p)
        if (!bt->iter[p].entries.empty() &&
            hipMemcpyAsync(bt->ws + bt->iter_off[p], bt->iter[p].entries.data(),
                           bt->iter[p].entries.size() * sizeof(GroupEntry), hipMemcpyHostToDevice,
                           bt->pst) != hipSuccess)
            return fail(SMG_EHIP);
    if (hipMemcpyAsync(bt->ws + bt->scs_off, scs.data(), nbox * sizeof(KScalars *), hipMemcpyHostToDevice,
                       bt->pst) != hipSuccess ||
        hipStreamSynchronize(bt->pst) != hipSuccess)
        return fail(SMG_EHIP);
    if (use_graph) {
        for (int p = 0; p < 2; ++p) {
            hipGraph_t graph = nullptr;
            if (hipStreamBeginCapture(bt->pst, hipStreamCaptureModeThreadLocal) != hipSuccess) return fail(SMG_EHIP);
            const hipError_t le = launch_program(bt->iter[p],
                                                 reinterpret_cast<const GroupEntry *>(bt->ws + bt->iter_off[p]),
                                                 bt->pst);
            const hipError_t ce = hipStreamEndCapture(bt->pst, &graph);
            if (le != hipSuccess || ce != hipSuccess || !graph) {
                if (graph) (void)hipGraphDestroy(graph);
                return fail(SMG_EHIP);
            }
            const hipError_t ie = hipGraphInstantiate(&bt->gexec[p], graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) return fail(SMG_EHIP);
        }
    }
    *out = bt;
    return SMG_OK;
}

int smg_batch_fpcg(smg_batch *bt, const krylov_opts *o, krylov_info *infos, void *stream)
{
    if (!bt || !o || !infos) return SMG_EINVAL;
    if (o->max_iter < 0 || !(o->rtol >= 0.0) || o->precond != SMG_PRECOND_SMG || o->history || o->history_c ||
        o->stop_norm != SMG_STOP_2NORM || o->xstar || o->err_a || o->sin_angle)
        return SMG_EINVAL;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t cst = static_cast<hipStream_t>(stream);
    hipStream_t st = bt->pst;
    const int nbox = bt->nbox;
    KScalars *const *dscs = reinterpret_cast<KScalars *const *>(bt->ws + bt->scs_off);
    int *dcnt = reinterpret_cast<int *>(bt->ws + bt->cnt_off);
    KScalars *dgath = reinterpret_cast<KScalars *>(bt->ws + bt->gath_off);
    const GroupEntry *daux = reinterpret_cast<const GroupEntry *>(bt->ws + bt->aux_off);
    if (hipEventRecord(bt->ev_in, cst) != hipSuccess || hipStreamWaitEvent(st, bt->ev_in, 0) != hipSuccess)
        return SMG_EHIP;

    // start: x = 0 (x0_zero), q = 0, r = b - A x, the recurrence state and the stopping test
    std::vector<std::vector<LaunchRec>> seqs;
    record_boxes(nbox, seqs, [&](int i) {
        const KrylovView &v = bt->kv[i];
        const smg_grid &g = v.g;
        if (o->x0_zero) launch_fill(bt->x[i], 0.0, v.n, st);
        launch_fill(v.q, 0.0, v.n, st);
        launch_init_resid(bt->b[i], bt->x[i], v.r, o->x0_zero ? 1 : 0, g.nx, g.ny, g.nz, g.cx, g.cy, g.cz, v.part,
                          st);
        launch_finalize_batched(0, 1, v.part, v.sc, o->rtol, o->max_iter, st);
    });
    Program start;
    if (!merge(seqs, start) || start.entries.size() * sizeof(GroupEntry) > bt->aux_bytes) return SMG_EINVAL;
    if (hipMemcpyAsync(bt->ws + bt->aux_off, start.entries.data(), start.entries.size() * sizeof(GroupEntry),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        launch_program(start, daux, st) != hipSuccess)
        return SMG_EHIP;

    // iterations: replay until no box is active
    for (int it = 0; it < o->max_iter; ++it) {
        const int p = it & 1;
        hipError_t e;
        if (bt->use_graph)
            e = hipGraphLaunch(bt->gexec[p], st);
        else
            e = launch_program(bt->iter[p], reinterpret_cast<const GroupEntry *>(bt->ws + bt->iter_off[p]), st);
        if (e != hipSuccess) return SMG_EHIP;
        hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, st, dscs, nbox, dcnt);
        if (hipMemcpyAsync(bt->host_cnt, dcnt, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return SMG_EHIP;
        if (*bt->host_cnt == 0) break;
    }

    // end: true residuals (s is free scratch here), then every box's scalars
    record_boxes(nbox, seqs, [&](int i) {
        const KrylovView &v = bt->kv[i];
        const smg_grid &g = v.g;
        launch_true_resid(bt->b[i], bt->x[i], v.s, g.nx, g.ny, g.nz, g.cx, g.cy, g.cz, v.part, st);
        launch_finalize_batched(4, 1, v.part, v.sc, 0.0, 0, st);
    });
    Program fin;
    if (!merge(seqs, fin) || fin.entries.size() * sizeof(GroupEntry) > bt->aux_bytes) return SMG_EINVAL;
    if (hipMemcpyAsync(bt->ws + bt->aux_off, fin.entries.data(), fin.entries.size() * sizeof(GroupEntry),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        launch_program(fin, daux, st) != hipSuccess)
        return SMG_EHIP;
    hipLaunchKernelGGL(k_gather_scalars, dim3((nbox + 63) / 64), dim3(64), 0, st, dscs, nbox, dgath);
    if (hipMemcpyAsync(bt->host_sc, dgath, nbox * sizeof(KScalars), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess)
        return SMG_EHIP;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int worst = SMG_OK;
    for (int i = 0; i < nbox; ++i) {
        const KScalars &s = bt->host_sc[i];
        krylov_info &inf = infos[i];
        const double bn = std::sqrt(s.bb);
        const double bden = bn > 0.0 ? bn : 1.0;
        inf.iters = s.iters;
        inf.rel_res = std::sqrt(s.rr) / bden;
        inf.true_rel_res = std::sqrt(s.true_rr) / bden;
        inf.solve_seconds = secs;
        inf.rel_res_c = std::numeric_limits<double>::quiet_NaN();
        if (s.nonfinite)
            inf.status = SMG_ENONFINITE;
        else if (s.breakdown || !std::isfinite(inf.rel_res))
            inf.status = SMG_EBREAKDOWN;
        else
            inf.status = inf.rel_res <= o->rtol ? SMG_OK : SMG_NOT_CONVERGED;
        if (inf.status < 0 ? (worst >= 0 || inf.status < worst) : (worst == SMG_OK && inf.status != SMG_OK))
            worst = inf.status;
    }
    if (hipEventRecord(bt->ev_out, st) != hipSuccess || hipStreamWaitEvent(cst, bt->ev_out, 0) != hipSuccess)
        return SMG_EHIP;
    return worst;
}

int smg_batch_stats(const smg_batch *bt, int32_t *steps_per_iteration, int32_t *launches_per_iteration)
{
    if (!bt) return SMG_EINVAL;
    if (steps_per_iteration) *steps_per_iteration = static_cast<int32_t>(bt->iter[0].steps.size());
    if (launches_per_iteration) *launches_per_iteration = static_cast<int32_t>(bt->iter[0].entries.size());
    return SMG_OK;
}

int smg_batch_destroy(smg_batch *bt)
{
    if (!bt) return SMG_OK;
    for (int p = 0; p < 2; ++p)
        if (bt->gexec[p]) (void)hipGraphExecDestroy(bt->gexec[p]);
    if (bt->ev_in) (void)hipEventDestroy(bt->ev_in);
    if (bt->ev_out) (void)hipEventDestroy(bt->ev_out);
    if (bt->pst) (void)hipStreamDestroy(bt->pst);
    if (bt->host_cnt) (void)hipHostFree(bt->host_cnt);
    if (bt->host_sc) (void)hipHostFree(bt->host_sc);
    delete bt;
    return SMG_OK;
}

}  // extern "C"
