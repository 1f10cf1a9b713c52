// Host side of the learned post-smoother: workspace layout, forward and
// backward schedules, Adam, training loop, training-pair generation and the
// flexible-PCG correction hook.
#include <cmath>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "net_internal.h"

using namespace smg;
using namespace smg::net;

namespace {

constexpr int kCin[4] = {1, 16, 16, 16};
constexpr int kCout[4] = {16, 16, 16, 1};
constexpr int kLossRing = 1024;

LayerTable layer_table()
{
    LayerTable lt{};
    int off = 0;
    for (int l = 0; l < 4; ++l) {
        lt.off[l] = off;
        lt.cin[l] = kCin[l];
        lt.cout[l] = kCout[l];
        off += 27 * kCin[l] * kCout[l] + kCout[l];
    }
    lt.off[4] = off;
    lt.total = off;
    return lt;
}

hipStream_t as_st(void *s) { return static_cast<hipStream_t>(s); }

struct NetLayout {
    size_t p, wst, wtr, frag, ns, part, rp, sl, a1, a2;          // inference
    size_t a3, g0, g1, y, g4, grad, m, v, wpart, loss, b, xp, xs;  // training
    size_t total;
};

NetLayout make_net_layout(long long nvox, int prec, int train)
{
    const size_t es = prec == NET_PREC_BF16 ? 2 : 8;   // storage element
    const size_t ea = prec == NET_PREC_BF16 ? 4 : 8;   // accum element
    const size_t n = static_cast<size_t>(nvox);
    NetLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~static_cast<size_t>(255);
        return o;
    };
    L.p = take(NET_NPARAMS * ea);
    L.wst = take(NET_NPARAMS * es);
    L.wtr = take(NET_NPARAMS * es);
    L.frag = take(prec == NET_PREC_BF16 ? 4 * 14 * 64 * 8 * 2 : 0);
    L.ns = take(sizeof(NetScalars));
    L.part = take(2 * kRedBlocks * sizeof(double));
    L.rp = take(n * 8);
    L.sl = take(n * 8);
    L.a1 = take(16 * n * es);
    L.a2 = take(16 * n * es);
    if (train) {
        L.a3 = take(16 * n * es);
        L.g0 = take(16 * n * es);
        L.g1 = take(16 * n * es);
        L.y = take(n * ea);
        L.g4 = take(n * es);
        L.grad = take(NET_NPARAMS * ea);
        L.m = take(NET_NPARAMS * ea);
        L.v = take(NET_NPARAMS * ea);
        L.wpart = take(static_cast<size_t>(kWgradBlocks) * (27 * 16 * 16 + 16) * ea);
        L.loss = take(kLossRing * sizeof(double));
        L.b = take(n * 8);
        L.xp = take(n * 8);
        L.xs = take(n * 8);
    }
    L.total = off;
    return L;
}

}  // namespace

struct net_handle {
    int prec = 0, train = 0;
    long long max_vox = 0;
    char *ws = nullptr;
    NetLayout L{};
    LayerTable lt{};
    long long adam_t = 0;
    bool have_grad = false;
    template <typename P> P *at(size_t off) const { return reinterpret_cast<P *>(ws + off); }
};

namespace {

template <typename T, typename A>
struct Impl {
    static constexpr bool kMfma = std::is_same<T, bf16>::value;

    static A *p(net_handle *n) { return n->at<A>(n->L.p); }
    static T *wst(net_handle *n) { return n->at<T>(n->L.wst); }
    static T *wtr(net_handle *n) { return n->at<T>(n->L.wtr); }
    static const uint16_t *frag(net_handle *n, int layer, int bwd)
    {
        return n->at<uint16_t>(n->L.frag) + ((layer - 1) * 2 + bwd) * (14 * 64 * 8);
    }
    static const A *bias(net_handle *n, int l) { return p(n) + n->lt.off[l] + 27 * kCin[l] * kCout[l]; }

    static ConvVecArgs<T, A> cargs(int nx, int ny, int nz)
    {
        ConvVecArgs<T, A> c{};
        c.nx = nx;
        c.ny = ny;
        c.nz = nz;
        return c;
    }

    static void pack(net_handle *n, hipStream_t st)
    {
        launch_pack<T, A>(p(n), wst(n), wtr(n), n->lt, st);
        if constexpr (kMfma) {
            for (int l = 1; l <= 2; ++l)
                for (int bwd = 0; bwd < 2; ++bwd)
                    launch_pack_frag(reinterpret_cast<const float *>(p(n)), n->lt.off[l], bwd,
                                     n->at<uint16_t>(n->L.frag) + ((l - 1) * 2 + bwd) * (14 * 64 * 8), st);
        }
    }

    // bf16 1 -> 16 layer: layer 0 (which = 0, bias + ReLU) or the input
    // gradient of layer 3 (which = 1, masked)
    static void in16(net_handle *n, int which, const T *in, const double *in64, const NetScalars *ns,
                     const T *mask, T *out, int nx, int ny, int nz, hipStream_t st)
    {
        if constexpr (kMfma) {
            In16Args a{};
            a.in = in;
            a.in64 = in64;
            a.ns = ns;
            // [27][16] weights: layer 0 forward, or layer 3's flipped transpose (input gradient)
            a.w = which == 0 ? wst(n) + n->lt.off[0] : wtr(n) + n->lt.off[3];
            a.bias = which == 0 ? bias(n, 0) : nullptr;
            a.mask = mask;
            a.out = out;
            a.nx = nx;
            a.ny = ny;
            a.nz = nz;
            launch_in16_bf16(a, in64 ? 1 : 0, which, st);
        }
    }

    // bf16 16 -> 1 layer 3: y (EPI 2) or s_out = s_in + out_scale (acc + b) (EPI 3)
    static void out16(net_handle *n, const T *in, A *y, const NetScalars *ns, const double *s_in, double *s_out,
                      int nx, int ny, int nz, hipStream_t st)
    {
        if constexpr (kMfma) {
            Out16Args a{};
            a.in = in;
            a.w = reinterpret_cast<const unsigned int *>(wst(n) + n->lt.off[3]);
            a.bias = bias(n, 3);
            a.ns = ns;
            a.outA = y;
            a.s_in = s_in;
            a.s_out = s_out;
            a.nx = nx;
            a.ny = ny;
            a.nz = nz;
            launch_out16_bf16(a, s_out ? 3 : 2, st);
        }
    }

    // hidden 16 -> 16 layer l (1 or 2): out = relu(conv(in) + b)
    static void hidden(net_handle *n, int l, const T *in, T *out, int nx, int ny, int nz, hipStream_t st)
    {
        if constexpr (kMfma) {
            Conv16Args a{};
            a.in = in;
            a.frag = frag(n, l, 0);
            a.bias = bias(n, l);
            a.out = out;
            a.nx = nx;
            a.ny = ny;
            a.nz = nz;
            launch_conv16_mfma(a, 0, st);
        } else {
            auto c = cargs(nx, ny, nz);
            c.in = in;
            c.W = wst(n) + n->lt.off[l];
            c.bias = bias(n, l);
            c.out = out;
            launch_conv_vec<T, A, 16, 16, 0, 0>(c, st);
        }
    }

    // input gradient of hidden layer l, masked by (mask > 0)
    static void hidden_dgrad(net_handle *n, int l, const T *g, const T *mask, T *out, int nx, int ny, int nz,
                             hipStream_t st)
    {
        if constexpr (kMfma) {
            Conv16Args a{};
            a.in = g;
            a.frag = frag(n, l, 1);
            a.mask = mask;
            a.out = out;
            a.nx = nx;
            a.ny = ny;
            a.nz = nz;
            launch_conv16_mfma(a, 1, st);
        } else {
            auto c = cargs(nx, ny, nz);
            c.in = g;
            c.W = wtr(n) + n->lt.off[l];
            c.mask = mask;
            c.out = out;
            launch_conv_vec<T, A, 16, 16, 0, 1>(c, st);
        }
    }

    static void layer0(net_handle *n, const T *in, T *out, int nx, int ny, int nz, hipStream_t st)
    {
        if constexpr (kMfma) {
            in16(n, 0, in, nullptr, nullptr, nullptr, out, nx, ny, nz, st);
        } else {
            auto c = cargs(nx, ny, nz);
            c.in = in;
            c.W = wst(n) + n->lt.off[0];
            c.bias = bias(n, 0);
            c.out = out;
            launch_conv_vec<T, A, 1, 16, 0, 0>(c, st);
        }
    }

    static void layer3(net_handle *n, const T *in, A *y, int nx, int ny, int nz, hipStream_t st)
    {
        if constexpr (kMfma) {
            out16(n, in, y, nullptr, nullptr, nullptr, nx, ny, nz, st);
        } else {
            auto c = cargs(nx, ny, nz);
            c.in = in;
            c.W = wst(n) + n->lt.off[3];
            c.bias = bias(n, 3);
            c.outA = y;
            launch_conv_vec<T, A, 16, 1, 0, 2>(c, st);
        }
    }

    static int layer_forward(net_handle *n, int layer, int nx, int ny, int nz, const void *in, void *out,
                             hipStream_t st)
    {
        const T *ti = static_cast<const T *>(in);
        if (layer == 0) layer0(n, ti, static_cast<T *>(out), nx, ny, nz, st);
        else if (layer == 3) layer3(n, ti, static_cast<A *>(out), nx, ny, nz, st);
        else hidden(n, layer, ti, static_cast<T *>(out), nx, ny, nz, st);
        return SMG_OK;
    }

    // forward (keeping activations) + loss + backward; gradient into L.grad
    static void loss_grad(net_handle *n, int nx, int ny, int nz, const T *a0, const A *target, int kind,
                          double *loss_dev, hipStream_t st)
    {
        T *a1 = n->at<T>(n->L.a1), *a2 = n->at<T>(n->L.a2), *a3 = n->at<T>(n->L.a3);
        T *g0 = n->at<T>(n->L.g0), *g1 = n->at<T>(n->L.g1), *g4 = n->at<T>(n->L.g4);
        A *y = n->at<A>(n->L.y), *grad = n->at<A>(n->L.grad), *wpart = n->at<A>(n->L.wpart);
        layer0(n, a0, a1, nx, ny, nz, st);
        hidden(n, 1, a1, a2, nx, ny, nz, st);
        hidden(n, 2, a2, a3, nx, ny, nz, st);
        layer3(n, a3, y, nx, ny, nz, st);
        launch_loss<T, A>(kind, y, target, g4, nx, ny, nz, n->at<double>(n->L.part), loss_dev, st);

        WgradArgs<T, A> w{};
        w.part = wpart;
        w.nx = nx;
        w.ny = ny;
        w.nz = nz;
        w.in = a3;
        w.g = g4;
        launch_wgrad<T, A, 16, 1>(w, grad + n->lt.off[3], st);
        if constexpr (kMfma) {
            in16(n, 1, g4, nullptr, nullptr, a3, g0, nx, ny, nz, st);
        } else {
            auto c = cargs(nx, ny, nz);
            c.in = g4;
            c.W = wtr(n) + n->lt.off[3];
            c.mask = a3;
            c.out = g0;
            launch_conv_vec<T, A, 1, 16, 0, 1>(c, st);
        }
        w.in = a2;
        w.g = g0;
        launch_wgrad<T, A, 16, 16>(w, grad + n->lt.off[2], st);
        hidden_dgrad(n, 2, g0, a2, g1, nx, ny, nz, st);
        w.in = a1;
        w.g = g1;
        launch_wgrad<T, A, 16, 16>(w, grad + n->lt.off[1], st);
        hidden_dgrad(n, 1, g1, a1, g0, nx, ny, nz, st);
        w.in = a0;
        w.g = g0;
        launch_wgrad<T, A, 1, 16>(w, grad + n->lt.off[0], st);
    }

    static void adam(net_handle *n, double lr, hipStream_t st)
    {
        const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
        n->adam_t += 1;
        const double bc1 = 1.0 - std::pow(b1, static_cast<double>(n->adam_t));
        const double bc2 = 1.0 - std::pow(b2, static_cast<double>(n->adam_t));
        launch_adam<A>(p(n), n->at<A>(n->L.m), n->at<A>(n->L.v), n->at<A>(n->L.grad), NET_NPARAMS, lr, b1, b2, eps,
                       bc1, bc2, st);
        pack(n, st);
    }

    // out = s + sigma * N(r'/(cbar sigma)), r' = r - A s
    static void correct(net_handle *n, const smg_grid &g, const double *r, const double *s, double *out,
                        hipStream_t st)
    {
        const int nx = g.nx, ny = g.ny, nz = g.nz;
        const long long N = static_cast<long long>(nx) * ny * nz;
        double *rp = n->at<double>(n->L.rp), *part = n->at<double>(n->L.part);
        NetScalars *ns = n->at<NetScalars>(n->L.ns);
        T *a1 = n->at<T>(n->L.a1), *a2 = n->at<T>(n->L.a2);
        launch_init_resid(r, s, rp, 0, nx, ny, nz, g.cx, g.cy, g.cz, part, st);
        launch_net_scalars(part, kRedBlocks, (g.cx + g.cy + g.cz) / 3.0, static_cast<double>(N), ns, st);
        if constexpr (kMfma) {
            in16(n, 0, nullptr, rp, ns, nullptr, a1, nx, ny, nz, st);
        } else {
            auto c = cargs(nx, ny, nz);
            c.in64 = rp;
            c.ns = ns;
            c.W = wst(n) + n->lt.off[0];
            c.bias = bias(n, 0);
            c.out = a1;
            launch_conv_vec<T, A, 1, 16, 1, 0>(c, st);
        }
        hidden(n, 1, a1, a2, nx, ny, nz, st);
        hidden(n, 2, a2, a1, nx, ny, nz, st);
        if constexpr (kMfma) {
            out16(n, a1, nullptr, ns, s, out, nx, ny, nz, st);
        } else {
            auto d = cargs(nx, ny, nz);
            d.in = a1;
            d.ns = ns;
            d.W = wst(n) + n->lt.off[3];
            d.bias = bias(n, 3);
            d.s_in = s;
            d.s_out = out;
            launch_conv_vec<T, A, 16, 1, 0, 3>(d, st);
        }
    }

    static void pair_store(net_handle *n, long long N, void *inputs, void *targets, long long i, hipStream_t st)
    {
        launch_pair_store<T, A>(n->at<double>(n->L.rp), n->at<double>(n->L.xs), n->at<double>(n->L.xp),
                                n->at<NetScalars>(n->L.ns), static_cast<T *>(inputs) + i * N,
                                static_cast<A *>(targets) + i * N, N, st);
    }

    static int train(net_handle *n, int nx, int ny, int nz, const void *inputs, const void *targets, int steps,
                     const int32_t *order, const double *lr, int kind, double *hist, hipStream_t st)
    {
        const long long N = static_cast<long long>(nx) * ny * nz;
        double *ring = n->at<double>(n->L.loss);
        int flushed = 0;
        for (int k = 0; k < steps; ++k) {
            const long long i = order[k];
            loss_grad(n, nx, ny, nz, static_cast<const T *>(inputs) + i * N, static_cast<const A *>(targets) + i * N,
                      kind, ring + (k % kLossRing), st);
            adam(n, lr[k], st);
            if ((k + 1) % kLossRing == 0 || k + 1 == steps) {
                const int cnt = k + 1 - flushed;
                if (hist && hipMemcpyAsync(hist + flushed, ring, cnt * sizeof(double), hipMemcpyDeviceToHost, st) !=
                                hipSuccess)
                    return SMG_EHIP;
                if (hipStreamSynchronize(st) != hipSuccess) return SMG_EHIP;
                flushed = k + 1;
            }
        }
        n->have_grad = steps > 0;
        return hipGetLastError() == hipSuccess ? SMG_OK : SMG_EHIP;
    }
};

template <typename F>
int dispatch(net_handle *n, F &&f)
{
    if (n->prec == NET_PREC_BF16) return f(Impl<bf16, float>{});
    return f(Impl<double, double>{});
}

bool grid_ok(const net_handle *n, int nx, int ny, int nz)
{
    if (nx < 1 || ny < 1 || nz < 1) return false;
    return static_cast<long long>(nx) * ny * nz <= n->max_vox;
}

struct HookCtx {
    net_handle *n;
    smg_handle *h;
};

const double *hook_apply(void *ctx, const double *r, const double *s, hipStream_t st)
{
    HookCtx *c = static_cast<HookCtx *>(ctx);
    net_handle *n = c->n;
    double *out = n->at<double>(n->L.sl);
    const smg_grid &g = *smg_handle_grid(c->h);
    dispatch(n, [&](auto impl) {
        decltype(impl)::correct(n, g, r, s, out, st);
        return 0;
    });
    return hipGetLastError() == hipSuccess ? out : nullptr;
}

}  // namespace

extern "C" {

int net_workspace_bytes(int64_t max_voxels, int32_t precision, int32_t train, size_t *bytes)
{
    if (max_voxels < 1 || (precision != NET_PREC_BF16 && precision != NET_PREC_F64) || (train != 0 && train != 1) ||
        !bytes)
        return SMG_EINVAL;
    *bytes = make_net_layout(max_voxels, precision, train).total;
    return SMG_OK;
}

int net_setup(int64_t max_voxels, int32_t precision, int32_t train, void *ws, size_t ws_bytes, void *stream,
              net_handle **out)
{
    if (!out) return SMG_EINVAL;
    *out = nullptr;
    size_t need = 0;
    if (net_workspace_bytes(max_voxels, precision, train, &need) != SMG_OK || !ws) return SMG_EINVAL;
    if (ws_bytes < need) return SMG_EWORKSPACE;
    net_handle *n = new (std::nothrow) net_handle();
    if (!n) return SMG_EHIP;
    n->prec = precision;
    n->train = train;
    n->max_vox = max_voxels;
    n->ws = static_cast<char *>(ws);
    n->L = make_net_layout(max_voxels, precision, train);
    n->lt = layer_table();
    hipStream_t st = as_st(stream);
    // zero parameters (and Adam state) so that every kernel reads defined values
    if (hipMemsetAsync(n->ws, 0, n->L.part, st) != hipSuccess) {
        delete n;
        return SMG_EHIP;
    }
    if (train && (hipMemsetAsync(n->ws + n->L.grad, 0, n->L.wpart - n->L.grad, st) != hipSuccess)) {
        delete n;
        return SMG_EHIP;
    }
    if (hipStreamSynchronize(st) != hipSuccess) {
        delete n;
        return SMG_EHIP;
    }
    *out = n;
    return SMG_OK;
}

int net_destroy(net_handle *n)
{
    delete n;
    return SMG_OK;
}

int net_set_params(net_handle *n, const double *params, void *stream)
{
    if (!n || !params) return SMG_EINVAL;
    for (int i = 0; i < NET_NPARAMS; ++i)
        if (!std::isfinite(params[i])) return SMG_ENONFINITE;
    hipStream_t st = as_st(stream);
    return dispatch(n, [&](auto impl) {
        using I = decltype(impl);
        using A = std::remove_pointer_t<decltype(I::p(n))>;
        std::vector<A> h(params, params + NET_NPARAMS);
        if (hipMemcpyAsync(I::p(n), h.data(), NET_NPARAMS * sizeof(A), hipMemcpyHostToDevice, st) != hipSuccess)
            return SMG_EHIP;
        if (n->train) {
            if (hipMemsetAsync(n->ws + n->L.m, 0, NET_NPARAMS * sizeof(A), st) != hipSuccess ||
                hipMemsetAsync(n->ws + n->L.v, 0, NET_NPARAMS * sizeof(A), st) != hipSuccess)
                return SMG_EHIP;
        }
        n->adam_t = 0;
        n->have_grad = false;
        I::pack(n, st);
        return hipStreamSynchronize(st) == hipSuccess && hipGetLastError() == hipSuccess ? SMG_OK : SMG_EHIP;
    });
}

int net_get_params(net_handle *n, double *params, void *stream)
{
    if (!n || !params) return SMG_EINVAL;
    hipStream_t st = as_st(stream);
    return dispatch(n, [&](auto impl) {
        using I = decltype(impl);
        using A = std::remove_pointer_t<decltype(I::p(n))>;
        std::vector<A> h(NET_NPARAMS);
        if (hipMemcpyAsync(h.data(), I::p(n), NET_NPARAMS * sizeof(A), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return SMG_EHIP;
        for (int i = 0; i < NET_NPARAMS; ++i) params[i] = static_cast<double>(h[i]);
        return SMG_OK;
    });
}

int net_layer_forward(net_handle *n, int32_t layer, int32_t nx, int32_t ny, int32_t nz, const void *in, void *out,
                      void *stream)
{
    if (!n || !in || !out || layer < 0 || layer > 3 || !grid_ok(n, nx, ny, nz)) return SMG_EINVAL;
    hipStream_t st = as_st(stream);
    return dispatch(n, [&](auto impl) {
        const int rc = decltype(impl)::layer_forward(n, layer, nx, ny, nz, in, out, st);
        return rc == SMG_OK && hipGetLastError() == hipSuccess ? SMG_OK : SMG_EHIP;
    });
}

int net_loss_grad(net_handle *n, int32_t nx, int32_t ny, int32_t nz, const void *input, const void *target,
                  int32_t loss_kind, double *loss, double *grad, void *stream)
{
    if (!n || !n->train || !input || !target || !grid_ok(n, nx, ny, nz)) return SMG_EINVAL;
    if (loss_kind != NET_LOSS_MSE && loss_kind != NET_LOSS_ENERGY) return SMG_EINVAL;
    hipStream_t st = as_st(stream);
    return dispatch(n, [&](auto impl) {
        using I = decltype(impl);
        using A = std::remove_pointer_t<decltype(I::p(n))>;
        using T = std::remove_pointer_t<decltype(I::wst(n))>;
        double *ld = n->at<double>(n->L.loss);
        I::loss_grad(n, nx, ny, nz, static_cast<const T *>(input), static_cast<const A *>(target), loss_kind, ld,
                     st);
        n->have_grad = true;
        double lh = 0.0;
        std::vector<A> gh(grad ? NET_NPARAMS : 0);
        if (hipMemcpyAsync(&lh, ld, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess) return SMG_EHIP;
        if (grad && hipMemcpyAsync(gh.data(), n->at<A>(n->L.grad), NET_NPARAMS * sizeof(A), hipMemcpyDeviceToHost,
                                   st) != hipSuccess)
            return SMG_EHIP;
        if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) return SMG_EHIP;
        if (loss) *loss = lh;
        if (grad)
            for (int i = 0; i < NET_NPARAMS; ++i) grad[i] = static_cast<double>(gh[i]);
        return SMG_OK;
    });
}

int net_adam_step(net_handle *n, double lr, void *stream)
{
    if (!n || !n->train || !n->have_grad || !(lr >= 0.0)) return SMG_EINVAL;
    hipStream_t st = as_st(stream);
    return dispatch(n, [&](auto impl) {
        decltype(impl)::adam(n, lr, st);
        return hipGetLastError() == hipSuccess ? SMG_OK : SMG_EHIP;
    });
}

int net_train(net_handle *n, int32_t nx, int32_t ny, int32_t nz, const void *inputs, const void *targets,
              int32_t npairs, int32_t steps, const int32_t *order, const double *lr, int32_t loss_kind,
              double *loss_history, void *stream)
{
    if (!n || !n->train || !inputs || !targets || npairs < 1 || steps < 0 || (steps > 0 && (!order || !lr)) ||
        !grid_ok(n, nx, ny, nz) || (loss_kind != NET_LOSS_MSE && loss_kind != NET_LOSS_ENERGY))
        return SMG_EINVAL;
    for (int k = 0; k < steps; ++k)
        if (order[k] < 0 || order[k] >= npairs || !(lr[k] >= 0.0)) return SMG_EINVAL;
    hipStream_t st = as_st(stream);
    return dispatch(n, [&](auto impl) {
        return decltype(impl)::train(n, nx, ny, nz, inputs, targets, steps, order, lr, loss_kind, loss_history,
                                     st);
    });
}

int net_correct(net_handle *n, smg_handle *h, const double *r, const double *s, double *out, double *sigma,
                void *stream)
{
    if (!n || !h || !r || !s || !out || smg_handle_is_var(h)) return SMG_EINVAL;
    const smg_grid *g = smg_handle_grid(h);
    if (!grid_ok(n, g->nx, g->ny, g->nz)) return SMG_EINVAL;
    hipStream_t st = as_st(stream);
    dispatch(n, [&](auto impl) {
        decltype(impl)::correct(n, *g, r, s, out, st);
        return 0;
    });
    if (hipGetLastError() != hipSuccess) return SMG_EHIP;
    if (sigma) {
        NetScalars hs{};
        if (hipMemcpyAsync(&hs, n->at<NetScalars>(n->L.ns), sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return SMG_EHIP;
        *sigma = hs.sigma;
    }
    return SMG_OK;
}

int net_make_pairs(net_handle *n, smg_handle *h_pre, smg_handle *h_exact, int32_t npairs, uint64_t seed0,
                   double exact_rtol, int32_t exact_max_iter, void *inputs, void *targets, double *sigma,
                   void *stream)
{
    if (!n || !n->train || !h_pre || !h_exact || npairs < 1 || !inputs || !targets || !(exact_rtol > 0.0) ||
        exact_max_iter < 1 || smg_handle_is_var(h_pre) || smg_handle_is_var(h_exact))
        return SMG_EINVAL;
    const smg_grid *g = smg_handle_grid(h_pre);
    const smg_grid *ge = smg_handle_grid(h_exact);
    if (g->nx != ge->nx || g->ny != ge->ny || g->nz != ge->nz || g->cx != ge->cx || g->cy != ge->cy ||
        g->cz != ge->cz || !grid_ok(n, g->nx, g->ny, g->nz))
        return SMG_EINVAL;
    hipStream_t st = as_st(stream);
    const long long N = static_cast<long long>(g->nx) * g->ny * g->nz;
    double *b = n->at<double>(n->L.b), *xp = n->at<double>(n->L.xp), *xs = n->at<double>(n->L.xs);
    double *rp = n->at<double>(n->L.rp), *part = n->at<double>(n->L.part);
    NetScalars *ns = n->at<NetScalars>(n->L.ns);
    int result = SMG_OK;
    for (int i = 0; i < npairs; ++i) {
        launch_uniform_pm1(static_cast<unsigned long long>(seed0) + static_cast<unsigned long long>(i), N, b, st);
        int rc = smg_apply(h_pre, b, xp, 1, N, stream);
        if (rc != SMG_OK) return rc;
        krylov_opts ko{};
        ko.rtol = exact_rtol;
        ko.max_iter = exact_max_iter;
        ko.precond = SMG_PRECOND_SMG;
        ko.x0_zero = 1;
        krylov_info ki{};
        rc = fpcg_solve(h_exact, b, xs, &ko, &ki, stream);
        if (rc < 0) return rc;
        if (rc == SMG_NOT_CONVERGED) result = SMG_NOT_CONVERGED;
        launch_init_resid(b, xp, rp, 0, g->nx, g->ny, g->nz, g->cx, g->cy, g->cz, part, st);
        launch_net_scalars(part, kRedBlocks, (g->cx + g->cy + g->cz) / 3.0, static_cast<double>(N), ns, st);
        dispatch(n, [&](auto impl) {
            decltype(impl)::pair_store(n, N, inputs, targets, i, st);
            return 0;
        });
        if (sigma) {
            NetScalars hs{};
            if (hipMemcpyAsync(&hs, ns, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess) return SMG_EHIP;
            if (hipStreamSynchronize(st) != hipSuccess) return SMG_EHIP;
            sigma[i] = hs.sigma;
        }
    }
    if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) return SMG_EHIP;
    return result;
}

int fpcg_learned_solve(smg_handle *h, net_handle *n, const double *b, double *x, const krylov_opts *o,
                       krylov_info *info, net_solve_info *ninfo, void *stream)
{
    if (!h || !n || !o || smg_handle_is_var(h)) return SMG_EINVAL;
    const smg_grid *g = smg_handle_grid(h);
    if (!grid_ok(n, g->nx, g->ny, g->nz) || o->precond != SMG_PRECOND_SMG) return SMG_EINVAL;
    HookCtx ctx{n, h};
    PrecondHook hook{};
    hook.ctx = &ctx;
    hook.apply = hook_apply;
    hook.active = 1;
    hook.fallback_iter = -1;
    hook.fallback_reason = NET_FALLBACK_NONE;
    const int rc = krylov_run(h, 1, b, x, o, info, stream, &hook);
    if (ninfo) {
        ninfo->fallback_iter = hook.fallback_iter;
        ninfo->fallback_reason = hook.fallback_reason;
    }
    return rc;
}

}  // extern "C"
