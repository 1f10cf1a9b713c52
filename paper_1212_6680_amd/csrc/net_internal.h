// Internal declarations of the learned post-smoother (not part of the C ABI).
#pragma once

#include "smg_internal.h"
#include "../../include/smg_net.h"

namespace smg {
namespace net {

constexpr int kWgradBlocks = 512;   // fixed grid of the weight-gradient partial sums
constexpr int kLossBlocks = 1024;   // fixed grid of the loss partial sums

struct NetScalars {         // device-resident normalisation of the network input
    double sigma;           // rms of r'/cbar
    double in_scale;        // 1/(cbar*sigma): r' -> network input
    double out_scale;       // sigma: network output -> correction
    double inv_sigma;       // 1/sigma (training targets)
};

struct LayerTable {         // offsets of each layer in the flat parameter vector
    int off[5];
    int cin[4];
    int cout[4];
    int total;
};

struct Conv16Args {
    const bf16 *in;         // 16 channels per voxel
    const uint16_t *frag;   // 14 x 64 x 8 MFMA A-operand fragments
    const float *bias;      // 16 (EPI 0)
    const bf16 *mask;       // 16 channels per voxel (EPI 1)
    bf16 *out;              // 16 channels per voxel
    int nx, ny, nz;
    int zc;                 // planes per block (set by the launcher)
};

template <typename T, typename A>
struct ConvVecArgs {
    const T *in;            // CIN channels per voxel (INM 0)
    const double *in64;     // single FP64 channel (INM 1), scaled by ns->in_scale
    const NetScalars *ns;
    const T *W;             // [tap][ci][co]
    const A *bias;
    const T *mask;          // EPI 1
    T *out;                 // EPI 0, 1
    A *outA;                // EPI 2
    const double *s_in;     // EPI 3
    double *s_out;          // EPI 3
    int nx, ny, nz;
};

struct In16Args {            // bf16 1 -> 16 layer
    const bf16 *in;          // INM 0
    const double *in64;      // INM 1
    const NetScalars *ns;
    const bf16 *w;           // [27][16] weights (tap, output channel)
    const float *bias;       // EPI 0
    const bf16 *mask;        // EPI 1
    bf16 *out;
    int nx, ny, nz, zc;
};

struct Out16Args {           // bf16 16 -> 1 layer
    const bf16 *in;
    const unsigned int *w;   // 27 x 8 channel pairs
    const float *bias;
    const NetScalars *ns;    // EPI 3
    float *outA;             // EPI 2
    const double *s_in;      // EPI 3
    double *s_out;           // EPI 3
    int nx, ny, nz, zc;
};

template <typename T, typename A>
struct WgradArgs {
    const T *in;            // layer input, CIN channels
    const T *g;             // gradient at the layer output (after the ReLU mask), COUT channels
    A *part;                // kWgradBlocks x (27*CIN*COUT + COUT) partial sums
    int nx, ny, nz;
};

void launch_conv16_mfma(const Conv16Args &a, int epi, hipStream_t st);
void launch_in16_bf16(const In16Args &a, int inm, int epi, hipStream_t st);
void launch_out16_bf16(const Out16Args &a, int epi, hipStream_t st);
template <typename T, typename A, int CIN, int COUT, int INM, int EPI>
void launch_conv_vec(const ConvVecArgs<T, A> &a, hipStream_t st);
int wgrad_blocks(int nx, int ny, int nz);
template <typename T, typename A, int CIN, int COUT>
void launch_wgrad(const WgradArgs<T, A> &a, A *grad, hipStream_t st);
template <typename T, typename A>
void launch_loss(int kind, const A *y, const A *t, T *g, int nx, int ny, int nz, double *partials, double *loss_out,
                 hipStream_t st);
void launch_net_scalars(const double *partials, int np, double cbar, double n, NetScalars *ns, hipStream_t st);
template <typename A>
void launch_adam(A *p, A *m, A *v, const A *g, int n, double lr, double b1, double b2, double eps, double bc1,
                 double bc2, hipStream_t st);
template <typename T, typename A>
void launch_pack(const A *p, T *wst, T *wtr, const LayerTable &lt, hipStream_t st);
void launch_pack_frag(const float *p, int off, int bwd, uint16_t *frag, hipStream_t st);
template <typename T, typename A>
void launch_pair_store(const double *rp, const double *xs, const double *xp, const NetScalars *ns, T *input,
                       A *target, long long n, hipStream_t st);
void launch_uniform_pm1(unsigned long long seed, long long n, double *out, hipStream_t st);

}  // namespace net

// Optional correction of the preconditioned residual inside the Krylov loop
// (the learned post-smoother).  apply returns the vector to use as s_k, or
// nullptr on a HIP error.  The loop clears `active` and records the iteration
// and reason when it falls back to the plain preconditioner.
struct PrecondHook {
    void *ctx;
    const double *(*apply)(void *ctx, const double *r, const double *s, hipStream_t st);
    int active;
    int fallback_iter;
    int fallback_reason;
};

int krylov_run(smg_handle *h, int method, const double *b, double *x, const krylov_opts *o, krylov_info *info,
               void *stream, PrecondHook *hook);

}  // namespace smg

const smg_grid *smg_handle_grid(const smg_handle *h);
