/*
 * smg_net.h -- C ABI of the learned post-smoother that accompanies the SMG
 * preconditioner of smg.h.
 *
 * This part is an addition beside the paper's method, which it relies on in
 * one place: flexible PCG (Section 2, equation (2)) stays locally optimal for
 * a preconditioner that changes from step to step or is nonlinear, so a
 * learned correction may follow the V-cycle inside fpcg_solve's recurrence.
 *
 * Network N: four 3x3x3 convolutions (cross-correlations) with zero padding,
 * channels 1 -> 16 -> 16 -> 16 -> 1, a bias per output channel and ReLU
 * after the first three layers; NET_NPARAMS = 14737 parameters.  Flat
 * parameter order (host arrays of doubles): for each layer, the weights
 * W[dz][dy][dx][ci][co] (C order, each of dz, dy, dx in 0..2 selecting the
 * input voxel at offset -1..+1) followed by the biases b[co].
 *
 * Use as a post-smoother (the preconditioner of fpcg_learned_solve):
 *     s  = T r                       (SMG V-cycle, normally (pre,post) = (1,0))
 *     r' = r - A s,  sigma = rms(r'/cbar),  cbar = (cx + cy + cz)/3
 *     s <- s + sigma * N(r' / (cbar*sigma))
 * The division by cbar maps the operator to its unit-stencil form (cbar = 1/h^2
 * on a cube), so a network trained on one grid applies to another.
 *
 * Training data (net_make_pairs): b ~ U[-1,1) from the SplitMix64 stream of
 * seed0 + i (the same generator as the library's test inputs), x' = T b,
 * r' = b - A x', e' = A^{-1} b - x' with A^{-1} b from an accurate FPCG solve;
 * the stored input is r'/(cbar*sigma) and the target e'/sigma.  Loss over the
 * grid, d = N(input) - target: NET_LOSS_MSE mean(d^2), or NET_LOSS_ENERGY
 * mean(d * L d) with L the unit 7-point stencil (6 on the diagonal, -1 to each
 * neighbour, zero outside), i.e. the error in the energy norm of the
 * unit-stencil operator.  Optimiser: Adam (Kingma and Ba, 2015) with
 * beta1 = 0.9, beta2 = 0.999, eps = 1e-8.
 *
 * Precision: NET_PREC_BF16 stores activations, gradients and the weights used
 * by the kernels in bfloat16 (round to nearest even), accumulates in FP32 and
 * keeps FP32 master weights and Adam moments; the 16 -> 16 layers run on the
 * matrix cores.  NET_PREC_F64 is a check mode that does everything in FP64.
 * Element types of caller buffers: "storage" = uint16 bfloat16 bits (BF16) or
 * double (F64); "accum" = float (BF16) or double (F64).
 *
 * Memory: all vector arguments are DEVICE pointers, channels-last for
 * multi-channel arrays (voxel index x + nx*(y + ny*z), then channel), caller
 * owned.  The network's device workspace is caller owned too.  Return codes
 * and stream semantics are those of smg.h.
 */
#ifndef SMG_NET_H
#define SMG_NET_H

#include <stddef.h>
#include <stdint.h>

#include "smg.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { NET_PREC_BF16 = 0, NET_PREC_F64 = 1 };
enum { NET_NPARAMS = 14737 };
enum { NET_LOSS_MSE = 0, NET_LOSS_ENERGY = 1 };
enum {
    NET_FALLBACK_NONE = 0,
    NET_FALLBACK_SR = 1,          /* (s, r) <= 0 with the learned correction */
    NET_FALLBACK_NONFINITE = 2,   /* non-finite corrected s */
    NET_FALLBACK_STAGNATION = 3   /* ||r_k|| > 0.9 ||r_{k-2}|| */
};

typedef struct net_handle net_handle;

/* Device workspace bytes for grids of up to max_voxels points.  train = 0:
 * inference only (fpcg_learned_solve, net_correct, net_layer_forward);
 * train = 1 adds activations and gradients for training, Adam state and the
 * buffers of net_make_pairs.  Host-only. */
int net_workspace_bytes(int64_t max_voxels, int32_t precision, int32_t train, size_t *bytes);

/* Lays the network out in the caller's workspace; parameters start at zero
 * (set them with net_set_params). */
int net_setup(int64_t max_voxels, int32_t precision, int32_t train, void *ws, size_t ws_bytes, void *stream,
              net_handle **out);
int net_destroy(net_handle *n);

/* Host FP64 parameters in the flat order above.  net_set_params also resets
 * the Adam moments and step counter.  Both synchronise the stream. */
int net_set_params(net_handle *n, const double *params, void *stream);
int net_get_params(net_handle *n, double *params, void *stream);

/* One layer (0..3) on an nx*ny*nz grid, for checks.  in: storage elements,
 * 1 channel for layer 0 and 16 otherwise; out: storage elements with bias and
 * ReLU for layers 0..2 (16 channels), accum elements with bias for layer 3
 * (1 channel). */
int net_layer_forward(net_handle *n, int32_t layer, int32_t nx, int32_t ny, int32_t nz, const void *in, void *out,
                      void *stream);

/* Loss (loss_kind NET_LOSS_*) on one nx*ny*nz sample and its gradient.
 * input: storage elements, target: accum elements.  loss (host, nullable);
 * grad (host, nullable, NET_NPARAMS doubles).  The gradient stays on the
 * device for net_adam_step.  Synchronises the stream. */
int net_loss_grad(net_handle *n, int32_t nx, int32_t ny, int32_t nz, const void *input, const void *target,
                  int32_t loss_kind, double *loss, double *grad, void *stream);

/* One Adam step with learning rate lr on the gradient of the last
 * net_loss_grad (or training step). */
int net_adam_step(net_handle *n, double lr, void *stream);

/* Training: steps Adam steps, step k on pair order[k] (host, 0 <= order[k] <
 * npairs) with learning rate lr[k] (host).  inputs/targets: npairs samples of
 * nx*ny*nz elements each (storage / accum), as written by net_make_pairs.
 * loss_history: host, nullable, steps entries (loss before each step).
 * Synchronises the stream. */
int net_train(net_handle *n, int32_t nx, int32_t ny, int32_t nz, const void *inputs, const void *targets,
              int32_t npairs, int32_t steps, const int32_t *order, const double *lr, int32_t loss_kind,
              double *loss_history, void *stream);

/* out = s + sigma * N(r' / (cbar*sigma)), r' = r - A s, on h's grid (FP64
 * device vectors; out must not overlap r or s).  sigma: host, nullable
 * (synchronises the stream when given). */
int net_correct(net_handle *n, smg_handle *h, const double *r, const double *s, double *out, double *sigma,
                void *stream);

/* Training pairs i = 0..npairs-1 on h_pre's grid: b_i from seed0 + i, x' =
 * T_pre b_i, A^{-1} b_i by fpcg_solve on h_exact (same grid) to exact_rtol.
 * inputs: npairs*N storage elements; targets: npairs*N accum elements;
 * sigma: host, nullable, npairs entries.  Returns SMG_NOT_CONVERGED if an
 * exact solve missed exact_rtol within exact_max_iter (pairs still written). */
int net_make_pairs(net_handle *n, smg_handle *h_pre, smg_handle *h_exact, int32_t npairs, uint64_t seed0,
                   double exact_rtol, int32_t exact_max_iter, void *inputs, void *targets, double *sigma,
                   void *stream);

typedef struct net_solve_info {
    int32_t fallback_iter;    /* iteration from which plain T was used; -1 = never */
    int32_t fallback_reason;  /* NET_FALLBACK_* */
} net_solve_info;

/* Flexible PCG (equation (2)) with s_k = T r_k corrected by the network as
 * above.  Falls back to plain s_k = T r_k for the rest of the solve when the
 * corrected s_k is non-finite, when (s_k, r_k) <= 0, or when the residual
 * norm fails to drop below 0.9 times its value two iterations earlier.
 * Arguments and result as fpcg_solve; ninfo (host, nullable). */
int fpcg_learned_solve(smg_handle *h, net_handle *n, const double *b, double *x, const krylov_opts *o,
                       krylov_info *info, net_solve_info *ninfo, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SMG_NET_H */
