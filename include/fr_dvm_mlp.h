/*
 * fr_dvm_mlp.h -- C ABI of the learned initial guess for the conservative-
 * equilibrium Newton solve of libfrdvm (see fr_dvm.h).
 *
 * The paper finds the modified equilibrium of eq. (discrete_compatibility)
 * per solution point by Newton's method (Section "Numerical method").  This
 * part of the library trains, on the GPU, a small network that predicts the
 * starting point of that Newton solve; Newton alone decides convergence on the
 * residual and falls back to the cold start when the prediction fails.
 *
 * Network: 13 -> H -> H -> H -> 5, SiLU on the hidden layers, FP32.
 *   inputs  x = [ln rho, U/u_max (3), ln theta, u_max/10, n_v/32,
 *                sin phi (3), cos phi (3)],  phi_d = 2 pi (U_d - umin_d)/du_d:
 *   the phase of the bulk velocity against the grid, on which the trapezoid
 *   aliasing error of a Gaussian depends periodically (Poisson summation)
 *   outputs y (normalised); prediction dz = y * scale + offset is added to
 *   the cold Newton unknowns z_cold = (-3/2 ln 2 pi, 0, 0, 0, 1) (BGK frame
 *   c = (u-U)/sqrt(theta)).
 * Flat parameter layout (floats): for each of the 4 layers W (out x in, row
 * major) then b (out); then scale[5], offset[5].
 *
 * All arrays are caller-owned DEVICE float arrays unless stated; every call
 * is asynchronous on `stream` (a hipStream_t passed as void*, may be NULL).
 * Return: 0 or a negative FR_DVM_E* code (fr_dvm.h).  Batches are row
 * major: X[B][FR_MLP_INPUTS], T[B][5].  GEMMs run on MFMA (v_mfma_f32_16x16x4_f32).
 */
#ifndef FR_DVM_MLP_H
#define FR_DVM_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "fr_dvm.h"

#define FR_MLP_INPUTS 13

#ifdef __cplusplus
extern "C" {
#endif

/* Number of floats of the flat parameter vector for hidden width H. */
size_t fr_mlp_param_count(int H);

/* Floats of scratch memory the forward / gradient calls need for a batch. */
size_t fr_mlp_workspace_floats(int H, int64_t B);

/* Prediction dz[B][5] (denormalised) for features X[B][FR_MLP_INPUTS]. */
int fr_mlp_forward(int H, const float *w, const float *X, int64_t B, float *dz, float *work, void *stream);

/* fr_mlp_forward without allocation or workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The intermediate activations live in a
 * fixed library scratch of FR_MLP_NOALLOC_FLOATS floats (16 MiB) per GPU,
 * held from the first call on that GPU until the process ends; a batch needs
 * B * (2 H + 5) floats of it (H = 64: B <= 31,536).  Larger requests return
 * FR_DVM_ESCRATCH before anything is launched.  No hipMalloc, hipFree or
 * allocating library routine is called.  Every call on one GPU shares its
 * scratch: calls that overlap on one GPU (other streams, other threads) race
 * and must be ordered by the caller.  Results equal fr_mlp_forward's bit for
 * bit (same kernels, same order). */
#define FR_MLP_NOALLOC_FLOATS ((size_t)1 << 22)
int fr_mlp_forward_noalloc(int H, const float *w, const float *X, int64_t B, float *dz, void *stream);

/* Mean-squared-error loss L = 1/(2B) sum |y - T|^2 on normalised targets T,
 * its gradient grad[param_count] (zero on the output affine) and L itself
 * (device float[1]). */
int fr_mlp_grad(int H, const float *w, const float *X, const float *T, int64_t B, float *grad, float *loss,
                float *work, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) at iteration `step` (1-based)
 * on the network weights; the output affine (last 10 floats) is not updated. */
int fr_mlp_adam(int H, float *w, const float *grad, float *m, float *v, int step, float lr, void *stream);

/* Conservative equilibria for n given moment vectors Q[n][5] (rho, rho U, E)
 * on the handle's velocity grid (BGK form): FP64 Newton from the cold start
 * (guess = FR_DVM_GUESS_COLD) or from the better (smaller residual) of the
 * cold start and the handle's MLP prediction (FR_DVM_GUESS_MLP).
 * Outputs (device, nullable): z[n][5] Newton unknowns in the frame
 * c = (u-U)/sqrt(theta), iters[n] linear solves, evals[n] residual/Jacobian
 * evaluations (sum passes over the grid), status[n] (FR_DVM_NEWTON_*),
 * resid[n] final scaled residual.  Uses the handle's tolerance and
 * iteration cap.  Synchronises the handle's stream. */
int fr_dvm_equilibrium(fr_dvm_t h, const double *Q, int64_t n, int guess, double *z, int32_t *iters,
                       int32_t *evals, int32_t *status, double *resid);

#ifdef __cplusplus
}
#endif
#endif /* FR_DVM_MLP_H */
