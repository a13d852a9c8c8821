/*
 * pn_nn.h -- C ABI of the learned initial guess / preconditioner of the P_N
 * solver (MI355X, gfx950): a 3D convolutional U-Net trained on solutions the
 * solver itself generates.  The paper has no learned component; the network,
 * its layout and its training are this library's own design.
 *
 * Tensors are DEVICE arrays, channels-last bfloat16 (raw 16-bit words):
 * t[b][z][y][x][c] with 32 channels, x fastest among the spatial indices.
 * Weights of a 3x3x3 convolution: w[t][co][ci] (27 x 32 x 32 bfloat16), tap
 * t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1) for the offsets dz, dy, dx in
 * {-1, 0, 1}; zero padding at the grid border.  Every product runs on the
 * matrix cores in bfloat16 with FP32 accumulation.
 *
 * The network (4 levels, 32 channels everywhere, 15 convolutions):
 *   level l = 0..3 encoder: two conv+ReLU, then 2x2x2 average pooling (l < 3);
 *   decoder l = 2..0: nearest 2x upsampling + the level's encoder output,
 *   two conv+ReLU; output: one conv without activation (32 channels, the loss
 *   uses the first nout).  Parameters: FP32 master copy [15][27*32*32 weights,
 *   32 biases]; Adam (Kingma & Ba 2015) with beta1 0.9, beta2 0.999, eps 1e-8.
 *
 * Errors: status codes of pn.h; pn_net_last_error / pn_nn_last_error give
 * text.  Calls on one network must not overlap.  Asynchronous on `stream`
 * unless stated.
 */
#ifndef PN_NN_H
#define PN_NN_H

#include <stdint.h>

#include "pn.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------- primitives -- */
/* y = conv(x, w) + bias (bias FP32 [32] or NULL), ReLU if relu != 0; y is
 * FP32 if out_f32 != 0 else bfloat16.  Extents nx, ny, nz >= 1, batch B. */
pn_status pn_nn_conv3d(int B, int nx, int ny, int nz, const uint16_t* x, const uint16_t* w,
                       const float* bias, int relu, int out_f32, void* y, void* stream);
/* dx = conv^T(g, w): the gradient of <conv(x, w), g> with respect to x. */
pn_status pn_nn_conv3d_dgrad(int B, int nx, int ny, int nz, const uint16_t* g, const uint16_t* w,
                             uint16_t* dx, void* stream);
/* dw[t][co][ci] = sum over voxels of g[v][co] x[v + d_t][ci] (FP32, 27*32*32),
 * db[co] = sum over voxels of g[v][co] (FP32, 32).  Allocates a temporary
 * workspace; synchronous. */
pn_status pn_nn_conv3d_wgrad(int B, int nx, int ny, int nz, const uint16_t* x, const uint16_t* g,
                             float* dw, float* db, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the weight
 * gradient of pn_nn_conv3d_wgrad with the same arguments, results and
 * kernels, whose per-block partial sums live in a static device array of
 * 128 x (27*32*32 + 32) floats (14.2 MB, held by every device the library
 * runs on until the process ends) instead of a temporary allocation.
 * Allocates nothing.  Asynchronous on `stream`.  Volumes needing more than
 * 128 partial blocks (B*nx*ny*nz > 32768) fail with PN_ERR_ARG.  All calls on
 * one device share its array: calls that overlap on one device (different
 * streams, or host threads) race and must be serialised by the caller. */
pn_status pn_nn_conv3d_wgrad_noalloc(int B, int nx, int ny, int nz, const uint16_t* x, const uint16_t* g,
                                     float* dw, float* db, void* stream);
/* 2x2x2 average pooling of x (extents nx, ny, nz even) into y (half extents). */
pn_status pn_nn_pool2(int B, int nx, int ny, int nz, const uint16_t* x, uint16_t* y, void* stream);
/* gf = adjoint of pool2 applied to gc (half extents) + skip (NULL: none). */
pn_status pn_nn_pool2_bwd_add(int B, int nx, int ny, int nz, const uint16_t* gc, const uint16_t* skip,
                              uint16_t* gf, void* stream);
/* y = nearest 2x upsampling of xc (half extents) + skip (NULL: none). */
pn_status pn_nn_up2_add(int B, int nx, int ny, int nz, const uint16_t* xc, const uint16_t* skip,
                        uint16_t* y, void* stream);
/* gc = adjoint of up2: sums of gf over 2x2x2 blocks (gc has half extents). */
pn_status pn_nn_up2_bwd(int B, int nx, int ny, int nz, const uint16_t* gf, uint16_t* gc, void* stream);
/* One Adam step (step >= 1) on FP32 arrays of n entries, in place (beta1,
 * beta2 in FP64 so that 1 - beta is exact to FP32). */
pn_status pn_nn_adam(float* w, const float* g, float* m, float* v, long long n, long long step, float lr,
                     double beta1, double beta2, float eps, void* stream);
const char* pn_nn_last_error(void);

/* ------------------------------------------------------------- network -- */
typedef struct pn_net pn_net;

/* Number of FP32 parameters (15 * (27*32*32 + 32)). */
int pn_net_nparams(void);
/* He-normal initial weights from `seed` (output convolution scaled by 0.1),
 * zero biases.  Synchronous. */
pn_status pn_net_create(unsigned long long seed, void* stream, pn_net** out);
void pn_net_destroy(pn_net* net);
const char* pn_net_last_error(const pn_net* net);
/* Host copies of the parameters and/or of the gradients of the last training
 * step (either pointer may be NULL, not both).  Synchronous. */
pn_status pn_net_get_params(pn_net* net, float* params, float* grads);
/* Replaces the parameters (host array) and resets the optimizer state. */
pn_status pn_net_set_params(pn_net* net, const float* params);
/* Binary parameter file (magic "PNUNET01", parameter count, step, FP32
 * parameters).  Synchronous. */
pn_status pn_net_save(pn_net* net, const char* path);
pn_status pn_net_load(pn_net* net, const char* path);
/* y (FP32 [B][nz][ny][nx][32]) = net(x); extents multiples of 8.  Buffers of
 * the activations are (re)allocated when the shape changes. */
pn_status pn_net_forward(pn_net* net, int B, int nx, int ny, int nz, const uint16_t* x, float* y);
/* One training step on the batch: forward, mean squared error of the first
 * nout output channels against target (bfloat16 [B][nz][ny][nx][nout]),
 * backward; with lr > 0 one Adam step (lr = 0: gradients only).  *loss (may be
 * NULL) receives the loss before the update.  Synchronous. */
pn_status pn_net_train_step(pn_net* net, int B, int nx, int ny, int nz, const uint16_t* x,
                            const uint16_t* target, int nout, float lr, double* loss);

/* Training loop: `epochs` passes over nsamples samples given as HOST arrays
 * of DEVICE pointers (x[i]: [nz][ny][nx][32] bfloat16 input, t[i]:
 * [nz][ny][nx][nout] bfloat16 target), in a seeded random order, `batch`
 * samples per step (gathered into staging buffers the call allocates and
 * frees), learning rate decayed from lr to 0 on a cosine.  *loss_out (may be
 * NULL): mean loss of the last epoch.  Synchronous. */
pn_status pn_net_train(pn_net* net, int nsamples, int nx, int ny, int nz, const uint16_t* const* x,
                       const uint16_t* const* t, int nout, int epochs, int batch, float lr,
                       unsigned long long seed, double* loss_out);

/* Stream of the network's launches (NULL: the null stream). */
pn_status pn_net_set_stream(pn_net* net, void* stream);
void* pn_net_get_stream(const pn_net* net);

/* ------------------------------------------------- solver connection -- */
/* Network grid of a solver context: the cell grid rounded up to multiples
 * of 8 (the extra cells carry zero features). */
pn_status pn_net_grid(const pn_ctx* ctx, int* nx8, int* ny8, int* nz8);
/* Network input for the context's medium and a source (device FP32 vector in
 * the context's packed layout: the emission Q, or a residual):
 * x [nz8][ny8][nx8][32] bfloat16 with channels sigma_t h (thresholded),
 * sigma_a h, then for k < min(16, coefficients) the source's coefficient k at
 * the lattice point with the cell's indices divided by the largest such
 * |value|, then zeros (an isotropic emission fills channel 2 only).  On the
 * context's stream. */
pn_status pn_net_features(pn_ctx* ctx, const float* src, uint16_t* x);
/* Training target for a solution (device FP64 vector, packed layout):
 * t [nz8][ny8][nx8][16] bfloat16, channel k = coefficient k (bands l <= 3) at
 * the lattice point with the cell's indices, divided by the largest |L00|
 * over the cells; zero where there is none.  On the context's stream. */
pn_status pn_net_targets(pn_ctx* ctx, const double* solution, uint16_t* t);
/* The same for the difference solution - sub (both device FP64 vectors in
 * the packed layout; sub NULL: none): the target of a correction step, the
 * remaining correction x* - x_j of a partially converged iterate x_j.  On the
 * context's stream. */
pn_status pn_net_targets_diff(pn_ctx* ctx, const double* solution, const double* sub, uint16_t* t);
/* Attaches a network to a solver context (NULL detaches); pn_solve uses it
 * as opts->learned asks, on the solver's stream (the network's own stream is
 * restored afterwards).  The network must outlive the attachment. */
pn_status pn_attach_net(pn_ctx* ctx, pn_net* net);

#ifdef __cplusplus
}
#endif
#endif /* PN_NN_H */
