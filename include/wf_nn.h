/* Learned warm start for the messenger iteration: a convolutional network
 * that predicts the Wiener solution from (d, N_pix, mask), trained and run on
 * the GPU with bfloat16 matrix-core convolutions and float32 accumulation.
 *
 * The paper's iteration may start from any field (Section 2: the start does
 * not change the solution); this library supplies a start.  The network is
 * not from the paper.
 *
 * Network (fixed architecture, 15 convolutions, periodic 3x3 kernels):
 *   levels l = 0..3 with channels C = {32, 64, 96, 128}, each level at half
 *   the resolution of the previous one (2x2 average pooling); two
 *   convolution + ReLU stages per encoder level; per decoder level a nearest
 *   upsampling, a convolution + ReLU to C_l channels, the encoder skip added,
 *   and a second convolution + ReLU; a final convolution to one channel.
 * Inputs (four channels): d / sigma, log(N_pix / sigma^2) on observed
 * pixels (0 on masked ones), the mask, and the mean of d / sigma over the
 * observed pixels of the pixel's row (row-constant stripe noise spans whole
 * rows), with sigma^2 = mean N_pix over observed pixels of that map.
 * Output: the predicted field / sigma.
 *
 * Parameters: one float32 vector.  Convolution i in network order holds
 * W_i [3][3][ci_i][co_i] (row-major, the tap (dy+1, dx+1) first, then the
 * input channel, then the output channel) followed by b_i [co_i], with
 * ci_0 = 32 (four real input channels, the rest must be zero) and
 * co_14 = 32 (one real output channel, the rest must be zero).  The
 * convolution is a cross-correlation on the torus:
 *   out[y][x][co] = b[co] + sum_{dy,dx,ci} in[(y+dy)%H][(x+dx)%W][ci] W[dy+1][dx+1][ci][co].
 *
 * Maps: [n][H][W] stacked, H and W powers of two from 64 to 2048.  Map
 * pointers are DEVICE pointers in the precision of the context (float32 or
 * float64); the mask is uint8 (1 = observed) or NULL.  Every call is
 * stream-ordered on `stream`; calls returning host values synchronise it.
 * Errors: negative wf_status (wf.h); outputs are then unspecified.
 */
#ifndef WF_NN_H
#define WF_NN_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t h, w;        /* map size                                            */
  int32_t batch_max;   /* largest n passed to any call                        */
  int32_t precision;   /* wf_precision of the map arguments                   */
} wf_nn_shape;

/* Number of float32 parameters (the layout above). */
int64_t wf_nn_param_count(void);

/* Create a network workspace (activations for batch_max maps, optimiser
 * state).  Parameters start at zero; set them with wf_nn_set_params. */
wf_status wf_nn_create(const wf_nn_shape* shape, void** out);
void wf_nn_destroy(void* net);

/* Copy the parameter vector in (DEVICE float32 [param_count]); resets the
 * optimiser state.  Padded entries must be zero. */
wf_status wf_nn_set_params(void* net, const float* params, hipStream_t stream);
/* Copy the parameter vector out (DEVICE float32 [param_count]). */
wf_status wf_nn_get_params(void* net, float* params, hipStream_t stream);

/* Predict s for n maps: s_out [n][H][W] (DEVICE, context precision). */
wf_status wf_nn_predict(void* net, int32_t n, const void* d, const void* n_pix,
                        const uint8_t* mask, void* s_out, hipStream_t stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the mean squared error
 * between the network output and s_target / sigma over every pixel of the n
 * maps.  loss: HOST, receives the loss before the step (may be NULL). */
wf_status wf_nn_train_step(void* net, int32_t n, const void* d, const void* n_pix,
                           const uint8_t* mask, const void* s_target, float lr,
                           double* loss, hipStream_t stream);

/* Network alone, on given features: x [n][H][W][4] float32 (DEVICE).
 * y [n][H][W] float32 (DEVICE) receives the output channel. */
wf_status wf_nn_forward_features(void* net, int32_t n, const float* x, float* y,
                                 hipStream_t stream);

/* Gradient of the mean squared error between the output and target
 * [n][H][W] float32 (DEVICE) for features x: grad [param_count] float32
 * (DEVICE); loss HOST (may be NULL).  No update. */
wf_status wf_nn_gradient_features(void* net, int32_t n, const float* x, const float* target,
                                  float* grad, double* loss, hipStream_t stream);

/* One convolution building block on caller buffers (bfloat16 stored as
 * uint16, [P][C] with P = n*H*W pixels, channels contiguous):
 *   mode 0  out = in (*) W + b          out bf16 [P][co]
 *   mode 1  out = max(0, in (*) W + b)  out bf16 [P][co]
 *   mode 2  out = adjoint in the input: g [P][co] -> out bf16 [P][ci]
 *   mode 3  out = weight gradient: sum_p in[p + tap]^T g[p], float32 [3][3][ci][co]
 * w is bf16 [3][3][ci][co] (modes 0-2); b float32 [co] or NULL; for mode 3
 * `w` is unused and `g` is the output gradient.  ci, co multiples of 32 up to
 * 128; n*H*W a multiple of 64.  Allocates and frees a temporary (modes 0, 1
 * and 3) and synchronises the stream: a building block for tests, not for
 * the training loop. */
wf_status wf_nn_conv3x3(int32_t mode, int32_t n, int32_t h, int32_t w, int32_t ci, int32_t co,
                        const uint16_t* in, const uint16_t* wt, const float* b,
                        const uint16_t* g, void* out, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* WF_NN_H */
