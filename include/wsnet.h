/*
 * wsnet: the learned initial guess for the BiCGSafe solvers (C ABI).
 *
 * A small U-Net maps the coefficient fields of a 2D convection-diffusion
 * problem on an H x W grid (NHWC float input, `cin` channels per node) to an
 * approximation of its solution (one float per node).  The solver then starts
 * from that approximation instead of x0 = 0 (ps_options.x0_fallback keeps
 * x0 = 0 whenever the guess is worse than zero).  This predictor is not part
 * of the paper's method; it is an extension that shortens the Krylov
 * iteration by starting closer to the solution.
 *
 * Architecture (c = base channels, all convolutions 3x3, zero padding, ReLU):
 *   level 0 (H x W):      conv(cin->c), conv(c->c) = s0
 *   level 1 (H/2):  pool, conv(c->2c), conv(2c->2c) = s1
 *   level 2 (H/4):  pool, conv(2c->4c), conv(4c->4c) = s2
 *   level 3 (H/8):  pool, conv(4c->4c)
 *   up, concat s2, conv(8c->4c); up, concat s1, conv(6c->2c);
 *   up, concat s0, conv(3c->c); 1x1 conv(c->1) without activation.
 * 2x2 average pooling, nearest 2x upsampling.  Activations, gradients and the
 * convolution weights used by the kernels are bfloat16 (round to nearest
 * even); every 3x3 convolution and its two gradients run as matrix-core
 * products with fp32 accumulation; the master parameters, their Adam moments,
 * the 1x1 head and the loss are fp32.
 *
 * Parameter vector (fp32): for each 3x3 layer in the order above, the weights
 * W[co][tap][ci] (tap = 3*(dy+1) + (dx+1), input channels padded to a multiple
 * of 16 for the first layer) then the biases [co]; then the head weights [c]
 * and its bias.
 *
 * Return codes: 0 ok, -1 invalid argument, -2 out of memory, -3 HIP error,
 * -5 no gfx950 device.  Handles are not thread-safe.
 */
#ifndef WSNET_H
#define WSNET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ws_net ws_net;

/* H, W: multiples of 8; cin in [1, 16]; c in {16} (base channels).  The
   parameters are initialised from `seed` (He-uniform weights, zero biases). */
int ws_create(ws_net **out, int32_t H, int32_t W, int32_t cin, int32_t c, uint64_t seed);
int ws_destroy(ws_net *net);

/* number of fp32 parameters */
int64_t ws_num_params(const ws_net *net);
/* copy the fp32 parameters to / from HOST float[ws_num_params] (resets Adam) */
int ws_get_params(ws_net *net, float *host);
int ws_set_params(ws_net *net, const float *host);

/* Predict for `count` inputs: x DEVICE float[count][H][W][cin], y DEVICE
   float[count][H][W] = scale * network output.  Ordered on `stream`
   (hipStream_t, NULL = the null stream); returns after completion. */
int ws_forward(ws_net *net, const float *x, float *y, int32_t count, float scale, void *stream);

/* Forward, mean squared error against t DEVICE float[count][H][W], and the
   gradient of that loss with respect to every parameter, without updating:
   grad HOST float[ws_num_params], *loss HOST (the mean over count*H*W
   nodes).  count <= 64. */
int ws_gradients(ws_net *net, const float *x, const float *t, int32_t count, float *grad,
                 double *loss);

/* Train with Adam (beta1 0.9, beta2 0.999, eps 1e-8) on `count` samples x, t
   (DEVICE, layouts as above) in mini-batches of `batch` (<= 64) for `epochs`
   passes, the sample order of each pass drawn from `seed`; the learning rate
   falls from lr to lr/10 over the run (cosine).  loss_hist: NULL or HOST
   double[epochs], the mean loss of each pass. */
int ws_train(ws_net *net, const float *x, const float *t, int64_t count, int32_t batch,
             int32_t epochs, float lr, uint64_t seed, double *loss_hist);

#ifdef __cplusplus
}
#endif

#endif /* WSNET_H */
