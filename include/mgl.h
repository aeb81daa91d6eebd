/*
 * mgl.h — C ABI of the learned initial guess for the three screened
 * photon-group solves of the radiative-transfer model (paper Sec. 2: the
 * three-term Helmholtz equations (kappa_i^2 - lap) Psi_i = f_i, all driven
 * by the same ionisation source s).
 *
 * A 3D convolutional U-net maps the source field s to the three fields
 * kappa_i^2 Psi_i; each becomes the initial iterate of its own multigrid
 * solve (mg_solve with MG_GUESS, which falls back to a zero start when the
 * guess's residual exceeds that of zero).  The network runs in bfloat16
 * with FP32 accumulation on the matrix cores, in hand-written kernels, for
 * inference and for training (forward, input and weight gradients, Adam).
 *
 * Network (channels-last tensors [z][y][x][c]):
 *   level 0 (n)    e0a conv3 1->16, e0b conv3 16->16 (skip 0), d0 down2 16->32
 *   level 1 (n/2)  e1a conv3 32->32, e1b conv3 32->32 (skip 1), d1 down2 32->64
 *   level 2 (n/4)  e2a conv3 64->64, e2b conv3 64->64 (skip 2), d2 down2 64->64
 *   level 3 (n/8)  b3a conv3 64->64, b3b conv3 64->64, u2 up2 64->64
 *   level 2        c2a conv3 (64+64)->64, c2b conv3 64->64, u1 up2 64->32
 *   level 1        c1a conv3 (32+32)->32, c1b conv3 32->32, u0 up2 32->16
 *   level 0        c0a conv3 (16+16)->16, c0b conv3 16->16,
 *                  head: linear map of (c0b's 16 channels, x at the 27 taps
 *                  of the cell) -> 3
 * conv3 = 3x3x3 cross-correlation with zero padding, down2 = 2x2x2
 * stride-2 cross-correlation, up2 = its transpose, (a+b) = concatenation
 * (upsampled channels first); every layer but the head adds a bias and
 * applies ReLU.  Input x = s / max|s|; outputs y_i are in units of scale_i:
 * kappa_i^2 Psi_i = max|s| * scale_i * y_i.  The head's direct 3x3x3 path
 * from x (FP32) carries the local part of the fields past the bfloat16
 * network.
 *
 * Parameters: one flat FP32 vector, the layers in the order above, each as
 * W[cout][tap][cin] (C order; taps t = (dz+1)*9 + (dy+1)*3 + (dx+1) for
 * conv3 with offset (dz,dy,dx), t = tz*4 + ty*2 + tx for down2/up2; the
 * head is W[3][16 + 27]) followed by b[cout].  mgl_num_params() gives its
 * length.  The FP32 vector is the master copy; the kernels use bfloat16
 * copies of the weights (FP32 biases and head).
 *
 * Fields: FP64 [nz][ny][nx] device arrays as in mg.h; targets are FP32
 * [nz][ny][nx][3] device arrays.  Status codes are those of mg.h; the text
 * of the last error on the calling thread comes from mgl_last_error().
 * All device work is enqueued on the stream given to mgl_create; calls that
 * return host values synchronise it.  A network object must not be used
 * from two threads at once.
 */
#ifndef MGL_H_INCLUDED
#define MGL_H_INCLUDED

#include <stddef.h>

#include "mg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgl_net mgl_net; /* opaque, owned by the library */

/* Grid the network runs on; every axis a positive multiple of 8. */
typedef struct {
    int nx, ny, nz;
} mgl_desc;

/* Adam hyper-parameters (Kingma & Ba, Algorithm 1). */
typedef struct {
    float lr, beta1, beta2, eps;
} mgl_adam;

/* Allocates the network's activations, gradients and optimiser state for
 * one grid on the device; parameters start at zero (set them with
 * mgl_init_params, mgl_set_params or mgl_load) and scales at 1. */
int mgl_create(const mgl_desc *d, void *hip_stream, mgl_net **out);
int mgl_destroy(mgl_net *n);
const char *mgl_last_error(void);
size_t mgl_num_params(void);

/* He-normal weights (std sqrt(2/fan_in), 1/fan_in for the head) and zero
 * biases from a counter-based generator seeded by `seed`; resets Adam. */
int mgl_init_params(mgl_net *n, unsigned long long seed);
/* Copy the FP32 master parameters from / to host memory (count must equal
 * mgl_num_params()).  Setting resets Adam. */
int mgl_set_params(mgl_net *n, const float *host, size_t count);
int mgl_get_params(mgl_net *n, float *host, size_t count);
/* Output scales scale_i (> 0, finite). */
int mgl_set_scales(mgl_net *n, const double scale[3]);
int mgl_get_scales(const mgl_net *n, double scale[3]);

/* Training target of one source: t[v][i] = kappa2_i psi_i[v] / (max|s|
 * scale_i), with psi_i the three converged solutions for source s.  If
 * maxabs is given it receives max_v |t[v][i]| per channel (synchronises). */
int mgl_make_target(mgl_net *n, const double *s_dev, const double *const psi_dev[3], const double kappa2[3],
                    float *t_dev, double maxabs[3]);

/* One optimiser step on a mini-batch of `count` samples: forward, mean
 * squared error over cells and the 3 channels, backward, gradients summed
 * over the samples, then one Adam update with the mean gradient (opt may
 * be NULL, or have lr = 0, to compute gradients only).  *loss (optional)
 * receives the mean loss over the samples (synchronises). */
int mgl_train_step(mgl_net *n, int count, const double *const *s_dev, const float *const *t_dev,
                   const mgl_adam *opt, double *loss);
/* Loss of one sample without a gradient (synchronises). */
int mgl_eval_loss(mgl_net *n, const double *s_dev, const float *t_dev, double *loss);
/* Summed gradient of the last mgl_train_step, FP32, flat layout. */
int mgl_get_grads(mgl_net *n, float *host, size_t count);

/* Initial guesses Psi_i = max|s| scale_i y_i / kappa2_i (FP64 device
 * arrays, overwritten) for the source s. */
int mgl_predict(mgl_net *n, const double *s_dev, const double kappa2[3], double *const guess_dev[3]);

/* Parameters and scales to / from a file: "MGLW", a version, the parameter
 * count, the 3 scales (FP64) and the FP32 parameter vector, little-endian. */
int mgl_save(mgl_net *n, const char *path);
int mgl_load(mgl_net *n, const char *path);

/* Inspection: layer `layer` (0..19 in the order above, the head excluded)
 * output activation (which = 0, after ReLU) or gradient of its
 * pre-activation output (which = 1) from the last forward / backward pass,
 * as FP32 into host memory [z][y][x][c].  layer = -1, which = 0 is the
 * scaled input x (8 channels, channel 0 used). */
int mgl_read_tensor(mgl_net *n, int which, int layer, float *host, size_t count);
/* Shape of that tensor: dims[0..3] = nz, ny, nx, channels. */
int mgl_tensor_shape(const mgl_net *n, int layer, int dims[4]);

#ifdef __cplusplus
}
#endif

#endif /* MGL_H_INCLUDED */
