// Internal declarations of the learned initial guess: device kernels of the
// 3D convolutional network (BF16 MFMA, FP32 accumulation) and their
// launchers.  Tensors are channels-last [z][y][x][c], bfloat16 stored as raw
// 16-bit patterns.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace nn {

using bf16_t = uint16_t;

// Geometry of a convolution, seen from its output:
//   SAME3: y[v]      = sum_t W_t x[v + o_t]   3x3x3 taps, zero padding
//   DOWN2: y[V]      = sum_t W_t x[2V + t]    2x2x2 taps, stride 2
//   UP2  : y[2V + t] =       W_t x[V]         transpose of DOWN2
enum Geom { G_SAME3 = 0, G_DOWN2 = 1, G_UP2 = 2 };

inline int geom_taps(int g) { return g == G_SAME3 ? 27 : 8; }

// One convolution (forward, or the input gradient of another convolution).
// Input: the channel concatenation of srcA (ca channels) and srcB (cb
// channels, may be 0) on the input grid.  Weights: w[cout][T][ca+cb]
// (T = 27 or 8).  Output channels [0, da) go to dstA, [da, da+db) to dstB
// on the output grid.  Epilogue per output value: + bias (if given), ReLU
// (if relu), times (mask > 0) (if a mask is given, same shape as the
// destination), + the destination's old value (if acc).
struct ConvArgs {
    int inx, iny, inz;
    int onx, ony, onz;
    const bf16_t *srcA;
    int ca;
    const bf16_t *srcB;
    int cb;
    const bf16_t *w;
    const float *bias;
    int relu;
    bf16_t *dstA;
    int da;
    bf16_t *dstB;
    int db;
    const bf16_t *maskA;
    const bf16_t *maskB;
    int accA, accB;
};
// cout = da + db must be 16, 32, 64 or 128; ca, cb multiples of 8.
hipError_t conv(hipStream_t s, int geom, const ConvArgs &a);

// Weight gradient of a convolution: partials[slice][cout][T][cin] (FP32)
// for the layer input x (concatenation of xA, xB on grid xdims) and the
// gradient g of its pre-activation output (cout channels on grid gdims).
struct WgradArgs {
    int xnx, xny, xnz;
    int gnx, gny, gnz;
    const bf16_t *xA;
    int ca;
    const bf16_t *xB;
    int cb;
    const bf16_t *g;
    int cout;
    float *partials;
    int nslice;
};
hipError_t wgrad(hipStream_t s, int geom, const WgradArgs &a);
// number of slices wgrad() uses for a layer whose reduction runs over a
// qx*qy*qz grid (the output grid, or the coarse input grid for UP2); the
// partials buffer holds nslice * cout * T * cin floats
int wgrad_slices(int geom, int qx, int qy, int qz, int cin, int cout, size_t max_floats);

// Bias gradient: partials[slice][c] = sum over the slice's cells of g[.][c]
// (c = 16, 32 or 64).
hipError_t bias_grad(hipStream_t s, const bf16_t *g, size_t cells, int c, float *partials, int nslice);

// out[map(i)] (+)= sum_j partials[j * stride + i] for i < n, summed in slice
// order; map(i) = (i / cinp) * cin_real + i % cinp, entries with
// i % cinp >= cin_real dropped (so a channel-padded weight gradient
// [cout][T][cinp] lands in its unpadded layout; cinp = cin_real = n for a
// plain vector).
// More than kReduceGroups slices are first summed in kReduceGroups groups
// into work (kReduceGroups * n floats), then the groups in order.
constexpr int kReduceGroups = 64;
hipError_t reduce_partials(hipStream_t s, const float *partials, int nslice, int n, int stride, int cinp,
                           int cin_real, float *out, int accumulate, float *work);

// max |s| over n FP64 values into *out (FP64); *out must hold 0 or less.
hipError_t maxabs(hipStream_t s, const double *x, size_t n, double *out);
// x8[v][0] = bf16(s[v] / *sigma) (1 if *sigma == 0), x8[v][1..7] = 0.
hipError_t prep_input(hipStream_t s, const double *src, size_t n, const double *sigma, bf16_t *x8);

// Head: y = wh f + bh with FP32 weights wh[3][kHeadIn], bias bh[3], and
// features f = (16 channels of a, then x = s / sigma at the 27 taps of the
// cell, FP32, zero outside the grid).
constexpr int kHeadIn = 16 + 27;
constexpr int kHeadRed = 3 * kHeadIn + 3 + 1;  // dW, db, sum of squared errors
// Prediction: guess_i[v] = sigma * coef_i * y_i[v]   (FP64 out)
hipError_t head_predict(hipStream_t s, const bf16_t *a, const double *src, int nx, int ny, int nz, const float *wh,
                        const float *bh, const double *sigma, const double coef[3], double *g0, double *g1,
                        double *g2);
// Training: mean-squared error against t[v][3]; writes the masked input
// gradient ga[v][16] (bf16) and per-block partials of (dW, db, sum of
// squared errors), kHeadRed floats per block.
int head_train_blocks(int nx, int ny, int nz);
hipError_t head_train(hipStream_t s, const bf16_t *a, const double *src, int nx, int ny, int nz, const float *wh,
                      const float *bh, const double *sigma, const float *t, bf16_t *ga, float *partials);
// Targets: t[v][i] = kappa2_i psi_i[v] / (*sigma * scale_i) (FP32), and
// max_i |t| into maxbits[i] (as float bit patterns; must start at 0).
hipError_t make_target(hipStream_t s, const double *psi0, const double *psi1, const double *psi2,
                       size_t n, const double kappa2[3], const double scale[3], const double *sigma,
                       float *t, unsigned *maxbits);

// Adam (Kingma & Ba, Algorithm 1) on n FP32 parameters with gradient
// g * gscale; step counts from 1.
hipError_t adam(hipStream_t s, float *theta, float *m, float *v, const float *g, size_t n, float gscale,
                float lr, float beta1, float beta2, float eps, int step);

// BF16 copies of one layer's weights from the FP32 master W[cout][T][cin]:
// wf[cout][T][cinp] (forward; channels >= cin are zero) and, if wd is
// given, the input-gradient weights wd[cin][T][cout] with taps mirrored
// (t -> T-1-t) for SAME3.
hipError_t pack_weights(hipStream_t s, int geom, const float *W, int cout, int cin, int cinp, bf16_t *wf,
                        bf16_t *wd);

hipError_t fill_zero(hipStream_t s, void *p, size_t bytes);
hipError_t bf16_to_f32(hipStream_t s, const bf16_t *src, float *dst, size_t n);

}  // namespace nn
