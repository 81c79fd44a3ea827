// Internal declarations of the warm-start network kernels (unet_kernels.hip)
// used by its host runtime (unet_host.cpp). Not part of the public C ABI.
//
// Tensors are NHWC: element (b, y, x, c) at ((b * H + y) * W + x) * C + c,
// x = the flow axis x1 (periodic: circular padding), y = x2 (zero padding).
// Activations and MFMA operands are bfloat16 (stored as raw 16-bit words,
// rounded to nearest even); accumulation, biases, gradients of activations and
// master weights are FP32.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace pdvm_nn {

constexpr int kMaxBatch = 32;
constexpr int kInC = 8;  // input channels: solid, scaled log Kn, six zero pads
constexpr int kColsumPix = 1024;  // rows per block of the column sums (bias gradients)

struct Slots {
  int32_t s[kMaxBatch];
};

// Convolution as an implicit GEMM: out[p][n] = sum_k A[p][k] Wt[n][k] (+ bias,
// ReLU), k = tap * Cin + c over `taps` (9: 3x3, or 1: 1x1) and the
// concatenated input channels [A (Ca, optionally read at (y/2, x/2)), B (Cb)].
struct ConvArgs {
  const uint16_t *xa;
  const uint16_t *xb;
  int Ca, Cb, ups;
  const uint16_t *wt;  // [nrows][taps * (Ca + Cb)]
  int nrows;           // weight rows allocated (>= every stored n)
  const float *bias;   // [nrows] or null
  int taps;
  int B, H, W;
  int relu;
  uint16_t *yb;        // bf16 output or null
  float *yf;           // fp32 output or null
  int nstore, ystride; // channels stored, channel stride of the output
};

// Weight gradient partials: part[split][m][k] = sum over the split's pixels of
// G[p][m] * A[p][k], with G the bf16 gradient at the conv output (channel
// stride gstride) and A the im2col matrix of the conv input.
struct WgradArgs {
  const uint16_t *g;
  int gstride, M;      // M = output channels (rows of dW)
  const uint16_t *xa;
  const uint16_t *xb;
  int Ca, Cb, ups, taps;
  int B, H, W;
  int pix_per_split;
  float *part;         // [splits][M][K]
};

hipError_t launch_conv(const ConvArgs &a, hipStream_t st);
hipError_t launch_wgrad(const WgradArgs &a, int splits, hipStream_t st);
hipError_t launch_sum_splits(const float *part, int splits, int64_t n, float *out, hipStream_t st);
// splits = ceil(P / kColsumPix) blocks; part[split][C]
hipError_t launch_colsum(const uint16_t *g, int64_t P, int C, int gstride, float *part, int splits, hipStream_t st);
hipError_t launch_build_input(const uint8_t *solid_set, const float *feat_set, Slots sl, int B, int H, int W,
                              uint16_t *x, hipStream_t st);
hipError_t launch_relu_grad(const float *dy, const uint16_t *y, int64_t n, uint16_t *g, hipStream_t st);
hipError_t launch_maxpool(const uint16_t *x, int B, int H, int W, int C, uint16_t *y, uint8_t *idx, hipStream_t st);
hipError_t launch_maxpool_back(const float *dy, const uint8_t *idx, int B, int H, int W, int C, float *dx,
                               hipStream_t st);
hipError_t launch_concat_back(const float *dcat, int B, int H, int W, int Ca, int Cb, float *da_half, float *db,
                              hipStream_t st);
hipError_t launch_loss(const float *pred, const uint8_t *solid_set, const float *target_set, const float *wsamp,
                       Slots sl, int B, int H, int W, uint16_t *g, float *part, int nblk, hipStream_t st);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t st);
hipError_t launch_to_bf16(const float *src, int64_t n, uint16_t *dst, hipStream_t st);
hipError_t launch_wt_back(const uint16_t *wt, int Cout, int Cin, int taps, uint16_t *wb, hipStream_t st);
hipError_t launch_targets(const uint8_t *solid, const double *rho, const double *u, int H, int W, double jump,
                          double kn256, float *target, float *wsamp_one, hipStream_t st);
hipError_t launch_fields(const float *pred, const uint8_t *solid, int H, int W, double jump, double kn256,
                         double *rho, double *u, hipStream_t st);

// Normalisation shared by training targets and predictions.
constexpr double kUScale = 10.0;   // U
constexpr double kKnKnee = 10.0;   // a in sigma(K) = a K / (1 + a K)
constexpr double kRefLen = 256.0;  // voxels of the reference length of Kn and of the gradient

}  // namespace pdvm_nn
