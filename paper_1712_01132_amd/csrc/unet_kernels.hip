// Kernels of the warm-start network: a U-Net trained on converged fields of the
// iteration that maps a solid mask and Kn to an initial density and velocity
// field (the iteration itself then runs unchanged from that start).
//
// The dense contractions (every 3x3 and 1x1 convolution, forward, backward
// with respect to the input, and the weight gradient) run on the gfx950 matrix
// cores: v_mfma_f32_16x16x32_bf16, bf16 operands, FP32 accumulation. Lane
// layout of that instruction (checked on the device): lane l holds
// A[m = l % 16][k = 8 (l / 16) + i] and B[k = 8 (l / 16) + i][n = l % 16],
// i = 0..7, and receives D[m = 4 (l / 16) + r][n = l % 16], r = 0..3.
#include <algorithm>

#include "unet_internal.h"

namespace pdvm_nn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);                                           // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

constexpr int kPitch = 40;  // LDS row pitch in bf16: 32 k values + 8 pad (conflict-free 16-byte reads)

// One 8-channel group of the im2col matrix: row = output pixel (b, y, x),
// columns k .. k+7 (k a multiple of 8). Zero outside the image along y (zero
// padding), circular along x (the periodic flow axis), zero beyond K.
struct Im2col {
  const uint16_t *xa, *xb;
  int Ca, Cb, ups, taps, H, W, K, Cin;
  __device__ __forceinline__ uint4 load(int b, int y, int x, int k) const {
    uint4 v = make_uint4(0, 0, 0, 0);
    if (k >= K) return v;
    const int tap = k / Cin;
    const int c = k - tap * Cin;
    const int dy = taps == 9 ? tap / 3 - 1 : 0;
    const int dx = taps == 9 ? tap % 3 - 1 : 0;
    const int yy = y + dy;
    if (yy < 0 || yy >= H) return v;
    int xx = x + dx;
    xx = xx < 0 ? xx + W : (xx >= W ? xx - W : xx);
    const uint16_t *src;
    if (c < Ca) {
      src = ups ? xa + ((int64_t)((b * (H >> 1) + (yy >> 1)) * (W >> 1) + (xx >> 1))) * Ca + c
                : xa + ((int64_t)((b * H + yy) * W + xx)) * Ca + c;
    } else {
      src = xb + ((int64_t)((b * H + yy) * W + xx)) * Cb + (c - Ca);
    }
    return *reinterpret_cast<const uint4 *>(src);
  }
};

// out tile: 128 pixels x BN output channels, 4 wavefronts of 32 pixels each.
template <int BN>
__global__ void __launch_bounds__(256) conv_kernel(ConvArgs a) {
  __shared__ uint4 As[128 * kPitch / 8];
  __shared__ uint4 Bs[BN * kPitch / 8];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int P = a.B * a.H * a.W;
  const int p0 = blockIdx.x * 128;
  const int n0 = blockIdx.y * BN;
  const int Cin = a.Ca + a.Cb;
  const int K = a.taps * Cin;
  const int nk = (K + 31) / 32;
  const Im2col im{a.xa, a.xb, a.Ca, a.Cb, a.ups, a.taps, a.H, a.W, K, Cin};

  int pb[2], py[2], px[2];
  bool pv[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int p = p0 + (tid >> 2) + 64 * i;
    pv[i] = p < P;
    const int q = pv[i] ? p : 0;
    px[i] = q % a.W;
    const int t = q / a.W;
    py[i] = t % a.H;
    pb[i] = t / a.H;
  }
  const int kg = (tid & 3) * 8;
  const int brow = tid >> 2;
  const bool bload = brow < BN && n0 + brow < a.nrows;

  uint4 ra[2], rb = make_uint4(0, 0, 0, 0);
  auto gload = [&](int kt) {
    const int k = kt * 32 + kg;
#pragma unroll
    for (int i = 0; i < 2; ++i) ra[i] = pv[i] ? im.load(pb[i], py[i], px[i], k) : make_uint4(0, 0, 0, 0);
    rb = make_uint4(0, 0, 0, 0);
    if (bload && k < K) rb = *reinterpret_cast<const uint4 *>(a.wt + (int64_t)(n0 + brow) * K + k);
  };

  f32x4 acc[2][BN / 16];
#pragma unroll
  for (int ms = 0; ms < 2; ++ms)
#pragma unroll
    for (int ns = 0; ns < BN / 16; ++ns) acc[ms][ns] = f32x4{0.f, 0.f, 0.f, 0.f};

  gload(0);
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) As[((tid >> 2) + 64 * i) * (kPitch / 8) + (tid & 3)] = ra[i];
    if (brow < BN) Bs[brow * (kPitch / 8) + (tid & 3)] = rb;
    __syncthreads();
    if (kt + 1 < nk) gload(kt + 1);
    bf16x8 fa[2], fb[BN / 16];
#pragma unroll
    for (int ms = 0; ms < 2; ++ms)
      fa[ms] = __builtin_bit_cast(bf16x8, As[(32 * wv + 16 * ms + (lane & 15)) * (kPitch / 8) + (lane >> 4)]);
#pragma unroll
    for (int ns = 0; ns < BN / 16; ++ns)
      fb[ns] = __builtin_bit_cast(bf16x8, Bs[(16 * ns + (lane & 15)) * (kPitch / 8) + (lane >> 4)]);
#pragma unroll
    for (int ms = 0; ms < 2; ++ms)
#pragma unroll
      for (int ns = 0; ns < BN / 16; ++ns)
        acc[ms][ns] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[ms], fb[ns], acc[ms][ns], 0, 0, 0);
  }

#pragma unroll
  for (int ns = 0; ns < BN / 16; ++ns) {
    const int n = n0 + 16 * ns + (lane & 15);
    if (n >= a.nstore) continue;
    const float bias = a.bias ? a.bias[n] : 0.f;
#pragma unroll
    for (int ms = 0; ms < 2; ++ms)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = p0 + 32 * wv + 16 * ms + 4 * (lane >> 4) + r;
        if (p >= P) continue;
        float v = acc[ms][ns][r] + bias;
        if (a.relu) v = fmaxf(v, 0.f);
        if (a.yb) a.yb[(int64_t)p * a.ystride + n] = f2bf(v);
        else a.yf[(int64_t)p * a.ystride + n] = v;
      }
  }
}

// dW partials: tile 64 output channels (rows m) x 32 columns k of the im2col
// matrix, reduction over 32 pixels per step. Both operands are pixel-major in
// memory, so they are transposed on their way into LDS.
__global__ void __launch_bounds__(256) wgrad_kernel(WgradArgs a) {
  __shared__ uint4 As[64 * kPitch / 8];
  __shared__ uint4 Bs[32 * kPitch / 8];
  uint16_t *As16 = reinterpret_cast<uint16_t *>(As);
  uint16_t *Bs16 = reinterpret_cast<uint16_t *>(Bs);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int P = a.B * a.H * a.W;
  const int m0 = blockIdx.x * 64;
  const int k0 = blockIdx.y * 32;
  const int pbeg = blockIdx.z * a.pix_per_split;
  const int pend = min(P, pbeg + a.pix_per_split);
  const int Cin = a.Ca + a.Cb;
  const int K = a.taps * Cin;
  const Im2col im{a.xa, a.xb, a.Ca, a.Cb, a.ups, a.taps, a.H, a.W, K, Cin};

  f32x4 acc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
  const int ga_pix = tid >> 3, ga_m = (tid & 7) * 8;  // G: 32 pixels x 64 rows
  const int gb_pix = tid >> 2, gb_k = (tid & 3) * 8;  // im2col: 32 pixels x 32 columns (tid < 128)
  for (int pp = pbeg; pp < pend; pp += 32) {
    uint4 va = make_uint4(0, 0, 0, 0), vb = make_uint4(0, 0, 0, 0);
    {
      const int p = pp + ga_pix;
      if (p < pend && m0 + ga_m < a.M)
        va = *reinterpret_cast<const uint4 *>(a.g + (int64_t)p * a.gstride + m0 + ga_m);
    }
    if (tid < 128) {
      const int p = pp + gb_pix;
      if (p < pend) {
        const int x = p % a.W, t = p / a.W;
        vb = im.load(t / a.H, t % a.H, x, k0 + gb_k);
      }
    }
    __syncthreads();
    {
      const uint16_t *e = reinterpret_cast<const uint16_t *>(&va);
#pragma unroll
      for (int i = 0; i < 8; ++i) As16[(ga_m + i) * kPitch + ga_pix] = e[i];
    }
    if (tid < 128) {
      const uint16_t *e = reinterpret_cast<const uint16_t *>(&vb);
#pragma unroll
      for (int i = 0; i < 8; ++i) Bs16[(gb_k + i) * kPitch + gb_pix] = e[i];
    }
    __syncthreads();
    const bf16x8 fa = __builtin_bit_cast(bf16x8, As[(16 * wv + (lane & 15)) * (kPitch / 8) + (lane >> 4)]);
#pragma unroll
    for (int ns = 0; ns < 2; ++ns) {
      const bf16x8 fb = __builtin_bit_cast(bf16x8, Bs[(16 * ns + (lane & 15)) * (kPitch / 8) + (lane >> 4)]);
      acc[ns] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[ns], 0, 0, 0);
    }
  }
  float *out = a.part + (int64_t)blockIdx.z * a.M * K;
#pragma unroll
  for (int ns = 0; ns < 2; ++ns) {
    const int k = k0 + 16 * ns + (lane & 15);
    if (k >= K) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + 16 * wv + 4 * (lane >> 4) + r;
      if (m < a.M) out[(int64_t)m * K + k] = acc[ns][r];
    }
  }
}

__global__ void sum_splits_kernel(const float *part, int splits, int64_t n, float *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int j = 0; j < splits; ++j) s += part[(int64_t)j * n + i];
  out[i] = s;
}

// Column sums of a bf16 matrix [P][gstride] over its first C columns (C divides
// 256), per block of kColsumPix rows: thread t sums column t % C over rows
// t / C, t / C + 256 / C, ...; then the block adds its 256 / C row lanes.
__global__ void __launch_bounds__(256) colsum_kernel(const uint16_t *g, int64_t P, int C, int gstride, float *part) {
  __shared__ float red[256];
  const int t = threadIdx.x;
  const int c = t % C, lanes = 256 / C;
  const int64_t beg = (int64_t)blockIdx.x * kColsumPix;
  const int64_t end = min(P, beg + kColsumPix);
  float s = 0.f;
  for (int64_t p = beg + t / C; p < end; p += lanes) s += bf2f(g[p * gstride + c]);
  red[t] = s;
  __syncthreads();
  if (t < C) {
    float a = 0.f;
    for (int j = 0; j < lanes; ++j) a += red[j * C + t];
    part[(int64_t)blockIdx.x * C + t] = a;
  }
}

// Input tensor [B][H][W][8]: solid (0/1), the scaled log Kn feature, zeros.
__global__ void build_input_kernel(const uint8_t *solid_set, const float *feat_set, Slots sl, int B, int H, int W,
                                   uint16_t *x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t HW = (int64_t)H * W;
  if (i >= B * HW) return;
  const int b = (int)(i / HW);
  const int64_t c = i - b * HW;
  const int s = sl.s[b];
  uint4 v = make_uint4(0, 0, 0, 0);
  v.x = (uint32_t)f2bf(solid_set[s * HW + c] ? 1.f : 0.f) | ((uint32_t)f2bf(feat_set[s]) << 16);
  reinterpret_cast<uint4 *>(x)[i] = v;  // kInC = 8 bf16 = 16 bytes per voxel
}

__global__ void relu_grad_kernel(const float *dy, const uint16_t *y, int64_t n, uint16_t *g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  g[i] = f2bf(bf2f(y[i]) > 0.f ? dy[i] : 0.f);
}

// 2x2 max pooling (first maximum in the order (0,0), (0,1), (1,0), (1,1)).
__global__ void maxpool_kernel(const uint16_t *x, int B, int H, int W, int C, uint16_t *y, uint8_t *idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int Ho = H / 2, Wo = W / 2;
  if (i >= (int64_t)B * Ho * Wo * C) return;
  const int c = (int)(i % C);
  int64_t t = i / C;
  const int xo = (int)(t % Wo);
  t /= Wo;
  const int yo = (int)(t % Ho);
  const int b = (int)(t / Ho);
  float best = 0.f;
  int bi = 0;
  for (int j = 0; j < 4; ++j) {
    const int yy = 2 * yo + (j >> 1), xx = 2 * xo + (j & 1);
    const float v = bf2f(x[((int64_t)(b * H + yy) * W + xx) * C + c]);
    if (j == 0 || v > best) {
      best = v;
      bi = j;
    }
  }
  y[i] = f2bf(best);
  idx[i] = (uint8_t)bi;
}

__global__ void maxpool_back_kernel(const float *dy, const uint8_t *idx, int B, int H, int W, int C, float *dx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int Ho = H / 2, Wo = W / 2;
  if (i >= (int64_t)B * Ho * Wo * C) return;
  const int c = (int)(i % C);
  int64_t t = i / C;
  const int xo = (int)(t % Wo);
  t /= Wo;
  const int yo = (int)(t % Ho);
  const int b = (int)(t / Ho);
  const int j = idx[i];
  const int yy = 2 * yo + (j >> 1), xx = 2 * xo + (j & 1);
  dx[((int64_t)(b * H + yy) * W + xx) * C + c] += dy[i];
}

// Gradient at a concatenated [up(A), B] input: A's part summed over each 2x2
// block (nearest upsampling), B's part copied.
__global__ void concat_back_kernel(const float *dcat, int B, int H, int W, int Ca, int Cb, float *da, float *db) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int C = Ca + Cb;
  const int Ho = H / 2, Wo = W / 2;
  const int64_t na = (int64_t)B * Ho * Wo * Ca;
  if (i < na) {
    const int c = (int)(i % Ca);
    int64_t t = i / Ca;
    const int xo = (int)(t % Wo);
    t /= Wo;
    const int yo = (int)(t % Ho);
    const int b = (int)(t / Ho);
    float s = 0.f;
    for (int j = 0; j < 4; ++j) {
      const int yy = 2 * yo + (j >> 1), xx = 2 * xo + (j & 1);
      s += dcat[((int64_t)(b * H + yy) * W + xx) * C + c];
    }
    da[i] = s;
  }
  const int64_t nb = (int64_t)B * H * W * Cb;
  if (i < nb) {
    const int c = (int)(i % Cb);
    const int64_t p = i / Cb;
    db[i] = dcat[p * C + Ca + c];
  }
}

// Masked squared error over the fluid voxels, per sample weight wsamp (1 / (3 nf)),
// averaged over the batch. Writes the bf16 gradient at the head output
// ([p][32], channels >= 3 zero) and per-block partial losses.
__global__ void loss_kernel(const float *pred, const uint8_t *solid_set, const float *target_set, const float *wsamp,
                            Slots sl, int B, int H, int W, uint16_t *g, float *part) {
  __shared__ float red[256];
  const int64_t HW = (int64_t)H * W;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (i < B * HW) {
    const int b = (int)(i / HW);
    const int64_t c = i - b * HW;
    const int s = sl.s[b];
    const bool fluid = solid_set[s * HW + c] == 0;
    const float w = wsamp[s] / (float)B;
    uint16_t o3[3];
    for (int ch = 0; ch < 3; ++ch) {
      const float d = fluid ? pred[i * 4 + ch] - target_set[(s * 3 + ch) * HW + c] : 0.f;
      l += w * d * d;
      o3[ch] = f2bf(2.f * w * d);
    }
    uint4 *dst = reinterpret_cast<uint4 *>(g + i * 32);
    dst[0] = make_uint4((uint32_t)o3[0] | ((uint32_t)o3[1] << 16), (uint32_t)o3[2], 0u, 0u);
    dst[1] = dst[2] = dst[3] = make_uint4(0, 0, 0, 0);
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void to_bf16_kernel(const float *src, int64_t n, uint16_t *dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = f2bf(src[i]);
}

// Weights of the input-gradient convolution: wb[c][t * Cout + o] = wt[o][(taps-1-t) * Cin + c].
__global__ void wt_back_kernel(const uint16_t *wt, int Cout, int Cin, int taps, uint16_t *wb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)Cout * Cin * taps) return;
  const int o = (int)(i % Cout);
  int64_t r = i / Cout;
  const int t = (int)(r % taps);
  const int c = (int)(r / taps);
  wb[i] = wt[(int64_t)o * taps * Cin + (int64_t)(taps - 1 - t) * Cin + c];
}

__device__ double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

__device__ __forceinline__ double usigma(double kn256) {
  const double a = kKnKnee * kn256;
  return a / (1.0 + a);
}

// Normalised targets of one sample (one block of 1024 threads):
// t0 = (rho + J (x1 - 1/2) - mean over fluid) N1 / (256 J),
// t1, t2 = U sigma(Kn256) u_j N1 / (256 J); zero on solid voxels.
__global__ void __launch_bounds__(1024) targets_kernel(const uint8_t *solid, const double *rho, const double *u,
                                                       int H, int W, double jump, double kn256, float *target,
                                                       float *wsamp_one) {
  __shared__ double red[1024];
  const int64_t HW = (int64_t)H * W;
  double s = 0, c = 0;
  for (int64_t i = threadIdx.x; i < HW; i += blockDim.x) {
    if (solid[i]) continue;
    const int x = (int)(i % W);
    s += rho[i] + jump * ((x + 0.5) / W - 0.5);
    c += 1;
  }
  s = block_sum(s, red);
  c = block_sum(c, red);
  const double mean = c > 0 ? s / c : 0.0;
  const double gscale = W / (kRefLen * jump);
  const double us = kUScale * usigma(kn256) * gscale;
  for (int64_t i = threadIdx.x; i < HW; i += blockDim.x) {
    const int x = (int)(i % W);
    const bool f = !solid[i];
    target[i] = f ? (float)((rho[i] + jump * ((x + 0.5) / W - 0.5) - mean) * gscale) : 0.f;
    target[HW + i] = f ? (float)(u[i] * us) : 0.f;
    target[2 * HW + i] = f ? (float)(u[HW + i] * us) : 0.f;
  }
  if (threadIdx.x == 0) *wsamp_one = c > 0 ? (float)(1.0 / (3.0 * c)) : 0.f;
}

// Physical fields from the network output of one sample (the inverse of the
// target normalisation, mean density 0); solid voxels read 0.
__global__ void fields_kernel(const float *pred, const uint8_t *solid, int H, int W, double jump, double kn256,
                              double *rho, double *u) {
  const int64_t HW = (int64_t)H * W;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= HW) return;
  const int x = (int)(i % W);
  const bool f = !solid[i];
  const double gscale = W / (kRefLen * jump);
  const double us = kUScale * usigma(kn256) * gscale;
  rho[i] = f ? pred[i * 4] / gscale - jump * ((x + 0.5) / W - 0.5) : 0.0;
  u[i] = f ? pred[i * 4 + 1] / us : 0.0;
  u[HW + i] = f ? pred[i * 4 + 2] / us : 0.0;
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_conv(const ConvArgs &a, hipStream_t st) {
  const int P = a.B * a.H * a.W;
  const bool wide = a.nstore > 32 && a.nrows % 64 == 0;
  if (wide) {
    dim3 grid(nblocks(P, 128), (unsigned)((a.nstore + 63) / 64));
    conv_kernel<64><<<grid, 256, 0, st>>>(a);
  } else {
    dim3 grid(nblocks(P, 128), (unsigned)((a.nstore + 31) / 32));
    conv_kernel<32><<<grid, 256, 0, st>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_wgrad(const WgradArgs &a, int splits, hipStream_t st) {
  const int K = a.taps * (a.Ca + a.Cb);
  dim3 grid((unsigned)((a.M + 63) / 64), (unsigned)((K + 31) / 32), (unsigned)splits);
  wgrad_kernel<<<grid, 256, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_sum_splits(const float *part, int splits, int64_t n, float *out, hipStream_t st) {
  sum_splits_kernel<<<nblocks(n, 256), 256, 0, st>>>(part, splits, n, out);
  return hipGetLastError();
}

hipError_t launch_colsum(const uint16_t *g, int64_t P, int C, int gstride, float *part, int splits, hipStream_t st) {
  colsum_kernel<<<(unsigned)splits, 256, 0, st>>>(g, P, C, gstride, part);
  return hipGetLastError();
}

hipError_t launch_build_input(const uint8_t *solid_set, const float *feat_set, Slots sl, int B, int H, int W,
                              uint16_t *x, hipStream_t st) {
  build_input_kernel<<<nblocks((int64_t)B * H * W, 256), 256, 0, st>>>(solid_set, feat_set, sl, B, H, W, x);
  return hipGetLastError();
}

hipError_t launch_relu_grad(const float *dy, const uint16_t *y, int64_t n, uint16_t *g, hipStream_t st) {
  relu_grad_kernel<<<nblocks(n, 256), 256, 0, st>>>(dy, y, n, g);
  return hipGetLastError();
}

hipError_t launch_maxpool(const uint16_t *x, int B, int H, int W, int C, uint16_t *y, uint8_t *idx, hipStream_t st) {
  maxpool_kernel<<<nblocks((int64_t)B * (H / 2) * (W / 2) * C, 256), 256, 0, st>>>(x, B, H, W, C, y, idx);
  return hipGetLastError();
}

hipError_t launch_maxpool_back(const float *dy, const uint8_t *idx, int B, int H, int W, int C, float *dx,
                               hipStream_t st) {
  maxpool_back_kernel<<<nblocks((int64_t)B * (H / 2) * (W / 2) * C, 256), 256, 0, st>>>(dy, idx, B, H, W, C, dx);
  return hipGetLastError();
}

hipError_t launch_concat_back(const float *dcat, int B, int H, int W, int Ca, int Cb, float *da, float *db,
                              hipStream_t st) {
  const int64_t n = std::max((int64_t)B * (H / 2) * (W / 2) * Ca, (int64_t)B * H * W * Cb);
  concat_back_kernel<<<nblocks(n, 256), 256, 0, st>>>(dcat, B, H, W, Ca, Cb, da, db);
  return hipGetLastError();
}

hipError_t launch_loss(const float *pred, const uint8_t *solid_set, const float *target_set, const float *wsamp,
                       Slots sl, int B, int H, int W, uint16_t *g, float *part, int nblk, hipStream_t st) {
  loss_kernel<<<(unsigned)nblk, 256, 0, st>>>(pred, solid_set, target_set, wsamp, sl, B, H, W, g, part);
  return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t st) {
  adam_kernel<<<nblocks(n, 256), 256, 0, st>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float *src, int64_t n, uint16_t *dst, hipStream_t st) {
  to_bf16_kernel<<<nblocks(n, 256), 256, 0, st>>>(src, n, dst);
  return hipGetLastError();
}

hipError_t launch_wt_back(const uint16_t *wt, int Cout, int Cin, int taps, uint16_t *wb, hipStream_t st) {
  wt_back_kernel<<<nblocks((int64_t)Cout * Cin * taps, 256), 256, 0, st>>>(wt, Cout, Cin, taps, wb);
  return hipGetLastError();
}

hipError_t launch_targets(const uint8_t *solid, const double *rho, const double *u, int H, int W, double jump,
                          double kn256, float *target, float *wsamp_one, hipStream_t st) {
  targets_kernel<<<1, 1024, 0, st>>>(solid, rho, u, H, W, jump, kn256, target, wsamp_one);
  return hipGetLastError();
}

hipError_t launch_fields(const float *pred, const uint8_t *solid, int H, int W, double jump, double kn256,
                         double *rho, double *u, hipStream_t st) {
  fields_kernel<<<nblocks((int64_t)H * W, 256), 256, 0, st>>>(pred, solid, H, W, jump, kn256, rho, u);
  return hipGetLastError();
}

}  // namespace pdvm_nn
