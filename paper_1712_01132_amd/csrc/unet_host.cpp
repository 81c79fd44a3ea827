// Host runtime of the warm-start network (include/poredvm_unet.h): parameter
// and activation storage in one device arena, the layer schedule of the
// forward and backward passes, Adam, the device-resident training set.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/poredvm.h"
#include "../../include/poredvm_unet.h"
#include "unet_internal.h"

using namespace pdvm_nn;

namespace {

thread_local std::string g_unet_thread_error;

// Activation tensors (NHWC, bf16). Level l has resolution (H >> l) x (W >> l).
enum Act {
  X, E1A, E1, P1, E2A, E2, P2, E3A, E3, P3, B1, B2, D3A, D3, D2A, D2, D1A, D1, NACT
};
struct ActInfo {
  int level, ch;
};
const ActInfo kAct[NACT] = {{0, kInC}, {0, 32}, {0, 32}, {1, 32},  {1, 64},  {1, 64},
                            {2, 64},   {2, 128}, {2, 128}, {3, 128}, {3, 256}, {3, 256},
                            {2, 128},  {2, 128}, {1, 64},  {1, 64},  {0, 32},  {0, 32}};

struct LayerDef {
  int in_a, in_b;  // input tensors (in_b = -1: none); in_a is upsampled when in_b >= 0
  int out;         // output tensor (-1: the head's FP32 prediction)
  int cout, taps;
};
constexpr int kLayers = 15;
const LayerDef kLayer[kLayers] = {
    {X, -1, E1A, 32, 9},    {E1A, -1, E1, 32, 9},   {P1, -1, E2A, 64, 9},   {E2A, -1, E2, 64, 9},
    {P2, -1, E3A, 128, 9},  {E3A, -1, E3, 128, 9},  {P3, -1, B1, 256, 9},   {B1, -1, B2, 256, 9},
    {B2, E3, D3A, 128, 9},  {D3A, -1, D3, 128, 9},  {D3, E2, D2A, 64, 9},   {D2A, -1, D2, 64, 9},
    {D2, E1, D1A, 32, 9},   {D1A, -1, D1, 32, 9},   {D1, -1, -1, 3, 1}};
constexpr int kHeadRows = 32;  // the head's 3 output rows are padded to one 32-row MFMA tile

int cin_of(int l) { return kAct[kLayer[l].in_a].ch + (kLayer[l].in_b >= 0 ? kAct[kLayer[l].in_b].ch : 0); }
int rows_of(int l) { return l == kLayers - 1 ? kHeadRows : kLayer[l].cout; }
int level_of(int l) { return kLayer[l].in_b >= 0 ? kAct[kLayer[l].in_b].level : kAct[kLayer[l].in_a].level; }

int64_t logical_params() {
  int64_t n = 0;
  for (int l = 0; l < kLayers; ++l) n += (int64_t)kLayer[l].cout * kLayer[l].taps * cin_of(l) + kLayer[l].cout;
  return n;
}

constexpr int kPixPerSplit = 4096;

}  // namespace

struct pdvm_unet {
  int n1 = 0, n2 = 0, bmax = 0, smax = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  char *arena = nullptr;
  // parameters (internal layout: logical, with the head padded to kHeadRows rows)
  int64_t np = 0;
  std::vector<int64_t> offw, offb;
  float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
  uint16_t *wbf = nullptr, *wback = nullptr;
  int64_t adam_t = 0;
  // activations
  uint16_t *act[NACT] = {};
  float *gact[NACT] = {};
  uint8_t *pidx[3] = {};
  float *pred = nullptr, *dcat = nullptr, *part = nullptr, *bpart = nullptr, *loss_part = nullptr;
  uint16_t *gbuf = nullptr;
  int64_t part_n = 0, bpart_n = 0;
  int loss_blocks = 0;
  // training set (slot smax is the inference slot)
  uint8_t *ds_solid = nullptr;
  float *ds_feat = nullptr, *ds_target = nullptr, *ds_wsamp = nullptr;
  double *tmp_f64 = nullptr;
  float *h_loss = nullptr;  // pinned
  // timing of MFMA kernels
  bool timing = false;
  std::vector<hipEvent_t> tev;
  size_t tev_used = 0;

  int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    err = buf;
    return code;
  }
  int H(int level) const { return n2 >> level; }
  int W(int level) const { return n1 >> level; }
  int64_t pix(int B, int level) const { return (int64_t)B * H(level) * W(level); }
};

namespace {

#define UCHK(net, call)                                                                          \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) return (net)->fail(PDVM_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

hipError_t mfma_begin(pdvm_unet *n) {
  if (!n->timing) return hipSuccess;
  if (n->tev_used + 2 > n->tev.size()) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&b);
    if (e != hipSuccess) return e;
    n->tev.push_back(a);
    n->tev.push_back(b);
  }
  return hipEventRecord(n->tev[n->tev_used], n->stream);
}
hipError_t mfma_end(pdvm_unet *n) {
  if (!n->timing) return hipSuccess;
  hipError_t e = hipEventRecord(n->tev[n->tev_used + 1], n->stream);
  n->tev_used += 2;
  return e;
}

int check_slots(pdvm_unet *n, const int32_t *slots, int B, Slots &sl, bool allow_infer) {
  if (!slots || B < 1 || B > n->bmax) return n->fail(PDVM_E_INVAL, "batch must be 1..%d", n->bmax);
  for (int b = 0; b < B; ++b) {
    const int lim = allow_infer ? n->smax + 1 : n->smax;
    if (slots[b] < 0 || slots[b] >= lim) return n->fail(PDVM_E_INVAL, "slot %d out of range", slots[b]);
    sl.s[b] = slots[b];
  }
  return PDVM_OK;
}

ConvArgs conv_args(pdvm_unet *n, int l, int B) {
  const LayerDef &L = kLayer[l];
  ConvArgs a{};
  const int lev = level_of(l);
  a.xa = n->act[L.in_a];
  a.Ca = kAct[L.in_a].ch;
  a.xb = L.in_b >= 0 ? n->act[L.in_b] : nullptr;
  a.Cb = L.in_b >= 0 ? kAct[L.in_b].ch : 0;
  a.ups = L.in_b >= 0;
  a.wt = n->wbf + n->offw[l];
  a.nrows = rows_of(l);
  a.bias = n->params + n->offb[l];
  a.taps = L.taps;
  a.B = B;
  a.H = n->H(lev);
  a.W = n->W(lev);
  if (L.out >= 0) {
    a.relu = 1;
    a.yb = n->act[L.out];
    a.nstore = L.cout;
    a.ystride = L.cout;
  } else {
    a.relu = 0;
    a.yf = n->pred;
    a.nstore = L.cout;
    a.ystride = 4;
  }
  return a;
}

int forward(pdvm_unet *n, const Slots &sl, int B) {
  hipStream_t st = n->stream;
  UCHK(n, launch_build_input(n->ds_solid, n->ds_feat, sl, B, n->n2, n->n1, n->act[X], st));
  auto pool = [&](Act in, Act out, int k) -> int {
    const int lev = kAct[in].level;
    UCHK(n, launch_maxpool(n->act[in], B, n->H(lev), n->W(lev), kAct[in].ch, n->act[out], n->pidx[k], st));
    return PDVM_OK;
  };
  for (int l = 0; l < kLayers; ++l) {
    UCHK(n, mfma_begin(n));
    UCHK(n, launch_conv(conv_args(n, l, B), st));
    UCHK(n, mfma_end(n));
    int rc = PDVM_OK;
    if (kLayer[l].out == E1) rc = pool(E1, P1, 0);
    if (kLayer[l].out == E2) rc = pool(E2, P2, 1);
    if (kLayer[l].out == E3) rc = pool(E3, P3, 2);
    if (rc != PDVM_OK) return rc;
  }
  return PDVM_OK;
}

// Backward pass from the bf16 gradient at the head output (n->gbuf).
int backward(pdvm_unet *n, int B) {
  hipStream_t st = n->stream;
  for (int l = kLayers - 1; l >= 0; --l) {
    const LayerDef &L = kLayer[l];
    const int lev = level_of(l);
    const int rows = rows_of(l);
    const int cin = cin_of(l);
    const int64_t P = n->pix(B, lev);
    // gradient at this layer's pre-activation: for l < head, from its output's gradient
    if (L.out >= 0) UCHK(n, launch_relu_grad(n->gact[L.out], n->act[L.out], P * L.cout, n->gbuf, st));
    // weight gradient
    WgradArgs w{};
    w.g = n->gbuf;
    w.gstride = rows;
    w.M = rows;
    w.xa = n->act[L.in_a];
    w.xb = L.in_b >= 0 ? n->act[L.in_b] : nullptr;
    w.Ca = kAct[L.in_a].ch;
    w.Cb = L.in_b >= 0 ? kAct[L.in_b].ch : 0;
    w.ups = L.in_b >= 0;
    w.taps = L.taps;
    w.B = B;
    w.H = n->H(lev);
    w.W = n->W(lev);
    w.pix_per_split = kPixPerSplit;
    const int splits = (int)((P + kPixPerSplit - 1) / kPixPerSplit);
    const int64_t nw = (int64_t)rows * L.taps * cin;
    if ((int64_t)splits * nw > n->part_n) return n->fail(PDVM_E_INVAL, "internal: partial buffer too small");
    w.part = n->part;
    UCHK(n, mfma_begin(n));
    UCHK(n, launch_wgrad(w, splits, st));
    UCHK(n, mfma_end(n));
    UCHK(n, launch_sum_splits(n->part, splits, nw, n->grads + n->offw[l], st));
    const int csplits = (int)((P + kColsumPix - 1) / kColsumPix);
    if ((int64_t)csplits * rows > n->bpart_n) return n->fail(PDVM_E_INVAL, "internal: bias partial buffer too small");
    UCHK(n, launch_colsum(n->gbuf, P, rows, rows, n->bpart, csplits, st));
    UCHK(n, launch_sum_splits(n->bpart, csplits, rows, n->grads + n->offb[l], st));
    if (l == 0) break;
    // input gradient: a convolution of the output gradient with the flipped, transposed weights
    UCHK(n, launch_wt_back(n->wbf + n->offw[l], rows, cin, L.taps, n->wback, st));
    ConvArgs a{};
    a.xa = n->gbuf;
    a.Ca = rows;
    a.wt = n->wback;
    a.nrows = cin;
    a.taps = L.taps;
    a.B = B;
    a.H = n->H(lev);
    a.W = n->W(lev);
    a.nstore = cin;
    a.ystride = cin;
    const bool cat = L.in_b >= 0;
    a.yf = cat ? n->dcat : n->gact[L.in_a];
    UCHK(n, mfma_begin(n));
    UCHK(n, launch_conv(a, st));
    UCHK(n, mfma_end(n));
    if (cat) {
      UCHK(n, launch_concat_back(n->dcat, B, n->H(lev), n->W(lev), kAct[L.in_a].ch, kAct[L.in_b].ch,
                                 n->gact[L.in_a], n->gact[L.in_b], st));
    }
    // a pooled input routes its gradient to the pooled tensor (added to the skip gradient)
    const int pin = L.in_a;
    if (!cat && (pin == P1 || pin == P2 || pin == P3)) {
      const int k = pin == P1 ? 0 : (pin == P2 ? 1 : 2);
      const Act src = pin == P1 ? E1 : (pin == P2 ? E2 : E3);
      const int slev = kAct[src].level;
      UCHK(n, launch_maxpool_back(n->gact[pin], n->pidx[k], B, n->H(slev), n->W(slev), kAct[src].ch, n->gact[src],
                                  st));
    }
  }
  return PDVM_OK;
}

int refresh_bf16(pdvm_unet *n) {
  UCHK(n, launch_to_bf16(n->params, n->np, n->wbf, n->stream));
  return PDVM_OK;
}

int loss_and_backward(pdvm_unet *n, const Slots &sl, int B, double *loss) {
  const int64_t HW = (int64_t)n->n1 * n->n2;
  const int nblk = (int)((B * HW + 255) / 256);
  UCHK(n, launch_loss(n->pred, n->ds_solid, n->ds_target, n->ds_wsamp, sl, B, n->n2, n->n1, n->gbuf, n->loss_part,
                      nblk, n->stream));
  int rc = backward(n, B);
  if (rc != PDVM_OK) return rc;
  if (loss) {
    UCHK(n, hipMemcpyAsync(n->h_loss, n->loss_part, sizeof(float) * nblk, hipMemcpyDeviceToHost, n->stream));
    UCHK(n, hipStreamSynchronize(n->stream));
    double s = 0;
    for (int i = 0; i < nblk; ++i) s += n->h_loss[i];
    *loss = s;
  }
  return PDVM_OK;
}

int adam_step(pdvm_unet *n, float lr) {
  n->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)n->adam_t));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)n->adam_t));
  UCHK(n, launch_adam(n->params, n->grads, n->adam_m, n->adam_v, n->np, lr, b1, b2, 1e-8f, c1, c2, n->stream));
  return refresh_bf16(n);
}

// logical <-> internal parameter layout (only the head differs: 3 of 32 rows)
void to_internal(const float *src, std::vector<float> &dst, int64_t np) {
  dst.assign(np, 0.f);
  int64_t s = 0;
  for (int l = 0; l < kLayers; ++l) {
    const int64_t rowlen = (int64_t)kLayer[l].taps * cin_of(l);
    int64_t d = 0;
    for (int ll = 0; ll < l; ++ll) d += (int64_t)rows_of(ll) * kLayer[ll].taps * cin_of(ll) + rows_of(ll);
    std::memcpy(&dst[d], src + s, sizeof(float) * kLayer[l].cout * rowlen);
    s += kLayer[l].cout * rowlen;
    d += (int64_t)rows_of(l) * rowlen;
    std::memcpy(&dst[d], src + s, sizeof(float) * kLayer[l].cout);
    s += kLayer[l].cout;
  }
}
void to_logical(const std::vector<float> &src, float *dst) {
  int64_t s = 0, d = 0;
  for (int l = 0; l < kLayers; ++l) {
    const int64_t rowlen = (int64_t)kLayer[l].taps * cin_of(l);
    std::memcpy(dst + d, &src[s], sizeof(float) * kLayer[l].cout * rowlen);
    d += kLayer[l].cout * rowlen;
    s += (int64_t)rows_of(l) * rowlen;
    std::memcpy(dst + d, &src[s], sizeof(float) * kLayer[l].cout);
    d += kLayer[l].cout;
    s += rows_of(l);
  }
}

double layer_flop(const pdvm_unet *n, int l, int B) {
  return 2.0 * (double)n->pix(B, level_of(l)) * kLayer[l].cout * kLayer[l].taps * cin_of(l);
}

}  // namespace

extern "C" {

int64_t pdvm_unet_num_params(void) { return logical_params(); }

int pdvm_unet_create(int32_t n1, int32_t n2, int32_t batch_max, int32_t dataset_max, void *hip_stream,
                     pdvm_unet **out) {
  if (!out) {
    g_unet_thread_error = "out is NULL";
    return PDVM_E_INVAL;
  }
  *out = nullptr;
  if (n1 < 8 || n2 < 8 || n1 % 8 || n2 % 8 || batch_max < 1 || batch_max > kMaxBatch || dataset_max < 0) {
    g_unet_thread_error = "n1, n2 must be positive multiples of 8, batch_max 1..32, dataset_max >= 0";
    return PDVM_E_INVAL;
  }
  if ((int64_t)n1 * n2 * batch_max * 32 >= ((int64_t)1 << 31)) {
    g_unet_thread_error = "batch_max * n1 * n2 * 32 must stay below 2^31";
    return PDVM_E_INVAL;
  }
  pdvm_unet *n = new pdvm_unet;
  n->n1 = n1;
  n->n2 = n2;
  n->bmax = batch_max;
  n->smax = dataset_max;
  // parameter offsets
  int64_t o = 0;
  for (int l = 0; l < kLayers; ++l) {
    n->offw.push_back(o);
    o += (int64_t)rows_of(l) * kLayer[l].taps * cin_of(l);
    n->offb.push_back(o);
    o += rows_of(l);
  }
  n->np = o;
  int64_t wback_max = 0;
  for (int l = 1; l < kLayers; ++l) wback_max = std::max(wback_max, (int64_t)rows_of(l) * kLayer[l].taps * cin_of(l));
  // partial buffers for the weight gradients
  for (int l = 0; l < kLayers; ++l) {
    const int64_t P = n->pix(batch_max, level_of(l));
    const int64_t splits = (P + kPixPerSplit - 1) / kPixPerSplit;
    n->part_n = std::max(n->part_n, splits * rows_of(l) * kLayer[l].taps * cin_of(l));
    n->bpart_n = std::max(n->bpart_n, (P + kColsumPix - 1) / kColsumPix * rows_of(l));
  }
  const int64_t HW = (int64_t)n1 * n2;
  n->loss_blocks = (int)((batch_max * HW + 255) / 256);
  int64_t dcat_n = 0;
  for (int l = 0; l < kLayers; ++l)
    if (kLayer[l].in_b >= 0) dcat_n = std::max(dcat_n, n->pix(batch_max, level_of(l)) * cin_of(l));
  // arena layout
  std::vector<std::pair<void **, size_t>> plan;
  auto add = [&](void **p, size_t bytes) { plan.push_back({p, (bytes + 255) / 256 * 256}); };
  add((void **)&n->params, sizeof(float) * n->np);
  add((void **)&n->grads, sizeof(float) * n->np);
  add((void **)&n->adam_m, sizeof(float) * n->np);
  add((void **)&n->adam_v, sizeof(float) * n->np);
  add((void **)&n->wbf, 2 * n->np);
  add((void **)&n->wback, 2 * wback_max);
  for (int a = 0; a < NACT; ++a) {
    const size_t cnt = (size_t)n->pix(batch_max, kAct[a].level) * kAct[a].ch;
    add((void **)&n->act[a], 2 * cnt);
    if (a != X) add((void **)&n->gact[a], 4 * cnt);
  }
  for (int k = 0; k < 3; ++k) add((void **)&n->pidx[k], (size_t)n->pix(batch_max, k + 1) * kAct[P1 + 3 * k].ch);
  add((void **)&n->pred, sizeof(float) * batch_max * HW * 4);
  add((void **)&n->dcat, sizeof(float) * dcat_n);
  add((void **)&n->part, sizeof(float) * n->part_n);
  add((void **)&n->bpart, sizeof(float) * n->bpart_n);
  add((void **)&n->loss_part, sizeof(float) * n->loss_blocks);
  add((void **)&n->gbuf, 2 * (size_t)batch_max * HW * 32);
  add((void **)&n->ds_solid, (size_t)(dataset_max + 1) * HW);
  add((void **)&n->ds_feat, sizeof(float) * (dataset_max + 1));
  add((void **)&n->ds_target, sizeof(float) * (size_t)(dataset_max + 1) * 3 * HW);
  add((void **)&n->ds_wsamp, sizeof(float) * (dataset_max + 1));
  add((void **)&n->tmp_f64, sizeof(double) * 3 * HW);
  size_t total = 0;
  for (auto &p : plan) total += p.second;
  if (hipMalloc(&n->arena, total) != hipSuccess) {
    g_unet_thread_error = "hipMalloc of the network arena failed";
    delete n;
    return PDVM_E_NOMEM;
  }
  size_t off = 0;
  for (auto &p : plan) {
    *p.first = n->arena + off;
    off += p.second;
  }
  if (hipHostMalloc((void **)&n->h_loss, sizeof(float) * n->loss_blocks) != hipSuccess) {
    g_unet_thread_error = "pinned host allocation failed";
    (void)hipFree(n->arena);
    delete n;
    return PDVM_E_NOMEM;
  }
  if (hip_stream) {
    n->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&n->stream, hipStreamNonBlocking) != hipSuccess) {
      g_unet_thread_error = "stream creation failed";
      (void)hipHostFree(n->h_loss);
      (void)hipFree(n->arena);
      delete n;
      return PDVM_E_HIP;
    }
    n->own_stream = true;
  }
  // everything starts at zero (parameters, Adam state, the training set)
  if (hipMemsetAsync(n->arena, 0, total, n->stream) != hipSuccess || hipStreamSynchronize(n->stream) != hipSuccess) {
    g_unet_thread_error = "clearing the arena failed";
    pdvm_unet_destroy(n);
    return PDVM_E_HIP;
  }
  *out = n;
  return PDVM_OK;
}

int pdvm_unet_set_params(pdvm_unet *n, const float *params, int64_t cnt) {
  if (!n || !params || cnt != logical_params()) return n ? n->fail(PDVM_E_INVAL, "expected %lld parameters", (long long)logical_params()) : PDVM_E_INVAL;
  std::vector<float> in;
  to_internal(params, in, n->np);
  UCHK(n, hipMemcpyAsync(n->params, in.data(), sizeof(float) * n->np, hipMemcpyHostToDevice, n->stream));
  UCHK(n, hipMemsetAsync(n->adam_m, 0, sizeof(float) * n->np, n->stream));
  UCHK(n, hipMemsetAsync(n->adam_v, 0, sizeof(float) * n->np, n->stream));
  n->adam_t = 0;
  int rc = refresh_bf16(n);
  if (rc != PDVM_OK) return rc;
  UCHK(n, hipStreamSynchronize(n->stream));
  return PDVM_OK;
}

static int get_vec(pdvm_unet *n, const float *dev, float *out, int64_t cnt) {
  if (!n || !out || cnt != logical_params()) return n ? n->fail(PDVM_E_INVAL, "expected %lld values", (long long)logical_params()) : PDVM_E_INVAL;
  std::vector<float> in(n->np);
  UCHK(n, hipMemcpyAsync(in.data(), dev, sizeof(float) * n->np, hipMemcpyDeviceToHost, n->stream));
  UCHK(n, hipStreamSynchronize(n->stream));
  to_logical(in, out);
  return PDVM_OK;
}

int pdvm_unet_get_params(pdvm_unet *n, float *params, int64_t cnt) { return get_vec(n, n ? n->params : nullptr, params, cnt); }
int pdvm_unet_get_grads(pdvm_unet *n, float *grads, int64_t cnt) { return get_vec(n, n ? n->grads : nullptr, grads, cnt); }

static int upload_sample(pdvm_unet *n, int slot, const uint8_t *solid, double kn, double jump, const double *rho,
                         const double *u) {
  const int64_t HW = (int64_t)n->n1 * n->n2;
  if (!solid || !(kn > 0) || !std::isfinite(jump) || jump == 0.0) return n->fail(PDVM_E_INVAL, "bad sample arguments");
  std::vector<uint8_t> s01(HW);
  for (int64_t i = 0; i < HW; ++i) s01[i] = solid[i] ? 1 : 0;
  const double kn256 = std::isinf(kn) ? 1e30 : kn * n->n1 / kRefLen;
  const float feat = (float)(std::log(std::min(kn256, 1e30)) / 3.0);
  UCHK(n, hipMemcpyAsync(n->ds_solid + (int64_t)slot * HW, s01.data(), HW, hipMemcpyHostToDevice, n->stream));
  UCHK(n, hipMemcpyAsync(n->ds_feat + slot, &feat, sizeof(float), hipMemcpyHostToDevice, n->stream));
  if (rho && u) {
    UCHK(n, hipMemcpyAsync(n->tmp_f64, rho, sizeof(double) * HW, hipMemcpyHostToDevice, n->stream));
    UCHK(n, hipMemcpyAsync(n->tmp_f64 + HW, u, sizeof(double) * 2 * HW, hipMemcpyHostToDevice, n->stream));
    UCHK(n, launch_targets(n->ds_solid + (int64_t)slot * HW, n->tmp_f64, n->tmp_f64 + HW, n->n2, n->n1, jump, kn256,
                           n->ds_target + (int64_t)slot * 3 * HW, n->ds_wsamp + slot, n->stream));
  }
  UCHK(n, hipStreamSynchronize(n->stream));  // the host buffers above are the caller's
  return PDVM_OK;
}

int pdvm_unet_set_sample(pdvm_unet *n, int32_t slot, const uint8_t *solid, double kn, double jump, const double *rho,
                         const double *u) {
  if (!n) return PDVM_E_INVAL;
  if (slot < 0 || slot >= n->smax) return n->fail(PDVM_E_INVAL, "slot %d outside 0..%d", slot, n->smax - 1);
  if (!rho || !u) return n->fail(PDVM_E_INVAL, "rho and u are required");
  return upload_sample(n, slot, solid, kn, jump, rho, u);
}

int pdvm_unet_train_step(pdvm_unet *n, const int32_t *slots, int32_t batch, float lr, int32_t update, double *loss) {
  if (!n) return PDVM_E_INVAL;
  Slots sl{};
  int rc = check_slots(n, slots, batch, sl, false);
  if (rc != PDVM_OK) return rc;
  rc = forward(n, sl, batch);
  if (rc != PDVM_OK) return rc;
  rc = loss_and_backward(n, sl, batch, loss);
  if (rc != PDVM_OK) return rc;
  if (update) {
    rc = adam_step(n, lr);
    if (rc != PDVM_OK) return rc;
  }
  UCHK(n, hipStreamSynchronize(n->stream));
  return PDVM_OK;
}

int pdvm_unet_forward(pdvm_unet *n, const int32_t *slots, int32_t batch, float *out) {
  if (!n || !out) return n ? n->fail(PDVM_E_INVAL, "out is NULL") : PDVM_E_INVAL;
  Slots sl{};
  int rc = check_slots(n, slots, batch, sl, false);
  if (rc != PDVM_OK) return rc;
  rc = forward(n, sl, batch);
  if (rc != PDVM_OK) return rc;
  const int64_t HW = (int64_t)n->n1 * n->n2;
  UCHK(n, hipMemcpyAsync(out, n->pred, sizeof(float) * batch * HW * 4, hipMemcpyDeviceToHost, n->stream));
  UCHK(n, hipStreamSynchronize(n->stream));
  return PDVM_OK;
}

int pdvm_unet_predict(pdvm_unet *n, const uint8_t *solid, double kn, double jump, double *rho, double *u) {
  if (!n || !rho || !u) return n ? n->fail(PDVM_E_INVAL, "rho and u are required") : PDVM_E_INVAL;
  const int slot = n->smax;
  int rc = upload_sample(n, slot, solid, kn, jump, nullptr, nullptr);
  if (rc != PDVM_OK) return rc;
  Slots sl{};
  sl.s[0] = slot;
  rc = forward(n, sl, 1);
  if (rc != PDVM_OK) return rc;
  const int64_t HW = (int64_t)n->n1 * n->n2;
  const double kn256 = std::isinf(kn) ? 1e30 : kn * n->n1 / kRefLen;
  UCHK(n, launch_fields(n->pred, n->ds_solid + (int64_t)slot * HW, n->n2, n->n1, jump, kn256, n->tmp_f64,
                        n->tmp_f64 + HW, n->stream));
  UCHK(n, hipMemcpyAsync(rho, n->tmp_f64, sizeof(double) * HW, hipMemcpyDeviceToHost, n->stream));
  UCHK(n, hipMemcpyAsync(u, n->tmp_f64 + HW, sizeof(double) * 2 * HW, hipMemcpyDeviceToHost, n->stream));
  UCHK(n, hipStreamSynchronize(n->stream));
  return PDVM_OK;
}

int pdvm_unet_time(pdvm_unet *n, const int32_t *slots, int32_t batch, int32_t reps, pdvm_unet_timing *out) {
  if (!n || !out || reps < 1) return n ? n->fail(PDVM_E_INVAL, "bad arguments") : PDVM_E_INVAL;
  Slots sl{};
  int rc = check_slots(n, slots, batch, sl, false);
  if (rc != PDVM_OK) return rc;
  hipEvent_t e0, e1, e2;
  UCHK(n, hipEventCreate(&e0));
  UCHK(n, hipEventCreate(&e1));
  UCHK(n, hipEventCreate(&e2));
  double fwd = 0, step = 0, mf = 0;
  for (int r = 0; r < reps && rc == PDVM_OK; ++r) {
    n->timing = true;
    n->tev_used = 0;
    UCHK(n, hipEventRecord(e0, n->stream));
    rc = forward(n, sl, batch);
    if (rc == PDVM_OK && hipEventRecord(e1, n->stream) != hipSuccess) rc = PDVM_E_HIP;
    if (rc == PDVM_OK) rc = loss_and_backward(n, sl, batch, nullptr);
    if (rc == PDVM_OK) rc = adam_step(n, 0.0f);  // a zero learning rate leaves the parameters as they are
    if (rc == PDVM_OK && hipEventRecord(e2, n->stream) != hipSuccess) rc = PDVM_E_HIP;
    if (rc == PDVM_OK && hipEventSynchronize(e2) != hipSuccess) rc = PDVM_E_HIP;
    float a = 0, b = 0;
    if (rc == PDVM_OK && (hipEventElapsedTime(&a, e0, e1) != hipSuccess || hipEventElapsedTime(&b, e0, e2) != hipSuccess))
      rc = PDVM_E_HIP;
    fwd += a;
    step += b;
    for (size_t i = 0; rc == PDVM_OK && i < n->tev_used; i += 2) {
      float c = 0;
      if (hipEventElapsedTime(&c, n->tev[i], n->tev[i + 1]) != hipSuccess) rc = PDVM_E_HIP;
      mf += c;
    }
    n->timing = false;
  }
  n->timing = false;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  if (rc != PDVM_OK) return rc == PDVM_E_HIP ? n->fail(PDVM_E_HIP, "event timing failed") : rc;
  double ff = 0, bf = 0;
  for (int l = 0; l < kLayers; ++l) {
    ff += layer_flop(n, l, batch);
    bf += (l > 0 ? 2.0 : 1.0) * layer_flop(n, l, batch);
  }
  out->forward_ms = fwd / reps;
  out->step_ms = step / reps;
  out->forward_flop = ff;
  out->step_flop = ff + bf;
  out->mfma_ms_per_step = mf / reps;
  return PDVM_OK;
}

void pdvm_unet_destroy(pdvm_unet *n) {
  if (!n) return;
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  for (auto e : n->tev) (void)hipEventDestroy(e);
  if (n->h_loss) (void)hipHostFree(n->h_loss);
  if (n->arena) (void)hipFree(n->arena);
  if (n->own_stream && n->stream) (void)hipStreamDestroy(n->stream);
  delete n;
}

const char *pdvm_unet_last_error(const pdvm_unet *n) { return n ? n->err.c_str() : g_unet_thread_error.c_str(); }

}  // extern "C"
