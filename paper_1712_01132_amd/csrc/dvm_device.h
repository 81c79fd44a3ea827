// Device helpers shared by the kernels of the iteration (dvm_sweep_diag.hip,
// dvm_sweep_rows.hip, dvm_iter.hip). Internal; not part of the C ABI.
#pragma once
#include <type_traits>

#include "dvm_internal.h"

namespace pdvm {
namespace {

struct Img {
  int r, mir, jmp;
};

// Image of a node coordinate c outside [0, n) along axis j: periodic with the
// pressure jump along x1 (Eq. periodic_BC), specular across the outer voxel
// face of a lateral axis (Eq. symmetric_BC) or plain periodic if requested.
__device__ __forceinline__ Img image_of(int j, int c, int n, int lat_periodic) {
  Img im{c, 0, 0};
  if (j == 0) {
    if (c < 0) { im.r = c + n; im.jmp = 1; }
    else       { im.r = c - n; im.jmp = -1; }
  } else if (lat_periodic) {
    im.r = c < 0 ? c + n : c - n;
  } else {
    im.r = c < 0 ? -c - 1 : 2 * n - 1 - c;
    im.mir = 1;
  }
  return im;
}

// Pointers read from the problem descriptors carry no address space; casting
// them to the global one lets the compiler emit global (not flat) accesses,
// whose completion counters do not alias the LDS ones.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T *p) {
  return (gptr<T>)p;
}

// Raw buffer stores (the 2D row pipeline): one resource per tile, the
// voxel's byte offset as a scalar and the lane's slot as a vector offset.
// Range checking is off in effect (the record count is the maximum).
constexpr int kBufferFlags = 0x00020000;  // 32-bit data format, as untyped buffer accesses need
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void buffer_store(double v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void buffer_store(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, 0);
}

// The few per-problem values the image and indexing helpers need, held in
// registers by the kernels that use them.
template <typename T>
struct Dom {
  int n[3];
  int64_t Kpad;
  int latp;
  T jump;
};

template <typename T>
__device__ __forceinline__ Dom<T> dom_of(const Geo<T> &g) {
  Dom<T> d;
  d.n[0] = g.n[0];
  d.n[1] = g.n[1];
  d.n[2] = g.n[2];
  d.Kpad = g.Kpad;
  d.latp = g.lateral_periodic;
  d.jump = g.jump;
  return d;
}

template <typename T>
__device__ __forceinline__ int64_t cell_of(const Dom<T> &g, int x, int y, int z) {
  return x + (int64_t)g.n[0] * (y + (int64_t)g.n[1] * z);
}

// h at an upstream fluid node along axis j: the current sweep inside the
// domain, the previous iteration's value at the image outside it (with the
// mirrored velocity across a specular face and the jump across the x1 wrap).
template <typename T, typename PC, typename PP>
__device__ __forceinline__ T upstream_fluid(const Dom<T> &g, PC hc, PP hp, int j, int x, int y, int z, int kofs,
                                            int kmir) {
  int c[3] = {x, y, z};
  // (node offset in 32 bits) x (voxel slots), one 32 x 32 -> 64 bit product
  auto at = [&]() { return (int64_t)((uint64_t)(uint32_t)(c[0] + g.n[0] * (c[1] + g.n[1] * c[2])) * (uint32_t)g.Kpad); };
  if (c[j] >= 0 && c[j] < g.n[j]) return hc[at() + kofs];
  const Img im = image_of(j, c[j], g.n[j], g.latp);
  c[j] = im.r;
  const T v = hp[at() + (im.mir ? kmir : kofs)];
  return im.jmp ? v + T(im.jmp) * g.jump : v;
}

// Address of h at an upstream node (x, y) along lateral axis 1 in 2D, as in
// upstream_fluid: the current sweep inside the domain, the previous
// iteration's image (mirrored velocity, no jump) outside it.
template <typename T>
__device__ __forceinline__ gptr<const T> upstream_addr(const Dom<T> &g, gptr<const T> hc, gptr<const T> hp, int j,
                                                       int x, int y, int kofs, int kmir) {
  int c[2] = {x, y};
  const bool in = c[j] >= 0 && c[j] < g.n[j];
  const Img im = image_of(j, c[j], g.n[j], g.latp);
  if (!in) c[j] = im.r;
  const int k = (!in && im.mir) ? kmir : kofs;
  // the node's offset in 32 bits (under 2^31 / 6 voxels) times the voxel's
  // bytes in one 32 x 32 -> 64 bit product: fewer scalar instructions than
  // 64-bit index arithmetic
  const uint32_t cell = (uint32_t)(c[0] + g.n[0] * c[1]);
  return (gptr<const T>)((gptr<const char>)(in ? hc : hp) + (uint64_t)cell * (uint32_t)(g.Kpad * sizeof(T))) + k;
}

// Wall value of a solid met at the second upstream node along axis j: the wall
// density seen from the first upstream (fluid) node y1 = x - s e_j, i.e. its
// incoming half-flux over D_j, carried through y1's image if y1 is outside.
template <typename T, typename PW>
__device__ __forceinline__ T wall_at_y1(const Dom<T> &g, PW wall, int j, int s, int pin, int x, int y, int z) {
  int c[3] = {x, y, z};
  c[j] -= s;
  if (c[j] >= 0 && c[j] < g.n[j]) return wall[cell_of(g, c[0], c[1], c[2]) * 6 + 2 * j + pin];
  const Img im = image_of(j, c[j], g.n[j], g.latp);
  c[j] = im.r;
  const int p = im.mir ? 1 - pin : pin;
  const T v = wall[cell_of(g, c[0], c[1], c[2]) * 6 + 2 * j + p];
  return im.jmp ? v + T(im.jmp) * g.jump : v;
}

// Offset form: the density ramp rho_r at voxel c, and rho_r(y1) - rho_r(x) for
// the upstream node y1 of the wall value (axis j, half p) that x stores: half 1
// serves the sweep along +e_j (y1 = x - e_j), half 0 the sweep along -e_j.
template <typename T>
__device__ __forceinline__ double ramp_at(const Geo<T> &g, int64_t c) {
  const int x = (int)(c % g.n[0]);
  return g.ramp * (0.5 - (x + 0.5) / (double)g.n[0]);
}
template <typename T>
__device__ __forceinline__ double ramp_step(const Geo<T> &g, int j, int p) {
  return j == 0 ? (p ? g.ramp : -g.ramp) / (double)g.n[0] : 0.0;
}

constexpr uint32_t R_SKIP = 0x80000000u;  // solid voxel or outside the tile
// row pipeline codes: the reciprocal denominators' LDS byte offset below
// kRdMask, Maxwell-wall bits (axis k: kWallBit << k) above it
constexpr uint32_t kRdMask = 0xFFFFu, kWallBit = 0x10000u;

// Index of the problem owning block b: off[p] <= b < off[p + 1].
__device__ __forceinline__ int owner_of(const int *off, int nprob, int b) {
  int lo = 0, hi = nprob;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

}  // namespace
}  // namespace pdvm
