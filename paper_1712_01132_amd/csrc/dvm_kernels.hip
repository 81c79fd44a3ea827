// HIP kernels for gfx950 (CDNA4): the iteration of the discrete-velocity
// solver of the steady linearised BGK equation (Sec. 3.1, Algorithm 1).
//
//   sweep_kernel      step (i): upwind forward substitution (Eq. numerical stencil,
//                     Eq. Discretised_linearised_Boltzmann_equations) for one
//                     diagonal of sweep tiles. One wavefront = one tile x 64
//                     discrete velocities of one sign octant: lanes are velocities,
//                     so every per-voxel decision (solid, stencil order, wall,
//                     image) is wavefront-uniform and each voxel's 64 values are
//                     one contiguous store.
//   moments_kernel    steps (ii)-(iii): quadrature moments rho, u and the half-fluxes
//                     Phi_j^+- of every fluid voxel (Eq. perturbed_quantities), the
//                     wall densities Phi/D (Eq. wall_density), the rebuilt source
//                     coefficients, and per-block FP64 residual / flux partials.
//   reduce_kernel     steps (iv)-(v): FP64 residual, G_p, k (Eq. k_Gp), Err(l)
//                     (Eq. convergence_criterion), stop decision, state flip.
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
  if (c[j] >= 0 && c[j] < g.n[j]) return hc[cell_of(g, c[0], c[1], c[2]) * g.Kpad + kofs];
  const Img im = image_of(j, c[j], g.n[j], g.latp);
  c[j] = im.r;
  const T v = hp[cell_of(g, c[0], c[1], c[2]) * g.Kpad + (im.mir ? kmir : kofs)];
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
  return (in ? hc : hp) + cell_of(g, c[0], c[1], 0) * g.Kpad + k;
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

// Step (i) for one diagonal of tiles. One wavefront = one tile x 64 discrete
// velocities of one sign octant (lanes = velocities), so every per-voxel
// decision is wavefront-uniform and each voxel's 64 values are one contiguous
// store. The tile is TT x TT voxels in (x1, x2), any depth along x3, walked
// plane by plane in the octant's order. Per plane, each lane first decodes one
// voxel of the plane into an LDS record (source coefficients and, per axis,
// the stencil weights on the two upstream values and the wall term); the
// wavefront then walks the plane's 2 TT - 1 anti-diagonals, whose voxels are
// independent of each other, so their loads and FMA chains overlap. The two
// previous anti-diagonals stay in registers; values outside the tile come
// from the current sweep of upstream tiles (earlier launches) or from the
// lagged images outside the domain.
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

// EXT bit 0 (PSI, 2D): slots of h and of psi; bit 1 (SH): the Shakhov
// heat-flux source, whose per-voxel values nu (4/5)(1 - Pr) q_j end the record;
// bit 2 (MW): Maxwell walls. A voxel whose axis-j stencil meets a wall (code
// bit 4 + j) adds a_j (1 - alpha) times its own previous-iteration value of
// the velocity mirrored in e_j; the record's wall term is alpha rho_w.
template <typename T, int DIM, int TT, bool Y2WALL, int EXT>
__global__ void __launch_bounds__(kWave)
    sweep_kernel(const Geo<T> *__restrict__ G, const int *__restrict__ item_off, int nprob, int diag) {
  constexpr bool PSI = (EXT & 1) != 0, SH = (EXT & 2) != 0, MW = (EXT & 4) != 0;
  static_assert(!(MW && Y2WALL), "Maxwell walls need stencil rule 1");
  constexpr int NC = TT * TT;
  constexpr int RW = 5 + 3 * DIM + (SH ? DIM : 0);  // record: src (4), nu tau, per axis (c1, c2, w), [q]
  __shared__ T rd_lds[8 * kWave];
  __shared__ T rec[NC * RW];
  __shared__ uint32_t rcode[NC];
  const int p = nprob > 1 ? owner_of(item_off, nprob, blockIdx.x) : 0;
  const Geo<T> &G_ = G[p];
  if (!G_.run) return;  // converged problems retire
  // every per-problem value is read once here; the loops below see registers
  const Dom<T> dm = dom_of(G_);
  const int ngroups = G_.ngroups, Ko = G_.Ko, Ko_pad = G_.Ko_pad, tau_fb = G_.tau_fb;
  const int tile[3] = {G_.tile[0], G_.tile[1], G_.tile[2]};
  const int ntile[3] = {G_.ntile[0], G_.ntile[1], G_.ntile[2]};
  const gptr<const T> absv = as_global(G_.absv), avv = as_global(G_.av), rden = as_global(G_.rden),
                      vsq = as_global(G_.vsqm);
  const gptr<T> hc = as_global(G_.hcur);
  const gptr<const T> hp = as_global(G_.hprev);
  const gptr<const T> src = as_global(G_.srccur);
  const gptr<const T> srct = as_global(G_.srctcur);
  const gptr<const T> srcq = as_global(G_.srcqcur);
  const gptr<const T> wall = as_global(G_.wallcur);
  const gptr<const uint32_t> flags = as_global(G_.flags);
  const int n0 = dm.n[0], n1 = dm.n[1];
  // tiles of diagonal `diag`: in 2D (a, b) with a + b = diag, computed; in 3D from the table
  int d0 = 0, ntd;
  if (DIM == 2) {
    const int amin = max(0, diag - (ntile[1] - 1)), amax = min(diag, ntile[0] - 1);
    d0 = amin;
    ntd = amax - amin + 1;
  } else {
    const gptr<const int32_t> diag_off = as_global(G_.diag_off);
    d0 = diag_off[diag];
    ntd = diag_off[diag + 1] - d0;
  }
  int item = nprob > 1 ? blockIdx.x - item_off[p] : blockIdx.x;
  const int t = item % ntd;
  item /= ntd;
  const int grp = item % ngroups;
  const int o = item / ngroups;
  const int lane = threadIdx.x;
  const int q = grp * kWave + lane;
  const bool active = q < Ko;
  const int qq = active ? q : 0;
  int s[3], sidx[3], pin[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    sidx[j] = (o >> j) & 1;
    s[j] = sidx[j] ? -1 : 1;
    pin[j] = 1 - sidx[j];  // incoming half at a wall emitting along s e_j has sign -s
  }
  // PSI: the lane's slot holds h (ph = 1) or psi (ph = 0), which has no
  // rho, u or wall term and no jump at the x1 wrap
  const T ph = PSI ? as_global(G_.phm)[qq] : T(1);
  Dom<T> dv = dm;  // as dm, with the jump this lane's values take
  if (PSI) dv.jump = dm.jump * ph;
  T vv[3] = {T(0), T(0), T(0)}, aa[3] = {T(0), T(0), T(0)}, cq[3] = {T(0), T(0), T(0)}, am[3] = {T(0), T(0), T(0)};
  const T qs = SH ? as_global(G_.qsf)[qq] : T(0);  // the Shakhov source's q.v factor
  const T spec = G_.spec, alpha = G_.alpha;
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    const T a = absv[j * Ko_pad + qq];
    const T av = a * ph;
    vv[j] = s[j] > 0 ? av : -av;
    aa[j] = avv[j * Ko_pad + qq];
    if (SH) cq[j] = (s[j] > 0 ? a : -a) * qs;
    if (MW) am[j] = aa[j] * spec;
  }
#pragma unroll
  for (int c = 0; c < (1 << DIM); ++c) rd_lds[c * kWave + lane] = rden[c * Ko_pad + qq];
  const T vsqm = tau_fb ? vsq[qq] : T(0);
  const int kofs = o * Ko_pad + qq;
  int kmir[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) kmir[j] = (o ^ (1 << j)) * Ko_pad + qq;

  int lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
  int tpos[3] = {0, 0, 0};
  if (DIM == 2) {
    tpos[0] = d0 + t;
    tpos[1] = diag - tpos[0];
  } else {
    const gptr<const int32_t> diag_tiles = as_global(G_.diag_tiles);
#pragma unroll
    for (int j = 0; j < 3; ++j) tpos[j] = diag_tiles[(d0 + t) * 4 + j];
  }
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    const int tp = tpos[j];
    const int tj = s[j] > 0 ? tp : ntile[j] - 1 - tp;
    lo[j] = tj * tile[j];
    cnt[j] = min(tile[j], dm.n[j] - lo[j]);
  }
  const int xs = s[0] > 0 ? lo[0] : lo[0] + cnt[0] - 1;
  const int ys = s[1] > 0 ? lo[1] : lo[1] + cnt[1] - 1;

  for (int c3 = 0; c3 < cnt[2]; ++c3) {
    const int z = s[2] > 0 ? lo[2] + c3 : lo[2] + cnt[2] - 1 - c3;
    // --- halos of the plane (before any store of this plane), issued first:
    // they depend on nothing below. Away from the domain faces they are plain
    // loads of the current sweep; only tiles touching a face resolve images.
    T L1[TT], L2[TT], B1[TT], B2[TT];
    const int64_t Kp = dm.Kpad;
    const gptr<T> hz = hc + (int64_t)(n1 * z) * n0 * Kp + kofs;  // plane z of the current sweep
    const bool xin = xs - 2 * s[0] >= 0 && xs - 2 * s[0] < n0;
    const bool yin = ys - 2 * s[1] >= 0 && ys - 2 * s[1] < n1;
#pragma unroll
    for (int k = 0; k < TT; ++k) {
      L1[k] = L2[k] = B1[k] = B2[k] = T(0);
      if (k < cnt[1]) {
        const int y = ys + k * s[1];
        if (xin) {
          L1[k] = hz[(int64_t)(y * n0 + xs - s[0]) * Kp];
          L2[k] = hz[(int64_t)(y * n0 + xs - 2 * s[0]) * Kp];
        } else {
          L1[k] = upstream_fluid(dv, hc, hp, 0, xs - s[0], y, z, kofs, kmir[0]);
          L2[k] = upstream_fluid(dv, hc, hp, 0, xs - 2 * s[0], y, z, kofs, kmir[0]);
        }
      }
      if (k < cnt[0]) {
        const int x = xs + k * s[0];
        if (yin) {
          B1[k] = hz[(int64_t)((ys - s[1]) * n0 + x) * Kp];
          B2[k] = hz[(int64_t)((ys - 2 * s[1]) * n0 + x) * Kp];
        } else {
          B1[k] = upstream_fluid(dv, hc, hp, 1, x, ys - s[1], z, kofs, kmir[1]);
          B2[k] = upstream_fluid(dv, hc, hp, 1, x, ys - 2 * s[1], z, kofs, kmir[1]);
        }
      }
    }
    // --- stage: lane = voxel of the plane ---------------------------------
    // The voxel's sources and wall values are loaded together with its flags
    // (valid addresses whatever the flags say), so one round trip serves all.
    if (lane < NC) {
      const int i = lane % TT, r = lane / TT;
      uint32_t code = R_SKIP;
      T *rp = rec + lane * RW;
#pragma unroll
      for (int k = 0; k < RW; ++k) rp[k] = T(0);  // a skipped voxel computes 0
      if (i < cnt[0] && r < cnt[1]) {
        const int x = xs + i * s[0], y = ys + r * s[1];
        const int c = (y + n1 * z) * n0 + x;
        const uint32_t f = flags[c];
        const gptr<const T> sp = src + c * kSrcStride;
        const T sv0 = sp[0], sv1 = sp[1], sv2 = sp[2], sv3 = DIM == 3 ? sp[3] : T(0);
        const T svt = tau_fb ? srct[c] : T(0);
        T wv[DIM];
#pragma unroll
        for (int j = 0; j < DIM; ++j) wv[j] = wall[c * 6 + 2 * j + pin[j]];
        if (!(f & F_SOLID)) {
          rp[0] = sv0;
          rp[1] = sv1;
          rp[2] = sv2;
          rp[3] = sv3;
          rp[4] = svt;
          if (SH) {
#pragma unroll
            for (int j = 0; j < DIM; ++j) rp[5 + 3 * DIM + j] = srcq[c * 4 + j];
          }
          code = 0;
#pragma unroll
          for (int j = 0; j < DIM; ++j) {
            const uint32_t fj = f >> fbit(j, sidx[j]);
            const bool first = fj & 1u, y1s = fj & 2u, y2s = fj & 4u;
            T c1 = first ? (y1s ? T(0) : T(1)) : T(2);
            T c2 = first ? T(0) : T(-0.5);
            T w = (first && y1s) ? (MW ? alpha * wv[j] : wv[j]) : T(0);
            if (Y2WALL && !first && y2s) {
              c2 = T(0);
              w = T(-0.5) * wall_at_y1(dm, wall, j, s[j], pin[j], x, y, z);
            }
            rp[5 + 3 * j] = c1;
            rp[6 + 3 * j] = c2;
            rp[7 + 3 * j] = w;
            code |= (first ? 1u : 0u) << j;
            if (MW && first && y1s) code |= 16u << j;
          }
        }
      }
      rcode[lane] = code;
    }
    const bool zin = DIM == 3 && z - 2 * s[2] >= 0 && z - 2 * s[2] < dm.n[2];
    const int64_t zstep = (int64_t)n1 * n0 * Kp * s[2];
    __syncthreads();
    // store addresses: row r of the tile starts at hrow[r]; voxel i of a row is icol[i] further
    gptr<T> hrow[TT];
    int64_t icol[TT];
#pragma unroll
    for (int k = 0; k < TT; ++k) {
      hrow[k] = hz + (int64_t)((ys + k * s[1]) * n0 + xs) * Kp;
      icol[k] = (int64_t)k * s[0] * Kp;
    }
    // --- the plane's anti-diagonals ---------------------------------------
    T D1[TT], D2[TT];
#pragma unroll
    for (int k = 0; k < TT; ++k) D1[k] = D2[k] = T(0);
#pragma unroll
    for (int d = 0; d < 2 * TT - 1; ++d) {
      T Nw[TT];
      uint32_t Nc[TT];
      T Z1[TT], Z2[TT];
#pragma unroll
      for (int r = 0; r < TT; ++r) {
        Nw[r] = T(0);
        Nc[r] = R_SKIP;
        Z1[r] = Z2[r] = T(0);
        const int i = d - r;
        if (DIM == 3 && i >= 0 && i < TT && i < cnt[0] && r < cnt[1]) {
          const int x = xs + i * s[0], y = ys + r * s[1];
          if (zin) {
            const gptr<const T> hv0 = hz + (int64_t)(y * n0 + x) * Kp;
            Z1[r] = hv0[-zstep];
            Z2[r] = hv0[-2 * zstep];
          } else {
            Z1[r] = upstream_fluid(dv, hc, hp, 2, x, y, z - s[2], kofs, kmir[2]);
            Z2[r] = upstream_fluid(dv, hc, hp, 2, x, y, z - 2 * s[2], kofs, kmir[2]);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < TT; ++r) {
        const int i = d - r;
        if (i < 0 || i >= TT) continue;
        // no branch before the store: the loads of all voxels of the
        // anti-diagonal can be issued together (a skipped voxel's record is 0)
        const uint32_t code = __builtin_amdgcn_readfirstlane(rcode[i + TT * r]);
        const T *rp = rec + (i + TT * r) * RW;
        T num = fma(rp[1], vv[0], PSI ? rp[0] * ph : rp[0]);
        num = fma(rp[2], vv[1], num);
        if (DIM == 3) num = fma(rp[3], vv[2], num);
        num = fma(rp[4], vsqm, num);  // rp[4] = vsqm = 0 without the feedback
        if (SH) {
#pragma unroll
          for (int j = 0; j < DIM; ++j) num = fma(rp[5 + 3 * DIM + j], cq[j], num);
        }
        if (MW) {
          // the voxel's own previous iterate at the mirrored velocity (a uniform branch)
          const gptr<const T> hv_prev = hp + ((hrow[r] + icol[i]) - hc) - kofs;
#pragma unroll
          for (int j = 0; j < DIM; ++j)
            if (code & (16u << j)) num = fma(am[j], hv_prev[kmir[j]], num);
        }
        const T x1a = i >= 1 ? D1[r] : L1[r];
        const T x1b = i >= 2 ? D2[r] : (i == 1 ? L1[r] : L2[r]);
        const T x2a = r >= 1 ? D1[r >= 1 ? r - 1 : 0] : B1[i];
        const T x2b = r >= 2 ? D2[r >= 2 ? r - 2 : 0] : (r == 1 ? B1[i] : B2[i]);
        num = fma(aa[0], fma(rp[5], x1a, fma(rp[6], x1b, PSI ? rp[7] * ph : rp[7])), num);
        num = fma(aa[1], fma(rp[8], x2a, fma(rp[9], x2b, PSI ? rp[10] * ph : rp[10])), num);
        if (DIM == 3) num = fma(aa[2], fma(rp[11], Z1[r], fma(rp[12], Z2[r], rp[13])), num);
        Nw[r] = num * rd_lds[(code & 7u) * kWave + lane];
        Nc[r] = code;
      }
      // the stores after the whole anti-diagonal: the loop above stays free
      // of control flow, so its loads and FMA chains interleave
#pragma unroll
      for (int r = 0; r < TT; ++r) {
        const int i = d - r;
        if (i < 0 || i >= TT) continue;
        if (active && !(Nc[r] & R_SKIP)) __builtin_nontemporal_store(Nw[r], &hrow[r][icol[i]]);
      }
#pragma unroll
      for (int r = 0; r < TT; ++r) {
        D2[r] = D1[r];
        D1[r] = Nw[r];
      }
    }
    __syncthreads();  // the next plane's staging overwrites the records
  }
}

// Step (i) in 2D as one launch: a pipeline of tile rows. Block (problem p,
// band b, chain c) holds NW wavefronts; wavefront w owns tile row j = b NW + w
// (in the octant's sweep order) of velocity chain c = (octant, 64-velocity
// group) and walks its tiles along x1 in sweep order. Within a tile the walk
// is the one of sweep_kernel (same records, same arithmetic, so both
// schedules give bitwise identical iterates). The left halo of a tile is the
// last two columns of the wavefront's previous tile, kept in registers. The
// bottom halo is the top two rows of tile (a, j - 1):
// * inside a band the wavefront below hands them over through an LDS ring of
//   two slots, with per-wavefront tile counters in LDS: `made` by the
//   producer after its slot writes, `used` by the consumer after its reads,
//   so a slot is rewritten only once it has been read. No global store is
//   waited for on this path;
// * across bands they are read from h once the band below has published its
//   progress counter. Stamps (seq * ntile0 + a + 1) never repeat, since seq
//   advances with every arm and every reduction, so counters are never reset.
// Producers have lower block indices than their consumers (block = row_off[p]
// + b * stride + c), so in-order dispatch cannot deadlock. Every wait is
// bounded in wall-clock time (Geo::wait_ticks): one that exceeds it flags
// ctl->fault and lets every wavefront finish.
//
// Two publication protocols between bands. LOCAL (the host has checked that
// every band of a chain runs on the same XCD, so producer and consumer share
// one L2): the producer drains its stores into the L2 (s_waitcnt) and then
// writes the counter with a relaxed agent-scope store; the consumer polls it
// with relaxed agent-scope loads, which no CU's L1 can serve stale, and then
// reads the halo through the shared L2. No L2 write-back or invalidation is
// needed. The halo lines cannot be stale in the consumer's L1: the L1 starts
// the kernel empty and a chain's 64-velocity segments of a band's top rows
// are read only by the band above, after the counter. (A workgroup-scope
// counter polled after an L1 invalidation was never observed on gfx950.)
// Otherwise: agent-scope release and acquire, correct for any placement.
//
// Lanes past the octant size (in the last 64-velocity group of a chain) read
// every per-velocity value and every halo from the octant's last slot, which
// a lane of the same wavefront owns, so they compute bit-exact copies of that
// lane's values and store them to its slot in the same instructions: every
// store is then decided by the voxel alone (uniform), without a per-lane mask.
// With TAU (the temperature fed back, which in 2D needs psi) a lane's slot
// holds h or psi, as in sweep_kernel with PSI.
// EXT as in sweep_kernel: bit 0 the temperature fed back (in 2D with psi),
// bit 1 the Shakhov heat-flux source (two more record values), bit 2 Maxwell
// walls (never with Y2WALL).
template <typename T, int TT, bool Y2WALL, bool LOCAL, int NW, int EXT>
__global__ void __launch_bounds__(kWave * NW)
    sweep_rows_kernel(const Geo<T> *__restrict__ G, const int *__restrict__ row_off, int nprob, int stride) {
  constexpr int DIM = 2;
  constexpr int NC = TT * TT;
  constexpr bool TAU = (EXT & 1) != 0, SH = (EXT & 2) != 0, MW = (EXT & 4) != 0;
  static_assert(!(MW && Y2WALL), "Maxwell walls need stencil rule 1");
  // record: src (3), then per axis (c1, c2, w), then the feedback source;
  // 10 values, so a record is five aligned 16-byte LDS reads (Shakhov: the
  // two heat-flux sources follow)
  constexpr int RW = SH ? 12 : 10;
  constexpr int RING = 2;
  __shared__ T rd_lds[4 * kWave];
  __shared__ T rec_lds[NW][NC * RW];
  __shared__ __attribute__((aligned(16))) uint32_t rcode_lds[NW][NC];
  __shared__ T ring[NW > 1 ? NW - 1 : 1][RING][2 * TT][kWave];
  __shared__ int32_t made[NW], used[NW];
  const int p = nprob > 1 ? owner_of(row_off, nprob, blockIdx.x) : 0;
  const Geo<T> &G_ = G[p];
  if (!G_.run) return;
  const Dom<T> dm = dom_of(G_);
  const int ngroups = G_.ngroups, Ko = G_.Ko, Ko_pad = G_.Ko_pad, tau_fb = G_.tau_fb;
  const int tile0 = G_.tile[0], tile1 = G_.tile[1];
  const int ntile0 = G_.ntile[0], ntile1 = G_.ntile[1];
  const gptr<const T> absv = as_global(G_.absv), avv = as_global(G_.av), rden = as_global(G_.rden),
                      vsq = as_global(G_.vsqm);
  const gptr<T> hc = as_global(G_.hcur);
  const gptr<const T> hcc = hc;
  const gptr<const T> hp = as_global(G_.hprev);
  const gptr<const T> src = as_global(G_.srccur);
  const gptr<const T> srct = as_global(G_.srctcur);
  const gptr<const T> wall = as_global(G_.wallcur);
  const gptr<const uint32_t> flags = as_global(G_.flags);
  const gptr<int32_t> progress = as_global(G_.progress);
  const gptr<int32_t> fault = as_global(&G_.ctl->fault);
  const uint32_t seq = (uint32_t)G_.seq;
  const int n0 = dm.n[0], n1 = dm.n[1];
  const int nchains = ngroups << DIM;
  // block = row_off[p] + band * stride + c; stride and row_off[p] are
  // multiples of 8, so chain c of every band runs on XCD (c mod 8) under
  // round-robin placement
  const int local_b = nprob > 1 ? blockIdx.x - row_off[p] : blockIdx.x;
  const int c = local_b % stride;
  const int band = local_b / stride;
  if (c >= nchains) return;  // padding of the band to a multiple of 8 blocks
  // the wavefront index, held in a scalar register so that everything that
  // depends on the row is wavefront-uniform to the compiler
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  const int j = band * NW + w;  // tile row in sweep order
  const int grp = c % ngroups;
  const int o = c / ngroups;
  const int q = grp * kWave + lane;
  const bool active = q < Ko;
  const int qq = active ? q : Ko - 1;
  int s[3], sidx[3], pin[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    sidx[k] = (o >> k) & 1;
    s[k] = sidx[k] ? -1 : 1;
    pin[k] = 1 - sidx[k];
  }
  const T ph = TAU ? as_global(G_.phm)[qq] : T(1);
  Dom<T> dv = dm;  // as dm, with the jump this lane's values take
  if (TAU) dv.jump = dm.jump * ph;
  T vv[2], aa[2], cq[2] = {T(0), T(0)}, am[2] = {T(0), T(0)};
  const T qs = SH ? as_global(G_.qsf)[qq] : T(0);  // the Shakhov source's q.v factor
  const T spec = G_.spec, alpha = G_.alpha;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const T a = absv[k * Ko_pad + qq];
    const T av = a * ph;
    vv[k] = s[k] > 0 ? av : -av;
    aa[k] = avv[k * Ko_pad + qq];
    if (SH) cq[k] = (s[k] > 0 ? a : -a) * qs;
    if (MW) am[k] = aa[k] * spec;
  }
  if (w == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) rd_lds[k * kWave + lane] = rden[k * Ko_pad + qq];
  }
  if (lane == 0) {
    made[w] = 0;
    used[w] = 0;
  }
  __syncthreads();          // the only block-wide barrier
  if (j >= ntile1) return;  // the last band may be partial
  T *const rec = rec_lds[w];
  uint32_t *const rcode = rcode_lds[w];
  const T vsqm = tau_fb ? vsq[qq] : T(0);
  const int kofs = o * Ko_pad + qq;
  // byte offset of this lane's slot in a voxel's distribution, for stores
  // from a wavefront-uniform voxel address
  const uint32_t kst = (uint32_t)kofs * (uint32_t)sizeof(T);
  int kmir[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) kmir[k] = (o ^ (1 << k)) * Ko_pad + qq;
  const int64_t Kp = dm.Kpad;
  // this row's voxel rows
  const int tj = s[1] > 0 ? j : ntile1 - 1 - j;
  const int lo1 = tj * tile1, cnt1 = min(tile1, n1 - lo1);
  const int ys = s[1] > 0 ? lo1 : lo1 + cnt1 - 1;
  const bool lwait = w > 0;                          // bottom halo from the wavefront below (LDS)
  const bool gwait = w == 0 && band > 0;             // from the band below (h)
  const bool lmake = w < NW - 1 && j + 1 < ntile1;   // top rows to the wavefront above (LDS)
  const bool gmake = w == NW - 1 && j + 1 < ntile1;  // progress to the band above
  const gptr<int32_t> wait_on = progress + (band > 0 ? (band - 1) * nchains + c : 0);
  const gptr<int32_t> publish = progress + band * nchains + c;
  const gptr<T> hz = hc;  // plane 0 of the current sweep
  // store offsets of a whole tile (buffer stores, in bytes): row r and column
  // i in sweep order, from the tile's lowest-addressed voxel
  // (the column offset is folded into the lane's vector offset)
  const int ylo = s[1] > 0 ? ys : ys - (TT - 1);
  uint32_t rowb[TT], vcol[TT];
#pragma unroll
  for (int k = 0; k < TT; ++k) {
    rowb[k] = (uint32_t)((s[1] > 0 ? k : TT - 1 - k) * (int64_t)n0 * Kp * (int64_t)sizeof(T));
    vcol[k] = kst + (uint32_t)((s[0] > 0 ? k : TT - 1 - k) * Kp * (int64_t)sizeof(T));
  }
  // this lane's reciprocal denominators, offset by the voxel code's byte offset
  const T *const rd_lane = rd_lds + lane;
  const int64_t wait_ticks = G_.wait_ticks;
  // Bounded wait: polls `ready` until it holds; after wait_ticks of the
  // wall clock (checked every 64 polls) it flags ctl->fault and gives up.
  auto bounded_wait = [&](auto ready, int sleep2) __attribute__((always_inline)) {
    int n = 0;
    int64_t t0 = 0;
    while (!ready()) {
      if ((++n & 63) == 0) {
        const int64_t t = wall_clock64();
        if (n == 64) {
          t0 = t;
        } else if (t - t0 > wait_ticks) {
          __hip_atomic_store(fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
      if (sleep2) __builtin_amdgcn_s_sleep(2);
      else __builtin_amdgcn_s_sleep(1);
    }
  };
  auto lds_wait = [&](int32_t *ctr, int32_t want) __attribute__((always_inline)) {
    bounded_wait([&] { return __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= want; }, 0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no LDS access below is moved above the poll
  };
  auto lds_post = [&](int32_t *ctr, int32_t v) __attribute__((always_inline)) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this wavefront's LDS accesses are done
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __hip_atomic_store(ctr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };

  T L1[TT], L2[TT];  // left halo: previous tile's last two columns, or images
#pragma unroll
  for (int k = 0; k < TT; ++k) L1[k] = L2[k] = T(0);

  // raw data of voxel `lane` of tile a of this row, loaded one tile ahead.
  // The loads are unconditional (lanes outside the tile read voxel 0 and
  // discard it), so the code is straight-line and the compiler can count the
  // loads in flight exactly: vector-memory loads complete in issue order, and
  // a wait for the halo must not also wait for this prefetch.
  struct Raw {
    uint32_t f;
    T sv0, sv1, sv2, svt, wv[2], sq[2];
  };
  auto fetch = [&](int a, Raw &R) {
    const int ta = s[0] > 0 ? a : ntile0 - 1 - a;
    const int lo0 = ta * tile0, cnt0 = min(tile0, n0 - lo0);
    const int xs = s[0] > 0 ? lo0 : lo0 + cnt0 - 1;
    const int i = lane % TT, r = lane / TT;
    const bool in = lane < NC && i < cnt0 && r < cnt1;
    const int cc = in ? (ys + r * s[1]) * n0 + xs + i * s[0] : 0;
    const uint32_t f = flags[cc];
    const gptr<const T> sp = src + cc * kSrcStride;
    R.sv0 = sp[0];
    R.sv1 = sp[1];
    R.sv2 = sp[2];
    const T st = srct[cc];
    R.svt = tau_fb ? st : T(0);
#pragma unroll
    for (int k = 0; k < DIM; ++k) R.wv[k] = wall[cc * 6 + 2 * k + pin[k]];
    if (SH) {
      const gptr<const T> qp = as_global(G_.srcqcur) + cc * 4;
      R.sq[0] = qp[0];
      R.sq[1] = qp[1];
    }
    R.f = in ? f : F_SOLID;
  };
  Raw nxt;
  fetch(0, nxt);

  // left halo of the first tile: images across the x1 wrap
  {
    const int lo0 = (s[0] > 0 ? 0 : ntile0 - 1) * tile0, cnt0 = min(tile0, n0 - lo0);
    const int xs = s[0] > 0 ? lo0 : lo0 + cnt0 - 1;
#pragma unroll
    for (int k = 0; k < TT; ++k)
      if (k < cnt1) {
        const int y = ys + k * s[1];
        L1[k] = upstream_fluid(dv, hc, hp, 0, xs - s[0], y, 0, kofs, kmir[0]);
        L2[k] = upstream_fluid(dv, hc, hp, 0, xs - 2 * s[0], y, 0, kofs, kmir[0]);
      }
  }
  // uniform byte address of row r's first voxel in the current tile
  gptr<char> hrow[TT];

  for (int a = 0; a < ntile0; ++a) {
    const int ta = s[0] > 0 ? a : ntile0 - 1 - a;
    const int lo0 = ta * tile0, cnt0 = min(tile0, n0 - lo0);
    const int xs = s[0] > 0 ? lo0 : lo0 + cnt0 - 1;
    const int slot = a % RING;
    // --- records of this tile from the prefetched data ----------------------
    const Raw cur = nxt;
    if (lane < NC) {
      const int i = lane % TT, r = lane / TT;
      uint32_t code = R_SKIP;
      T *rp = rec + lane * RW;
#pragma unroll
      for (int k = 0; k < RW; ++k) rp[k] = T(0);
      if (i < cnt0 && r < cnt1 && !(cur.f & F_SOLID)) {
        const int x = xs + i * s[0], y = ys + r * s[1];
        rp[0] = cur.sv0;
        rp[1] = cur.sv1;
        rp[2] = cur.sv2;
        rp[9] = cur.svt;
        if (SH) {
          rp[10] = cur.sq[0];
          rp[11] = cur.sq[1];
        }
        code = 0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          const uint32_t fj = cur.f >> fbit(k, sidx[k]);
          const bool first = fj & 1u, y1s = fj & 2u, y2s = fj & 4u;
          T c1 = first ? (y1s ? T(0) : T(1)) : T(2);
          T c2 = first ? T(0) : T(-0.5);
          T wl = (first && y1s) ? (MW ? alpha * cur.wv[k] : cur.wv[k]) : T(0);
          if (MW && first && y1s) code |= kWallBit << k;
          if (Y2WALL && !first && y2s) {
            c2 = T(0);
            wl = T(-0.5) * wall_at_y1(dm, wall, k, s[k], pin[k], x, y, 0);
          }
          rp[3 + 3 * k] = c1;
          rp[4 + 3 * k] = c2;
          rp[5 + 3 * k] = wl;
          code |= (first ? 1u : 0u) << k;
        }
      }
      // the byte offset of the voxel's reciprocal denominators in rd_lds
      // (and, with Maxwell walls, the wall bits above it)
      rcode[lane] = (code & (R_SKIP | kWallBit | (kWallBit << 1))) | ((code & 3u) * (uint32_t)(kWave * sizeof(T)));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // 4 x 4 tiles: the voxel codes and this lane's reciprocal denominators of
    // the whole tile are read before the walk, so that no voxel waits on two
    // chained LDS reads (code, then denominator); they depend only on this
    // wavefront's records, so they are read before the wait for the halo and
    // their latency overlaps it
    constexpr bool PRE = TT == 4;
    uint32_t cw[PRE ? NC : 1];
    T rdv[PRE ? NC : 1];
    if (PRE) {
#pragma unroll
      for (int k = 0; k < NC; ++k) cw[k] = __builtin_amdgcn_readfirstlane(rcode[k]);
#pragma unroll
      for (int k = 0; k < NC; ++k) rdv[k] = *(const T *)((const char *)rd_lane + (cw[k] & kRdMask));
    }

    // records of the voxels on the walk's first NPD anti-diagonals (i + r <
    // NPD), indexed by i + 3 r: three diagonals in FP32; two in FP64, where a
    // third costs more registers than its latency saves
    constexpr int NPD = sizeof(T) == 4 ? 3 : 2;
    T rpre[PRE ? 9 : 1][RW];
    if (PRE) {
#pragma unroll
      for (int v = 0; v < 9; ++v)
        if (v % 3 + v / 3 < NPD) {
#pragma unroll
          for (int k = 0; k < RW; ++k) rpre[v][k] = rec[(v % 3 + TT * (v / 3)) * RW + k];
        }
    }
    // --- bottom halo ------------------------------------------------------------
    T B1[TT], B2[TT];
    if (lwait) {
      lds_wait(&made[w - 1], a + 1);
#pragma unroll
      for (int k = 0; k < TT; ++k) {
        B1[k] = ring[w - 1][slot][k][lane];
        B2[k] = ring[w - 1][slot][TT + k][lane];
      }
    } else {
      if (gwait) {
        const int32_t want = (int32_t)(seq * (uint32_t)ntile0 + (uint32_t)(a + 1));
        bounded_wait(
            [&] {
              const int32_t got = __hip_atomic_load(wait_on, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              return (int32_t)(got - want) >= 0;
            },
            1);
        if (!LOCAL) __atomic_thread_fence(__ATOMIC_ACQUIRE);  // agent scope: the producer's stores are visible
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no load below is moved above the poll
#pragma unroll
      for (int k = 0; k < TT; ++k) {
        // straight-line: columns past the tile re-read its last one; only
        // voxels outside the tile, which are never stored, see them
        const int x = xs + min(k, cnt0 - 1) * s[0];
        B1[k] = *upstream_addr(dm, hcc, hp, 1, x, ys - s[1], kofs, kmir[1]);
        B2[k] = *upstream_addr(dm, hcc, hp, 1, x, ys - 2 * s[1], kofs, kmir[1]);
      }
    }
    // the next tile's records, in flight during this tile's walk; issued after
    // the halo loads so that the walk waits only for the halo (the last tile
    // fetches itself again, which keeps the code free of branches)
    fetch(min(a + 1, ntile0 - 1), nxt);
#pragma unroll
    for (int k = 0; k < TT; ++k) hrow[k] = (gptr<char>)(hz + (int64_t)((ys + k * s[1]) * n0 + xs) * Kp);
    const int64_t colb = (int64_t)s[0] * Kp * (int64_t)sizeof(T);  // bytes from one column to the next
    // a whole tile is stored through one buffer resource based at its
    // lowest-addressed voxel, with wavefront-constant row and column offsets
    const __amdgpu_buffer_rsrc_t tile_rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(T *)(hz + (int64_t)(ylo * n0 + (s[0] > 0 ? xs : xs - (TT - 1))) * Kp), (short)0, -1, kBufferFlags);

    // --- the tile's anti-diagonals (as in sweep_kernel) ---------------------
    // FULL: a whole TT x TT tile, so the columns and rows handed on are
    // compile-time ones; otherwise they are selected by the tile's extent.
    struct Out {
      T LN1[TT], LN2[TT], T1[TT], T2[TT];  // last two columns, top two rows
    };
    auto walk = [&](auto full) __attribute__((always_inline)) {
      constexpr bool FULL = decltype(full)::value;
      Out out;
      T D1[TT], D2[TT];
#pragma unroll
      for (int k = 0; k < TT; ++k) D1[k] = D2[k] = out.LN1[k] = out.LN2[k] = out.T1[k] = out.T2[k] = T(0);
#pragma unroll
      for (int d = 0; d < 2 * TT - 1; ++d) {
        T Nw[TT];
        uint32_t Nc[TT];
#pragma unroll
        for (int r = 0; r < TT; ++r) {
          Nw[r] = T(0);
          Nc[r] = R_SKIP;
        }
#pragma unroll
        for (int r = 0; r < TT; ++r) {
          const int i = d - r;
          if (i < 0 || i >= TT) continue;
          const uint32_t code = PRE ? cw[PRE ? i + TT * r : 0] : __builtin_amdgcn_readfirstlane(rcode[i + TT * r]);
          const T *rp = rec + (i + TT * r) * RW;
          // the first NPD anti-diagonals' records come from registers read before the halo wait
          auto rv = [&](int k) __attribute__((always_inline)) { return (PRE && d < NPD) ? rpre[PRE && d < NPD ? i + 3 * r : 0][k] : rp[k]; };
          T num = fma(rv(1), vv[0], TAU ? rv(0) * ph : rv(0));
          num = fma(rv(2), vv[1], num);
          if (TAU) num = fma(rv(9), vsqm, num);
          if (SH) num = fma(rv(11), cq[1], fma(rv(10), cq[0], num));
          if (MW) {
            // the voxel's own previous iterate at the mirrored velocity (a uniform branch)
            const gptr<const T> hv_prev = hp + (int64_t)((ys + r * s[1]) * n0 + xs + i * s[0]) * Kp;
#pragma unroll
            for (int k = 0; k < DIM; ++k)
              if (code & (kWallBit << k)) num = fma(am[k], hv_prev[kmir[k]], num);
          }
          const T x1a = i >= 1 ? D1[r] : L1[r];
          const T x1b = i >= 2 ? D2[r] : (i == 1 ? L1[r] : L2[r]);
          const T x2a = r >= 1 ? D1[r >= 1 ? r - 1 : 0] : B1[i];
          const T x2b = r >= 2 ? D2[r >= 2 ? r - 2 : 0] : (r == 1 ? B1[i] : B2[i]);
          num = fma(aa[0], fma(rv(3), x1a, fma(rv(4), x1b, TAU ? rv(5) * ph : rv(5))), num);
          num = fma(aa[1], fma(rv(6), x2a, fma(rv(7), x2b, TAU ? rv(8) * ph : rv(8))), num);
          Nw[r] = num * (PRE ? rdv[PRE ? i + TT * r : 0] : *(const T *)((const char *)rd_lane + (code & kRdMask)));
          Nc[r] = code;
          if (FULL) {
            if (i == TT - 1) out.LN1[r] = Nw[r];
            if (i == TT - 2) out.LN2[r] = Nw[r];
            if (r == TT - 1) out.T1[i] = Nw[r];
            if (r == TT - 2) out.T2[i] = Nw[r];
          } else {
            if (i == cnt0 - 1) out.LN1[r] = Nw[r];  // the tile's last column in sweep order
            if (i == cnt0 - 2) out.LN2[r] = Nw[r];
            if (r == cnt1 - 1) out.T1[i] = Nw[r];  // its top row
            if (r == cnt1 - 2) out.T2[i] = Nw[r];
          }
        }
#pragma unroll
        for (int r = 0; r < TT; ++r) {
          const int i = d - r;
          if (i < 0 || i >= TT) continue;
          if (Nc[r] & R_SKIP) continue;
          if (FULL) buffer_store(Nw[r], tile_rsrc, vcol[i], rowb[r]);
          else *(gptr<T>)(hrow[r] + i * colb + kst) = Nw[r];
        }
#pragma unroll
        for (int r = 0; r < TT; ++r) {
          D2[r] = D1[r];
          D1[r] = Nw[r];
        }
      }
      return out;
    };
    const Out res = (cnt0 == TT && cnt1 == TT) ? walk(std::true_type{}) : walk(std::false_type{});
    T T2[TT];
#pragma unroll
    for (int k = 0; k < TT; ++k) T2[k] = res.T2[k];
    // --- hand the tile on ---------------------------------------------------------
    if (lmake) {
      if (cnt1 == 1) {  // a one-row tile passes on its own row and the one below it
#pragma unroll
        for (int k = 0; k < TT; ++k) T2[k] = B1[k];
      }
      lds_wait(&used[w + 1], a + 1 - RING);  // the slot's previous tile has been read
#pragma unroll
      for (int k = 0; k < TT; ++k) {
        ring[w][slot][k][lane] = res.T1[k];
        ring[w][slot][TT + k][lane] = T2[k];
      }
      lds_post(&made[w], a + 1);
    }
    if (gmake) {
      const int32_t stamp = (int32_t)(seq * (uint32_t)ntile0 + (uint32_t)(a + 1));
      if (LOCAL) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_s_waitcnt(0);  // every store of the wavefront has reached the L2
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0) __hip_atomic_store(publish, stamp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        if (lane == 0) __hip_atomic_store(publish, stamp, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (lwait) lds_post(&used[w], a + 1);  // the ring slot has been read (the walk used it)
    // the next tile's left halo: this tile's last two columns (a tile one
    // voxel wide passes on its own column and the one before it)
#pragma unroll
    for (int k = 0; k < TT; ++k) {
      L2[k] = cnt0 >= 2 ? res.LN2[k] : L1[k];
      L1[k] = res.LN1[k];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();  // the next tile's records overwrite this tile's
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

// Sum over the 64 lanes of eight values at once: at each of the first three
// exchange steps a lane keeps one half of its values and sends the other
// half, so ten exchanges (not 8 x 6) leave in lane l the total of value
// ((l >> 5) & 1) * 4 + ((l >> 4) & 1) * 2 + ((l >> 3) & 1).
__device__ __forceinline__ double wave_sum8(const double (&v)[8], int lane) {
  double a[4], b[2];
  const bool u32 = lane & 32, u16 = lane & 16, u8 = lane & 8;
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k] = (u32 ? v[4 + k] : v[k]) + __shfl_xor(u32 ? v[k] : v[4 + k], 32, kWave);
#pragma unroll
  for (int k = 0; k < 2; ++k) b[k] = (u16 ? a[2 + k] : a[k]) + __shfl_xor(u16 ? a[k] : a[2 + k], 16, kWave);
  double c = (u8 ? b[1] : b[0]) + __shfl_xor(u8 ? b[0] : b[1], 8, kWave);
  c += __shfl_xor(c, 4, kWave);
  c += __shfl_xor(c, 2, kWave);
  c += __shfl_xor(c, 1, kWave);
  return c;
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, l), hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Steps (ii)-(iii). A wavefront takes fluid voxels i = w, w + nw, ... of the
// fluid list (nw wavefronts in all), one at a time: lane l owns the octant
// slots q = l + 64 m (m < NS) of every octant, keeps their quadrature weights
// in registers and accumulates rho, the half-fluxes and the energy; the eight
// sums are then reduced over the lanes together. The voxel indices of the
// next 64 voxels come in one load (a lane each), and the next voxel's
// distribution is loaded before the current one is reduced, so a wavefront
// always has a voxel's loads in flight. Slots past the octant size read a
// valid neighbour (same cache lines) and weigh 0.
template <typename T>
using vec2_t = T __attribute__((ext_vector_type(2)));

// PAIR (an even octant size Ko): lane l owns the adjacent slots 128 p + 2 l and
// 128 p + 2 l + 1 (m = 2 p, 2 p + 1), so a voxel's distribution is loaded with
// half as many, twice as wide loads. A pair at or past Ko (both slots, as Ko
// and the pair start are even) reads the last valid pair and weighs 0.
// SH: also the heat flux q_j (signed per octant from the weights
// W |v_j| (|v|^2 - 5/2)), stored as the Shakhov source nu (4/5)(1 - Pr) q_j.
template <typename T, int DIM, int NS, bool PAIR, bool SH>
__global__ void __launch_bounds__(kMomBlock)
    moments_kernel(const Geo<T> *__restrict__ G, const int *__restrict__ blk_off, int nprob) {
  const int pb = nprob > 1 ? owner_of(blk_off, nprob, blockIdx.x) : 0;
  const Geo<T> &g = G[pb];
  const int blk = nprob > 1 ? blockIdx.x - blk_off[pb] : blockIdx.x;
  if (!g.run) return;
  const int par = g.cpar, np = par ^ 1;
  const gptr<const T> h = as_global((const T *)(np ? g.h[1] : g.h[0]));
  const gptr<const double> uold = as_global((const double *)(par ? g.u[1] : g.u[0]));
  const gptr<double> rho_n = as_global(np ? g.rho[1] : g.rho[0]);
  const gptr<double> u_n = as_global(np ? g.u[1] : g.u[0]);
  const gptr<T> src_n = as_global(np ? g.src[1] : g.src[0]);
  const gptr<T> srct_n = as_global(np ? g.srct[1] : g.srct[0]);
  const gptr<T> srcq_n = as_global(np ? g.srcq[1] : g.srcq[0]);
  const gptr<T> wall_n = as_global(np ? g.wall[1] : g.wall[0]);
  const gptr<const int32_t> fidx = as_global(g.fluid_idx);
  const gptr<const double> wq = as_global(g.wq);
  const gptr<double> part = as_global(g.part);
  const int64_t N = g.N, Kpad = g.Kpad, nf = g.nfluid;
  const int Ko = g.Ko, Ko_pad = g.Ko_pad, tau_fb = g.tau_fb, mom_blocks = g.mom_blocks;
  const double nu = g.nu, Dj[3] = {g.D[0], g.D[1], g.D[2]};
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  constexpr int WPB = kMomBlock / kWave;
  const int64_t nw = (int64_t)mom_blocks * WPB;
  constexpr int NR = 2 + DIM + (SH ? DIM : 0);
  double wr[NS][NR];
  int qc[NS];
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    const int q = PAIR ? 2 * kWave * (m / 2) + 2 * lane + (m & 1) : lane + m * kWave;
    const bool ok = q < Ko;
    qc[m] = ok ? q : (PAIR ? Ko - 2 + (m & 1) : Ko - 1);
#pragma unroll
    for (int r = 0; r < 2 + DIM; ++r) wr[m][r] = ok ? wq[r * Ko_pad + q] : 0.0;
    if (SH) {
#pragma unroll
      for (int j = 0; j < DIM; ++j) wr[m][2 + DIM + j] = ok ? wq[(5 + j) * Ko_pad + q] : 0.0;
    }
  }
  const double shc = nu * g.sh_coef;
  auto load = [&](int64_t c, T (&hv)[1 << DIM][NS]) __attribute__((always_inline)) {
    const gptr<const T> hc = h + c * Kpad;
#pragma unroll
    for (int o = 0; o < (1 << DIM); ++o) {
      if (PAIR) {
#pragma unroll
        for (int m = 0; m < NS; m += 2) {
          const vec2_t<T> v = __builtin_nontemporal_load((const gptr<const vec2_t<T>>)(hc + o * Ko_pad + qc[m]));
          hv[o][m] = v.x;
          hv[o][m + 1] = v.y;
        }
      } else {
#pragma unroll
        for (int m = 0; m < NS; ++m) hv[o][m] = __builtin_nontemporal_load(&hc[o * Ko_pad + qc[m]]);
      }
    }
  };
  // the next voxel's distribution is held in registers only when it is small
  constexpr bool kAhead = (1 << DIM) * NS * sizeof(T) <= 256;
  double mdu = 0, mu = 0, su = 0;
  const int64_t first = (int64_t)blk * WPB + wid;
  for (int64_t base = first; base < nf; base += nw * kWave) {
    // this wavefront's next (up to) 64 voxels: lane t holds the index of voxel base + t nw
    const int64_t il = base + (int64_t)lane * nw;
    const int32_t cl = fidx[il < nf ? il : base];
    const int cnt = (int)min<int64_t>(kWave, (nf - base + nw - 1) / nw);
    T hv[1 << DIM][NS];
    int64_t c = __builtin_amdgcn_readlane(cl, 0);
    load(c, hv);
    for (int t = 0; t < cnt; ++t) {
      const int64_t cn = __builtin_amdgcn_readlane(cl, min(t + 1, cnt - 1));
      T hn[1 << DIM][NS];
      if (kAhead) load(cn, hn);  // in flight while this voxel is reduced
      double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // rho, half-fluxes (j, +/-), energy
      double qa[3] = {0, 0, 0};                 // SH: heat flux
#pragma unroll
      for (int o = 0; o < (1 << DIM); ++o) {
#pragma unroll
        for (int m = 0; m < NS; ++m) {
          const double x = (double)hv[o][m];
          v[0] = fma(wr[m][0], x, v[0]);
#pragma unroll
          for (int j = 0; j < DIM; ++j) v[1 + 2 * j + ((o >> j) & 1)] = fma(wr[m][1 + j], x, v[1 + 2 * j + ((o >> j) & 1)]);
          v[7] = fma(wr[m][1 + DIM], x, v[7]);
          if (SH) {
#pragma unroll
            for (int j = 0; j < DIM; ++j) qa[j] = fma(((o >> j) & 1) ? -wr[m][2 + DIM + j] : wr[m][2 + DIM + j], x, qa[j]);
          }
        }
      }
      // in 2D the heat flux fits the two unused sums (5, 6); in 3D it takes a second reduction
      if (SH && DIM == 2) {
        v[5] = qa[0];
        v[6] = qa[1];
      }
      const double tot = wave_sum8(v, lane);
      double qt = 0;
      if (SH && DIM == 3) {
        const double w2[8] = {qa[0], qa[1], qa[2], 0, 0, 0, 0, 0};
        qt = wave_sum8(w2, lane);
      }
      const double r = readlane_d(tot, 0);
      // every lane reads the totals here, outside the lane-0 branch below: a
      // read of another lane inside it could see a value whose last step the
      // compiler moved into the branch, where only lane 0 computes it
      double ph[3][2], qf[3] = {0, 0, 0};
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        ph[j][0] = readlane_d(tot, 8 * (1 + 2 * j));
        ph[j][1] = readlane_d(tot, 8 * (2 + 2 * j));
        if (SH) qf[j] = DIM == 2 ? readlane_d(tot, 8 * (5 + j)) : readlane_d(qt, 8 * j);
      }
      const double en = readlane_d(tot, 56);
      if (lane == 0) {
        rho_n[c] = r;
        const gptr<T> sp = src_n + c * kSrcStride;
        sp[0] = T(nu * r);
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
          const double uj = ph[j][0] - ph[j][1];
          mdu = fmax(mdu, fabs(uj - uold[j * N + c]));
          mu = fmax(mu, fabs(uj));
          u_n[j * N + c] = uj;
          sp[1 + j] = T(2.0 * nu * uj);
          wall_n[c * 6 + 2 * j] = T(ph[j][0] / Dj[j]);
          wall_n[c * 6 + 2 * j + 1] = T(ph[j][1] / Dj[j]);
        }
        if (tau_fb) srct_n[c] = T(nu * ((2.0 / 3.0) * en - r));
        if (SH) {
#pragma unroll
          for (int j = 0; j < DIM; ++j) srcq_n[c * 4 + j] = T(shc * qf[j]);
        }
        su += ph[0][0] - ph[0][1];
      }
      if (kAhead) {
#pragma unroll
        for (int o = 0; o < (1 << DIM); ++o)
#pragma unroll
          for (int m = 0; m < NS; ++m) hv[o][m] = hn[o][m];
      } else {
        load(cn, hv);
      }
      c = cn;
    }
  }
  __shared__ double sh[WPB][3];
  if (lane == 0) {
    sh[wid][0] = mdu;
    sh[wid][1] = mu;
    sh[wid][2] = su;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0, cc = 0;
    for (int w = 0; w < WPB; ++w) {
      a = fmax(a, sh[w][0]);
      b = fmax(b, sh[w][1]);
      cc += sh[w][2];
    }
    part[blk * 4 + 0] = a;
    part[blk * 4 + 1] = b;
    part[blk * 4 + 2] = cc;
  }
}

// The next iteration's buffers and run flag, written into the descriptor.
template <typename T>
__device__ void resolve(Geo<T> &g, int par, int run) {
  g.seq += 1;  // a fresh stamp range for the row pipeline's progress counters
  g.run = run;
  g.cpar = par;
  g.hcur = par ? g.h[0] : g.h[1];
  g.hprev = par ? g.h[1] : g.h[0];
  g.srccur = par ? g.src[1] : g.src[0];
  g.srctcur = par ? g.srct[1] : g.srct[0];
  g.srcqcur = par ? g.srcq[1] : g.srcq[0];
  g.wallcur = par ? g.wall[1] : g.wall[0];
}

template <typename T>
__global__ void __launch_bounds__(256) reduce_kernel(Geo<T> *__restrict__ G) {
  Geo<T> &g = G[blockIdx.x];
  Ctl *ctl = g.ctl;
  if (ctl->stop) return;
  const double *part = g.part;
  const int nblocks = g.mom_blocks;
  const int64_t N = g.N;
  __shared__ double sa[256], sb[256], sc[256];
  const int t = threadIdx.x;
  double a = 0, b = 0, c = 0;
  for (int i = t; i < nblocks; i += 256) {
    a = fmax(a, part[i * 4 + 0]);
    b = fmax(b, part[i * 4 + 1]);
    c += part[i * 4 + 2];
  }
  sa[t] = a;
  sb[t] = b;
  sc[t] = c;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) {
      sa[t] = fmax(sa[t], sa[t + w]);
      sb[t] = fmax(sb[t], sb[t + w]);
      sc[t] += sc[t + w];
    }
    __syncthreads();
  }
  if (t != 0) return;
  const double maxdu = sa[0], maxu = sb[0];
  const double r = maxu > 0 ? maxdu / maxu : maxdu;
  const double gp = sc[0] / (double)N;
  const double k = ctl->kn_coef * gp;
  if (!isfinite(r) || !isfinite(k) || !isfinite(maxu)) {
    ctl->status = -4;  // keep `par`: the previous iterate stays the state
    ctl->stop = 1;
    g.run = 0;
    return;
  }
  const int64_t it = ctl->iter + 1;
  ctl->iter = it;
  ctl->par ^= 1;
  ctl->r = r;
  ctl->gp = gp;
  ctl->k = k;
  if (it % 100 == 0) {
    const int64_t m = it / 100;
    ctl->kring[m % kRing] = k;
    if (m >= 2 && k != 0.0) ctl->err = fabs((k - ctl->kring[(m - 1) % kRing]) / k) / 100.0;
  }
  if (ctl->tol > 0) {
    if (ctl->mode == 0 && r <= ctl->tol) { ctl->status = 1; ctl->stop = 1; }
    if (ctl->mode == 1 && it % 100 == 0 && ctl->err >= 0 && ctl->err < ctl->tol) {
      ctl->status = 1;
      ctl->stop = 1;
    }
  }
  if (!ctl->stop && it >= ctl->iter_limit) {
    ctl->status = 2;
    ctl->stop = 1;
  }
  resolve(g, ctl->par, !ctl->stop);
}

template <typename T>
__global__ void arm_kernel(Geo<T> *__restrict__ G, int nprob, double tol, int mode, int64_t max_iters) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  Ctl *ctl = G[p].ctl;
  ctl->tol = tol;
  ctl->mode = mode;
  ctl->iter_limit = ctl->iter + max_iters;
  ctl->status = 0;
  ctl->stop = max_iters > 0 ? 0 : 1;
  ctl->fault = 0;
  resolve(G[p], ctl->par, !ctl->stop);
}

// Local linearised equilibrium of given fields (moments of the current state
// and the previous-iteration distribution that the boundaries read).
template <typename T, int DIM>
__global__ void init_moments_kernel(Geo<T> g, const double *rho, const double *u) {
  const int par = g.ctl->par;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < g.N; c += (int64_t)gridDim.x * blockDim.x) {
    const bool fl = !(g.flags[c] & F_SOLID);
    const double r = (fl && rho) ? rho[c] : 0.0;
    g.rho[par][c] = r;
    T *sp = g.src[par] + c * kSrcStride;
    for (int i = 0; i < kSrcStride; ++i) sp[i] = T(0);
    sp[0] = T(g.nu * r);
    g.srct[par][c] = T(0);
    if (g.shakhov)
      for (int j = 0; j < 4; ++j) g.srcq[par][c * 4 + j] = T(0);
    for (int j = 0; j < 3; ++j) {
      const double uj = (fl && u && j < DIM) ? u[j * g.N + c] : 0.0;
      if (j < DIM) {
        g.u[par][j * g.N + c] = uj;
        sp[1 + j] = T(2.0 * g.nu * uj);
        // Phi_j^+- = rho D_j +- u_j / 2 for h = rho + 2 u.v
        g.wall[par][c * 6 + 2 * j] = T((r * g.D[j] + 0.5 * uj) / g.D[j]);
        g.wall[par][c * 6 + 2 * j + 1] = T((r * g.D[j] - 0.5 * uj) / g.D[j]);
      } else {
        g.wall[par][c * 6 + 2 * j] = T(0);
        g.wall[par][c * 6 + 2 * j + 1] = T(0);
      }
    }
  }
}

template <typename T, int DIM>
__global__ void init_h_kernel(Geo<T> g, const double *rho, const double *u) {
  const int par = g.ctl->par;
  const int64_t total = g.N * g.Kpad;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / g.Kpad;
    const int k = (int)(e - c * g.Kpad);
    const int o = k / g.Ko_pad, q = k - o * g.Ko_pad;
    double v = 0.0;  // psi of the local equilibrium is tau / 2 = 0
    if (q < g.Ko && g.phm[q] != T(0) && !(g.flags[c] & F_SOLID)) {
      v = rho ? rho[c] : 0.0;
      if (u)
        for (int j = 0; j < DIM; ++j) {
          const double vj = ((o >> j) & 1) ? -(double)g.absv[j * g.Ko_pad + q] : (double)g.absv[j * g.Ko_pad + q];
          v += 2.0 * u[j * g.N + c] * vj;
        }
    }
    g.h[par][e] = T(v);
  }
}

// Temperature and heat-flux diagnostics from the stored distribution.
template <typename T, int DIM>
__global__ void __launch_bounds__(kMomBlock) diagnostics_kernel(Geo<T> g, double *tau, double *qf) {
  const int par = g.ctl->par;
  const T *h = g.h[par];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  constexpr int WPB = kMomBlock / kWave;
  for (int64_t c = (int64_t)blockIdx.x * WPB + wid; c < g.N; c += (int64_t)gridDim.x * WPB) {
    if (g.flags[c] & F_SOLID) {
      if (lane == 0) {
        tau[c] = 0;
        for (int j = 0; j < DIM; ++j) qf[j * g.N + c] = 0;
      }
      continue;
    }
    double e = 0, r = 0, qq[3] = {0, 0, 0};
    for (int o = 0; o < (1 << DIM); ++o)
      for (int q = lane; q < g.Ko; q += kWave) {
        const double hv = (double)h[c * g.Kpad + o * g.Ko_pad + q];
        double vsq = DIM == 2 ? 0.5 : 0.0;
        double vj[3];
        for (int j = 0; j < DIM; ++j) {
          const double a = (double)g.absv[j * g.Ko_pad + q];
          vj[j] = ((o >> j) & 1) ? -a : a;
          vsq += a * a;
        }
        if (g.psi && g.phm[q] == T(0)) {
          // psi = int (v3^2 - 1/2) h: the energy takes W psi, q_j takes W v_j psi
          const double w = g.wq[(1 + DIM) * g.Ko_pad + q];
          e += w * hv;
          for (int j = 0; j < DIM; ++j) qq[j] += w * vj[j] * hv;
          continue;
        }
        const double w = g.wq[q];
        r += w * hv;
        e += w * vsq * hv;
        for (int j = 0; j < DIM; ++j) qq[j] += w * vj[j] * (vsq - 2.5) * hv;
      }
    r = wave_sum(r);
    e = wave_sum(e);
    for (int j = 0; j < DIM; ++j) qq[j] = wave_sum(qq[j]);
    if (lane == 0) {
      tau[c] = (2.0 / 3.0) * e - r;
      for (int j = 0; j < DIM; ++j) qf[j * g.N + c] = qq[j];
    }
  }
}

// Copy one boundary layer (all voxels whose coordinate along `axis` is r) of
// the current distribution to / from a packed buffer (checkpointing).
template <typename T>
__global__ void face_copy_kernel(Geo<T> g, int axis, int r, T *buf, int to_buf) {
  const int par = g.ctl->par;
  T *h = g.h[par];
  const int64_t faces = g.N / g.n[axis];
  const int64_t total = faces * g.Kpad;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = e / g.Kpad;
    const int k = (int)(e - f * g.Kpad);
    int x[3];
    if (axis == 0) { x[0] = r; x[1] = (int)(f % g.n[1]); x[2] = (int)(f / g.n[1]); }
    else if (axis == 1) { x[1] = r; x[0] = (int)(f % g.n[0]); x[2] = (int)(f / g.n[0]); }
    else { x[2] = r; x[0] = (int)(f % g.n[0]); x[1] = (int)(f / g.n[0]); }
    const int64_t c = cell_of(dom_of(g), x[0], x[1], x[2]);
    if (to_buf) buf[e] = h[c * g.Kpad + k];
    else h[c * g.Kpad + k] = buf[e];
  }
}

int grid_for(int64_t work, int block) {
  int64_t b = (work + block - 1) / block;
  if (b > 65536) b = 65536;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

template <typename T, bool Y2WALL>
void launch_sweep_rule(const Batch<T> &B, int diag, hipStream_t st) {
  const int items = B.h_item_off[(size_t)diag * (B.nprob + 1) + B.nprob];
  if (items == 0) return;
  const int *off = B.d_item_off + (size_t)diag * (B.nprob + 1);
#define PDVM_SWEEP_E(D, X, E)                                                                           \
  hipLaunchKernelGGL((sweep_kernel<T, D, X, Y2WALL, E>), dim3(items), dim3(kWave), 0, st, B.d_geo, off, \
                     B.nprob, diag)
#define PDVM_SWEEP_T(D, E)              \
  if (B.tile_edge <= 4) PDVM_SWEEP_E(D, 4, E); \
  else PDVM_SWEEP_E(D, 8, E)
  // EXT: bit 0 psi (2D with tau fed back), bit 1 Shakhov, bit 2 Maxwell walls
  // (stencil rule 1 only, so never with Y2WALL)
  if constexpr (!Y2WALL) {
    if (B.maxwell) {
      if (B.dim == 2) {
        if (B.shakhov) { PDVM_SWEEP_T(2, 7); }
        else if (B.psi) { PDVM_SWEEP_T(2, 5); }
        else { PDVM_SWEEP_T(2, 4); }
      } else {
        if (B.shakhov) { PDVM_SWEEP_T(3, 6); }
        else { PDVM_SWEEP_T(3, 4); }
      }
      return;
    }
  }
  if (B.dim == 2) {
    if (B.shakhov) { PDVM_SWEEP_T(2, 3); }
    else if (B.psi) { PDVM_SWEEP_T(2, 1); }
    else { PDVM_SWEEP_T(2, 0); }
  } else {
    if (B.shakhov) { PDVM_SWEEP_T(3, 2); }
    else { PDVM_SWEEP_T(3, 0); }
  }
#undef PDVM_SWEEP_T
#undef PDVM_SWEEP_E
}

template <typename T>
hipError_t launch_sweep(const Batch<T> &B, int diag, hipStream_t st) {
  if (B.y2wall) launch_sweep_rule<T, true>(B, diag, st);
  else launch_sweep_rule<T, false>(B, diag, st);
  return hipGetLastError();
}

template <typename T, bool LOCAL>
void launch_rows_local(const Batch<T> &B, dim3 grid, hipStream_t st) {
#define PDVM_ROWS(TTV, Y2, E)                                                                   \
  hipLaunchKernelGGL((sweep_rows_kernel<T, TTV, Y2, LOCAL, band_waves(TTV), E>), grid,         \
                     dim3(kWave * band_waves(TTV)), 0, st, B.d_geo, B.d_row_off, B.nprob, B.row_stride)
  // EXT: bit 0 tau fed back (psi), bit 1 Shakhov, bit 2 Maxwell walls (rule 1 only)
#define PDVM_ROWS_EXT(TTV, Y2)                                   \
  if (B.shakhov) PDVM_ROWS(TTV, Y2, 3);                          \
  else if (B.tau_fb) PDVM_ROWS(TTV, Y2, 1);                      \
  else PDVM_ROWS(TTV, Y2, 0)
#define PDVM_ROWS_MW(TTV)                                        \
  if (B.shakhov) PDVM_ROWS(TTV, false, 7);                       \
  else if (B.tau_fb) PDVM_ROWS(TTV, false, 5);                   \
  else PDVM_ROWS(TTV, false, 4)
  if (B.tile_edge == 4) {
    if (B.maxwell) { PDVM_ROWS_MW(4); }
    else if (B.y2wall) { PDVM_ROWS_EXT(4, true); }
    else { PDVM_ROWS_EXT(4, false); }
  } else {
    if (B.maxwell) { PDVM_ROWS_MW(8); }
    else if (B.y2wall) { PDVM_ROWS_EXT(8, true); }
    else { PDVM_ROWS_EXT(8, false); }
  }
#undef PDVM_ROWS_MW
#undef PDVM_ROWS_EXT
#undef PDVM_ROWS
}

template <typename T>
hipError_t launch_sweep_rows(const Batch<T> &B, bool local, hipStream_t st) {
  const dim3 grid((unsigned)B.h_row_off[B.nprob]);
  if (local) launch_rows_local<T, true>(B, grid, st);
  else launch_rows_local<T, false>(B, grid, st);
  return hipGetLastError();
}

// The XCD (accelerator complex die) each block of a grid runs on.
__global__ void xcd_probe_kernel(uint32_t *out) {
  uint32_t x;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
  if (threadIdx.x == 0) out[blockIdx.x] = x;
}

hipError_t launch_xcd_probe(uint32_t *out, int blocks, int threads, hipStream_t st) {
  hipLaunchKernelGGL(xcd_probe_kernel, dim3((unsigned)blocks), dim3((unsigned)threads), 0, st, out);
  return hipGetLastError();
}

template <typename T, int D, int S, bool P>
void launch_moments_as(const Batch<T> &B, int blocks, hipStream_t st) {
  if (B.shakhov)
    hipLaunchKernelGGL((moments_kernel<T, D, S, P, true>), dim3(blocks), dim3(kMomBlock), 0, st, B.d_geo, B.d_blk_off,
                       B.nprob);
  else
    hipLaunchKernelGGL((moments_kernel<T, D, S, P, false>), dim3(blocks), dim3(kMomBlock), 0, st, B.d_geo, B.d_blk_off,
                       B.nprob);
}

template <typename T>
hipError_t launch_moments(const Batch<T> &B, hipStream_t st) {
  const int blocks = B.h_blk_off[B.nprob];
#define PDVM_MOM(D, S, P) launch_moments_as<T, D, S, P>(B, blocks, st)
  // paired slots (2 per lane and 128-slot block) in 2D: 9 % faster in FP32 on
  // the 512^2 rock, unchanged in FP64; slower on the 96^3 pack, so not in 3D
  // pairs only where they cover the octant with no more slots than single
  // slots do (Ko = 144: 256 paired slots against 192 single ones)
  const int ns1 = (B.Ko + kWave - 1) / kWave, ns2 = 2 * ((B.Ko + 2 * kWave - 1) / (2 * kWave));
  if (B.dim == 2 && B.Ko % 2 == 0 && B.Ko >= 2 && ns2 <= ns1) {
    const int ns = ns2;
    if (ns <= 2) PDVM_MOM(2, 2, true);
    else if (ns <= 4) PDVM_MOM(2, 4, true);
    else if (ns <= 8) PDVM_MOM(2, 8, true);
    else PDVM_MOM(2, 16, true);
    return hipGetLastError();
  }
  const int ns = (B.Ko + kWave - 1) / kWave;
  if (B.dim == 2) {
    if (ns <= 1) PDVM_MOM(2, 1, false);
    else if (ns <= 2) PDVM_MOM(2, 2, false);
    else if (ns <= 3) PDVM_MOM(2, 3, false);
    else if (ns <= 4) PDVM_MOM(2, 4, false);
    else if (ns <= 8) PDVM_MOM(2, 8, false);
    else PDVM_MOM(2, 16, false);
  } else {
    if (ns <= 1) PDVM_MOM(3, 1, false);
    else if (ns <= 2) PDVM_MOM(3, 2, false);
    else if (ns <= 4) PDVM_MOM(3, 4, false);
    else if (ns <= 8) PDVM_MOM(3, 8, false);
    else PDVM_MOM(3, 16, false);
  }
#undef PDVM_MOM
  return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce(const Batch<T> &B, hipStream_t st) {
  hipLaunchKernelGGL((reduce_kernel<T>), dim3(B.nprob), dim3(256), 0, st, const_cast<Geo<T> *>(B.d_geo));
  return hipGetLastError();
}

template <typename T>
__global__ void ctl_gather_kernel(const Geo<T> *__restrict__ G, int nprob, Ctl *out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nprob) out[p] = *G[p].ctl;
}

template <typename T>
hipError_t launch_ctl_gather(const Batch<T> &B, Ctl *out, hipStream_t st) {
  hipLaunchKernelGGL((ctl_gather_kernel<T>), dim3((B.nprob + 63) / 64), dim3(64), 0, st, B.d_geo, B.nprob, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_arm(const Batch<T> &B, double tol, int mode, int64_t max_iters, hipStream_t st) {
  hipLaunchKernelGGL((arm_kernel<T>), dim3((B.nprob + 63) / 64), dim3(64), 0, st, const_cast<Geo<T> *>(B.d_geo), B.nprob, tol,
                     mode, max_iters);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_init_state(const Geo<T> &g, const double *rho, const double *u, hipStream_t st) {
  const int gm = grid_for(g.N, 256), gh = grid_for(g.N * g.Kpad, 256);
  if (g.dim == 2) {
    hipLaunchKernelGGL((init_moments_kernel<T, 2>), dim3(gm), dim3(256), 0, st, g, rho, u);
    hipLaunchKernelGGL((init_h_kernel<T, 2>), dim3(gh), dim3(256), 0, st, g, rho, u);
  } else {
    hipLaunchKernelGGL((init_moments_kernel<T, 3>), dim3(gm), dim3(256), 0, st, g, rho, u);
    hipLaunchKernelGGL((init_h_kernel<T, 3>), dim3(gh), dim3(256), 0, st, g, rho, u);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_diagnostics(const Geo<T> &g, double *tau, double *q, hipStream_t st) {
  const int grid = grid_for(g.N, kMomBlock / kWave);
  if (g.dim == 2) hipLaunchKernelGGL((diagnostics_kernel<T, 2>), dim3(grid), dim3(kMomBlock), 0, st, g, tau, q);
  else hipLaunchKernelGGL((diagnostics_kernel<T, 3>), dim3(grid), dim3(kMomBlock), 0, st, g, tau, q);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_face_copy(const Geo<T> &g, int axis, int r, T *buf, int to_buf, hipStream_t st) {
  const int grid = grid_for(g.N / g.n[axis] * g.Kpad, 256);
  hipLaunchKernelGGL((face_copy_kernel<T>), dim3(grid), dim3(256), 0, st, g, axis, r, buf, to_buf);
  return hipGetLastError();
}

template hipError_t launch_sweep<double>(const Batch<double> &, int, hipStream_t);
template hipError_t launch_sweep_rows<double>(const Batch<double> &, bool, hipStream_t);
template hipError_t launch_sweep_rows<float>(const Batch<float> &, bool, hipStream_t);
template hipError_t launch_sweep<float>(const Batch<float> &, int, hipStream_t);
template hipError_t launch_moments<double>(const Batch<double> &, hipStream_t);
template hipError_t launch_moments<float>(const Batch<float> &, hipStream_t);
template hipError_t launch_reduce<double>(const Batch<double> &, hipStream_t);
template hipError_t launch_reduce<float>(const Batch<float> &, hipStream_t);
template hipError_t launch_arm<double>(const Batch<double> &, double, int, int64_t, hipStream_t);
template hipError_t launch_ctl_gather<double>(const Batch<double> &, Ctl *, hipStream_t);
template hipError_t launch_ctl_gather<float>(const Batch<float> &, Ctl *, hipStream_t);
template hipError_t launch_arm<float>(const Batch<float> &, double, int, int64_t, hipStream_t);
template hipError_t launch_init_state<double>(const Geo<double> &, const double *, const double *, hipStream_t);
template hipError_t launch_init_state<float>(const Geo<float> &, const double *, const double *, hipStream_t);
template hipError_t launch_diagnostics<double>(const Geo<double> &, double *, double *, hipStream_t);
template hipError_t launch_diagnostics<float>(const Geo<float> &, double *, double *, hipStream_t);
template hipError_t launch_face_copy<double>(const Geo<double> &, int, int, double *, int, hipStream_t);
template hipError_t launch_face_copy<float>(const Geo<float> &, int, int, float *, int, hipStream_t);

}  // namespace pdvm
