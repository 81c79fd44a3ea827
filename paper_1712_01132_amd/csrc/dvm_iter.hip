// Steps (ii)-(v) of the iteration (Sec. 3.1, Algorithm 1) on gfx950:
//   moments_kernel    quadrature moments rho, u and the half-fluxes Phi_j^+- of every
//                     fluid voxel (Eq. perturbed_quantities), the wall densities Phi/D
//                     (Eq. wall_density), the rebuilt source coefficients, and
//                     per-block FP64 residual / flux partials;
//   reduce_kernel     FP64 residual, G_p, k (Eq. k_Gp), Err(l) (Eq. convergence_criterion),
//                     stop decision, state flip;
// and the state set-up, diagnostics and checkpoint copies.
#include "dvm_device.h"

namespace pdvm {
namespace {

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

// wave_sum8 within each half of the wavefront (lanes 0-31 and 32-63 sum
// separately): lane l holds the total of its half's value
// ((l >> 4) & 1) * 4 + ((l >> 3) & 1) * 2 + ((l >> 2) & 1).
__device__ __forceinline__ double half_sum8(const double (&v)[8], int lane) {
  double a[4], b[2];
  const bool u16 = lane & 16, u8 = lane & 8, u4 = lane & 4;
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k] = (u16 ? v[4 + k] : v[k]) + __shfl_xor(u16 ? v[k] : v[4 + k], 16, kWave);
#pragma unroll
  for (int k = 0; k < 2; ++k) b[k] = (u8 ? a[2 + k] : a[k]) + __shfl_xor(u8 ? a[k] : a[2 + k], 8, kWave);
  double c = (u4 ? b[1] : b[0]) + __shfl_xor(u4 ? b[0] : b[1], 4, kWave);
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
// HALF: two voxels at a time, one per half of the wavefront (lane l owns
// the slots q = (l & 31) + 32 m of its half's voxel), for octant sizes just
// above a multiple of 64 (144 velocities per octant: 160 slots per voxel
// instead of 192, and half the reductions and result stores per voxel).
template <typename T, int DIM, int NS, bool PAIR, bool SH, bool HALF = false>
__global__ void __launch_bounds__(kMomBlock)
    moments_kernel(const Geo<T> *__restrict__ G, const int *__restrict__ blk_off, int nprob, double *part_scr) {
  static_assert(!(HALF && PAIR), "one slot layout at a time");
  constexpr int LW = HALF ? kWave / 2 : kWave;  // lanes per voxel
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
  const gptr<double> part = as_global(part_scr ? part_scr + 4 * (int64_t)(nprob > 1 ? blk_off[pb] : 0) : g.part);
  const int64_t N = g.N, Kpad = g.Kpad, nf = g.nfluid;
  const int Ko = g.Ko, Ko_pad = g.Ko_pad, tau_fb = g.tau_fb, mom_blocks = g.mom_blocks;
  const double nu = g.nu, Dj[3] = {g.D[0], g.D[1], g.D[2]};
  const int dev = g.dev;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  constexpr int WPB = kMomBlock / kWave;
  const int64_t nw = (int64_t)mom_blocks * WPB;
  constexpr int NR = 2 + DIM + (SH ? DIM : 0);
  double wr[NS][NR];
  int qc[NS];
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    const int q = PAIR ? 2 * kWave * (m / 2) + 2 * lane + (m & 1) : (lane & (LW - 1)) + m * LW;
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
    // HALF: step t takes voxels 2 t (lanes 0-31) and 2 t + 1 (lanes 32-63;
    // none past an odd count: that half re-reads the last one and stores nothing)
    const int hsel = HALF ? lane >> 5 : 0;
    auto voxel = [&](int t) __attribute__((always_inline)) {
      if (!HALF) return (int64_t)__builtin_amdgcn_readlane(cl, t);
      const int32_t a = __builtin_amdgcn_readlane(cl, 2 * t), b = __builtin_amdgcn_readlane(cl, min(2 * t + 1, cnt - 1));
      return (int64_t)(hsel ? b : a);
    };
    const int steps = HALF ? (cnt + 1) / 2 : cnt;
    T hv[1 << DIM][NS];
    int64_t c = voxel(0);
    load(c, hv);
    for (int t = 0; t < steps; ++t) {
      const int64_t cn = voxel(min(t + 1, steps - 1));
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
      const double tot = HALF ? half_sum8(v, lane) : wave_sum8(v, lane);
      double qt = 0;
      if (SH && DIM == 3) {
        const double w2[8] = {qa[0], qa[1], qa[2], 0, 0, 0, 0, 0};
        qt = HALF ? half_sum8(w2, lane) : wave_sum8(w2, lane);
      }
      // the lane of the total of value k: 8 k (wave_sum8), or in each half
      // 16 ((k >> 2) & 1) + 8 ((k >> 1) & 1) + 4 (k & 1) (half_sum8); with
      // HALF each lane selects its own half's totals
      auto total = [&](double x, int k) __attribute__((always_inline)) {
        if (!HALF) return readlane_d(x, 8 * k);
        const int l = 16 * ((k >> 2) & 1) + 8 * ((k >> 1) & 1) + 4 * (k & 1);
        const double a = readlane_d(x, l), b = readlane_d(x, 32 + l);
        return hsel ? b : a;
      };
      const double r = total(tot, 0);
      // every lane reads the totals here, outside the lane-0 branch below: a
      // read of another lane inside it could see a value whose last step the
      // compiler moved into the branch, where only lane 0 computes it
      double ph[3][2], qf[3] = {0, 0, 0};
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        ph[j][0] = total(tot, 1 + 2 * j);
        ph[j][1] = total(tot, 2 + 2 * j);
        if (SH) qf[j] = DIM == 2 ? total(tot, 5 + j) : total(qt, j);
      }
      const double en = total(tot, 7);
      if ((lane & (LW - 1)) == 0 && (!HALF || 2 * t + hsel < cnt)) {
        // Offset form: the sums above are moments of h - rho_r. rho_r adds
        // rho_r w0 to rho, rho_r D_j to each half-flux (so nothing to u) and
        // rho_r we to the energy. The records then describe the sweep of
        // h - rho_r: the upwind stencils reproduce a linear field exactly, so
        // moving rho_r to the right-hand side leaves -nu rho_r in the rho
        // term, adds J to the coefficient of v1 (a_1 times the ramp's
        // step), and turns each wall value w into w - rho_r(y1).
        const double rr = dev ? ramp_at(g, c) : 0.0;
        const double rt = r + rr * g.w0;
        rho_n[c] = rt;
        const gptr<T> sp = src_n + c * kSrcStride;
        sp[0] = T(nu * (rt - rr));
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
          const double uj = ph[j][0] - ph[j][1];
          mdu = fmax(mdu, fabs(uj - uold[j * N + c]));
          mu = fmax(mu, fabs(uj));
          u_n[j * N + c] = uj;
          sp[1 + j] = T(2.0 * nu * uj + (dev && j == 0 ? g.ramp : 0.0));
          wall_n[c * 6 + 2 * j] = T(ph[j][0] / Dj[j] - (dev ? ramp_step(g, j, 0) : 0.0));
          wall_n[c * 6 + 2 * j + 1] = T(ph[j][1] / Dj[j] - (dev ? ramp_step(g, j, 1) : 0.0));
        }
        if (tau_fb) srct_n[c] = T(nu * ((2.0 / 3.0) * (en + rr * g.we) - rt));
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
  if (HALF) {  // lane 32's voxels into lane 0's accumulators
    mdu = fmax(mdu, __shfl_xor(mdu, 32, kWave));
    mu = fmax(mu, __shfl_xor(mu, 32, kWave));
    su += __shfl_xor(su, 32, kWave);
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
__global__ void __launch_bounds__(256)
    reduce_kernel(Geo<T> *__restrict__ G, const int *__restrict__ blk_off, const int *__restrict__ row_off,
                  double *part_scr, uint8_t *xcc_scr, const int32_t *qctr, int q_total) {
  Geo<T> &g = G[blockIdx.x];
  Ctl *ctl = g.ctl;
  if (ctl->stop) return;
  const double *part = part_scr ? part_scr + 4 * (int64_t)blk_off[blockIdx.x] : g.part;
  const uint8_t *xcc_seen = g.xcc_seen && xcc_scr ? xcc_scr + row_off[blockIdx.x] : g.xcc_seen;  // row_off: the pipeline's block offsets
  const int nblocks = g.mom_blocks;
  const int64_t N = g.N;
  __shared__ double sa[256], sb[256], sc[256];
  __shared__ int misplaced;
  const int t = threadIdx.x;
  if (t == 0) {
    misplaced = 0;
    // queue sweep: every item must have been handled (a queue whose XCD got
    // no block would leave its chains unswept)
    if (qctr) {
      int h = 0;
      for (int x = 0; x < 8; ++x) h += qctr[(8 * kQueueSub + x) * kCtrPad];
      if (h != q_total) misplaced = 1;
    }
  }
  __syncthreads();
  // XCD-local row pipeline: all blocks of a velocity chain must have run on one
  // XCD (their hand-over relies on a shared L2); otherwise the iterate is void
  if (xcc_seen) {
    for (int i = t; i < g.row_blocks; i += 256) {
      const int ch = i % g.row_stride;
      if (ch < g.row_sets && xcc_seen[i] != xcc_seen[ch]) misplaced = 1;
    }
  }
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
  if (misplaced && ctl->fault == 0) ctl->fault = 2;
  if (ctl->fault) {
    ctl->status = -3;  // keep `par`: the iterate of an abandoned sweep is discarded
    ctl->stop = 1;
    g.run = 0;
    return;
  }
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
  if (ctl->fault) {  // poisoned by an abandoned sweep: stays stopped until the host restores a state
    ctl->status = -3;
    ctl->stop = 1;
  }
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
    const bool dev = g.dev && fl;  // offset form (moments_kernel); solid voxels keep zeros
    const double rr = dev ? ramp_at(g, c) : 0.0;
    g.rho[par][c] = r;
    T *sp = g.src[par] + c * kSrcStride;
    for (int i = 0; i < kSrcStride; ++i) sp[i] = T(0);
    sp[0] = T(g.nu * (r - rr));
    g.srct[par][c] = T(0);
    if (g.shakhov)
      for (int j = 0; j < 4; ++j) g.srcq[par][c * 4 + j] = T(0);
    for (int j = 0; j < 3; ++j) {
      const double uj = (fl && u && j < DIM) ? u[j * g.N + c] : 0.0;
      if (j < DIM) {
        g.u[par][j * g.N + c] = uj;
        sp[1 + j] = T(2.0 * g.nu * uj + (dev && j == 0 ? g.ramp : 0.0));
        // Phi_j^+- = rho D_j +- u_j / 2 for h = rho + 2 u.v (offset form: less rho_r(y1))
        g.wall[par][c * 6 + 2 * j] = T((r - rr) + 0.5 * uj / g.D[j] - (dev ? ramp_step(g, j, 0) : 0.0));
        g.wall[par][c * 6 + 2 * j + 1] = T((r - rr) - 0.5 * uj / g.D[j] - (dev ? ramp_step(g, j, 1) : 0.0));
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
      v = (rho ? rho[c] : 0.0) - (g.dev ? ramp_at(g, c) : 0.0);  // offset form: h - rho_r
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
    if (g.dev) {  // offset form: the moments of rho_r
      const double rr = ramp_at(g, c);
      r += rr * g.w0;
      e += rr * g.we;
    }
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

template <typename T, int D, int S, bool P, bool H = false>
void launch_moments_as(const Batch<T> &B, int blocks, hipStream_t st, double *part) {
  if (B.shakhov)
    hipLaunchKernelGGL((moments_kernel<T, D, S, P, true, H>), dim3(blocks), dim3(kMomBlock), 0, st, B.d_geo,
                       B.d_blk_off, B.nprob, part);
  else
    hipLaunchKernelGGL((moments_kernel<T, D, S, P, false, H>), dim3(blocks), dim3(kMomBlock), 0, st, B.d_geo,
                       B.d_blk_off, B.nprob, part);
}

template <typename T>
hipError_t launch_moments(const Batch<T> &B, hipStream_t st, const Scratch &scr) {
  const int blocks = B.h_blk_off[B.nprob];
#define PDVM_MOM(D, S, P) launch_moments_as<T, D, S, P>(B, blocks, st, scr.part)
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
  // two voxels per wavefront where an octant fills a half-wavefront's slots
  // better (the octant size is 1 to 32 past a multiple of 64: 144 velocities
  // take 160 slots instead of 192)
  const int nh = (B.Ko + kWave / 2 - 1) / (kWave / 2);
  if ((B.Ko - 1) % kWave < kWave / 2 && nh <= 9) {
#define PDVM_MOMH(D, S) launch_moments_as<T, D, S, false, true>(B, blocks, st, scr.part)
    if (B.dim == 2) {
      if (nh <= 1) PDVM_MOMH(2, 1);
      else if (nh <= 3) PDVM_MOMH(2, 3);
      else if (nh <= 5) PDVM_MOMH(2, 5);
      else PDVM_MOMH(2, 9);
    } else {
      if (nh <= 1) PDVM_MOMH(3, 1);
      else if (nh <= 3) PDVM_MOMH(3, 3);
      else if (nh <= 5) PDVM_MOMH(3, 5);
      else PDVM_MOMH(3, 9);
    }
#undef PDVM_MOMH
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
hipError_t launch_reduce(const Batch<T> &B, hipStream_t st, const Scratch &scr) {
  const int32_t *qctr = B.use_queue ? (scr.qctr ? scr.qctr : B.d_qctr) : nullptr;
  hipLaunchKernelGGL((reduce_kernel<T>), dim3(B.nprob), dim3(256), 0, st, const_cast<Geo<T> *>(B.d_geo), B.d_blk_off,
                     B.use_strips ? B.d_strip_off : B.d_row_off, scr.part, scr.xcc, qctr, B.q_total);
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

template hipError_t launch_moments<double>(const Batch<double> &, hipStream_t, const Scratch &);
template hipError_t launch_moments<float>(const Batch<float> &, hipStream_t, const Scratch &);
template hipError_t launch_reduce<double>(const Batch<double> &, hipStream_t, const Scratch &);
template hipError_t launch_reduce<float>(const Batch<float> &, hipStream_t, const Scratch &);
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
