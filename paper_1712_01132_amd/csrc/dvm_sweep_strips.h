// Step (i) of the iteration (Sec. 3.1, Algorithm 1) on gfx950 for 2D problems
// as one launch: a pipeline of strips of TH voxel rows, each walked along x1 as
// a skewed wavefront (Eq. numerical stencil, Eq.
// Discretised_linearised_Boltzmann_equations). Included by the two
// translation units that instantiate it per precision.
#pragma once
#include "dvm_device.h"

namespace pdvm {
namespace {

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// Block (problem p, band b, chain set cs) holds NW wavefronts; wavefront w owns
// strip j = b NW + w: the voxel rows [j TH, j TH + TH) in the sweep order of
// octant o, for the G 64-velocity groups of chain set cs = (o, pair) -- lane l
// carries velocity 64 g + l of each group g, so a voxel's record (sources,
// stencil coefficients, wall values), read once from LDS, serves 64 G
// velocities. The wavefront walks its strip along x1 as a skewed front: at
// step t, row r takes column t - r, so the row below (r - 1) has just finished
// that column and every upstream value is in registers -- the two previous
// columns of the row (x1 direction) and the two rows below in the same column
// (x2 direction). Rows 0 and 1 take the rows below the strip from a stream per
// column: the lateral images of the previous iteration (strip 0), the LDS ring
// of the wavefront below (inside a band), or h itself once the band below has
// published how many columns it has stored (across bands). The same
// arithmetic as the other sweep schedules, on the same records, so every
// schedule gives bitwise identical iterates.
//
// Records are staged per chunk of C = 64 / TH columns: each lane decodes one
// voxel of the chunk (flags, sources, wall values) into LDS, double-buffered;
// the raw loads of the next chunk are in flight during a chunk's walk.
// Hand-over inside a band: the producer writes its two top rows of each
// column into an LDS ring of R columns and posts the number of complete
// columns every CH steps; the consumer posts the columns it has read, which
// bounds the producer's lead to R columns. Across bands (the top wavefront of
// a band): after every CH steps its stores are drained into the L2
// (s_waitcnt) and the column count is published with a relaxed agent-scope
// store; the consumer polls it and reads the rows from h through the shared
// L2 -- LOCAL placement (every band of a chain set on one XCD) is checked at
// creation and, per block, recorded for the reduction kernel, as for the row
// pipeline. Every wait is bounded in wall-clock time and a fault, once
// flagged by any wavefront, ends every other wait at its next check.
template <typename T, int TH, int G, int NW, bool Y2WALL>
__global__ void __launch_bounds__(kWave * NW)
    sweep_strips_kernel(const Geo<T> *__restrict__ Gd, const int *__restrict__ strip_off, int nprob, int stride,
                        int32_t *__restrict__ prog_scr, uint8_t *__restrict__ xcc_scr) {
  constexpr int DIM = 2;
  constexpr int C = kWave / TH;  // columns per staging chunk: one voxel per lane
  constexpr int CH = 4;          // columns per hand-over
  constexpr int R = 8;           // hand-over ring, columns (a power of 2)
  constexpr int RW = sizeof(T) == 8 ? 10 : 12;  // record: src (3), per axis (c1, c2, w), padding
  static_assert(TH >= 2 && C % CH == 0 && R >= CH + TH && (R & (R - 1)) == 0, "strip shape");
  __shared__ __attribute__((aligned(16))) T rec_lds[NW][2][kWave * RW];
  __shared__ uint32_t code_lds[NW][2][kWave];
  __shared__ T rd_lds[4][G][kWave];
  // ring[w]: wavefront w's two top rows per column; the top wavefront's is
  // written too (never read), so the walk has no branch around it
  __shared__ T ring[NW][R][2][G][kWave];
  __shared__ int32_t made[NW], used[NW];

  const int p = nprob > 1 ? owner_of(strip_off, nprob, blockIdx.x) : 0;
  const Geo<T> &G_ = Gd[p];
  if (!G_.run) return;
  const int off0 = nprob > 1 ? strip_off[p] : 0;
  const int local_b = blockIdx.x - off0;
  const int ngroups = G_.ngroups, Ko = G_.Ko, Ko_pad = G_.Ko_pad;
  const int npairs = (ngroups + G - 1) / G, nsets = npairs << DIM;
  const int cs = local_b % stride, band = local_b / stride;
  if (cs >= nsets) return;  // padding of a band to a multiple of 8 blocks
  if (threadIdx.x == 0) {
    // the XCD this block runs on, for the reduction kernel's placement check
    uint32_t xcc;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
    as_global(xcc_scr ? xcc_scr + off0 : G_.xcc_seen)[local_b] = (uint8_t)(xcc & 0xFFu);
  }
  const Dom<T> dm = dom_of(G_);
  const int n0 = dm.n[0], n1 = dm.n[1];
  const int64_t Kp = dm.Kpad;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  const int o = cs / npairs, gp = cs % npairs;
  const int j = band * NW + w;  // strip in sweep order
  const int nstrips = (n1 + TH - 1) / TH;
  const int s0 = (o & 1) ? -1 : 1, s1 = (o & 2) ? -1 : 1;
  const int pin0 = (o & 1) ? 0 : 1, pin1 = (o & 2) ? 0 : 1;
  const gptr<const T> absv = as_global(G_.absv), avv = as_global(G_.av), rden = as_global(G_.rden);
  const gptr<T> hc = as_global(G_.hcur);
  const gptr<const T> hcc = hc;
  const gptr<const T> hp = as_global(G_.hprev);
  const gptr<const T> src = as_global(G_.srccur);
  const gptr<const T> wall = as_global(G_.wallcur);
  const gptr<const uint32_t> flags = as_global(G_.flags);
  const gptr<int32_t> progress = as_global(prog_scr ? prog_scr + off0 : G_.progress);
  const gptr<int32_t> fault = as_global(&G_.ctl->fault);
  const uint32_t seq = (uint32_t)G_.seq;
  const int64_t wait_ticks = G_.wait_ticks;

  // per group: this lane's velocity (lanes past the octant size repeat its
  // last slot, which a lane of the same wavefront owns: identical values to
  // the same place, so stores need no lane mask), and whether the group exists
  bool live[G];
  int kofs[G], kmir0[G], kmir1[G];
  T vv0[G], vv1[G], aa0[G], aa1[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int grp = gp * G + g;
    live[g] = grp < ngroups;
    const int q = grp * kWave + lane;
    const int qq = (live[g] && q < Ko) ? q : Ko - 1;
    kofs[g] = o * Ko_pad + qq;
    kmir0[g] = (o ^ 1) * Ko_pad + qq;
    kmir1[g] = (o ^ 2) * Ko_pad + qq;
    const T a0 = absv[qq], a1 = absv[Ko_pad + qq];
    vv0[g] = s0 > 0 ? a0 : -a0;
    vv1[g] = s1 > 0 ? a1 : -a1;
    aa0[g] = avv[qq];
    aa1[g] = avv[Ko_pad + qq];
    if (w == 0) {
#pragma unroll
      for (int c = 0; c < 4; ++c) rd_lds[c][g][lane] = rden[c * Ko_pad + qq];
    }
  }
  if (lane == 0) {
    made[w] = 0;
    used[w] = 0;
  }
  __syncthreads();  // the only block-wide barrier
  if (j >= nstrips) return;  // the last band may be partial

  const int lo1 = j * TH, cnt1 = min(TH, n1 - lo1);
  // memory coordinates of sweep-order column x' and strip row r
  auto xm = [&](int x) { return s0 > 0 ? x : n0 - 1 - x; };
  auto ym = [&](int r) { return s1 > 0 ? lo1 + r : n1 - 1 - (lo1 + r); };
  // stores: one buffer resource per row of the strip (a row of h spans below
  // 1 GiB, checked by the host); a voxel that is not stored (solid, past the
  // domain, a row past the strip, an absent group) gets an offset past the
  // resource's range, which the hardware drops -- no branch in the walk. The
  // two drop offsets (voxel, group) add up without wrapping.
  const uint32_t colb = (uint32_t)(Kp * (int64_t)sizeof(T));  // bytes per voxel
  __amdgpu_buffer_rsrc_t rowrs[TH];
#pragma unroll
  for (int r = 0; r < TH; ++r)
    rowrs[r] = __builtin_amdgcn_make_buffer_rsrc((void *)(T *)(hc + (int64_t)ym(min(r, cnt1 - 1)) * n0 * Kp), (short)0,
                                                 (int)(colb * (uint32_t)n0), kBufferFlags);
  constexpr uint32_t kDrop = 0x40000000u;
  uint32_t kst[G];
#pragma unroll
  for (int g = 0; g < G; ++g) kst[g] = live[g] ? (uint32_t)kofs[g] * (uint32_t)sizeof(T) : kDrop;

  const bool lwait = w > 0;                           // rows below from the LDS ring
  const bool gwait = w == 0 && band > 0;              // from h, after the band below published
  const bool lmake = w < NW - 1 && j + 1 < nstrips;   // top rows to the ring
  const bool gmake = w == NW - 1 && j + 1 < nstrips;  // column count to the band above
  const gptr<int32_t> wait_on = progress + (band > 0 ? (band - 1) * nsets + cs : 0);
  const gptr<int32_t> publish = progress + band * nsets + cs;

  auto bounded_wait = [&](auto ready, int sleep2) __attribute__((always_inline)) {
    int n = 0;
    int64_t t0 = 0;
    while (!ready()) {
      if ((++n & 63) == 0) {
        const int64_t tc = wall_clock64();
        if (__hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
        if (n == 64) {
          t0 = tc;
        } else if (tc - t0 > wait_ticks) {
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
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  };
  auto lds_post = [&](int32_t *ctr, int32_t v) __attribute__((always_inline)) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this wavefront's LDS writes are done
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __hip_atomic_store(ctr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };

  // ---- staging: raw data of one voxel per lane, then its LDS record ---------
  struct Raw {
    uint32_t f;
    T sv0, sv1, sv2, wv0, wv1;
  };
  const int rl = lane % TH, cl = lane / TH;  // this lane's voxel in a chunk: row rl of column cl
  auto fetch = [&](int k, Raw &Rw) __attribute__((always_inline)) {
    const int x = k * C + cl;
    const bool in = rl < cnt1 && x < n0;
    const int cc = in ? ym(rl) * n0 + xm(x) : 0;
    const uint32_t f = flags[cc];
    const gptr<const T> sp = src + (int64_t)cc * kSrcStride;
    Rw.sv0 = sp[0];
    Rw.sv1 = sp[1];
    Rw.sv2 = sp[2];
    Rw.wv0 = wall[(int64_t)cc * 6 + pin0];
    Rw.wv1 = wall[(int64_t)cc * 6 + 2 + pin1];
    Rw.f = in ? f : F_SOLID;
  };
  auto stage = [&](int k, const Raw &Rw) __attribute__((always_inline)) {
    T *rp = &rec_lds[w][k & 1][lane * RW];
    uint32_t code = R_SKIP;
    T v[RW];
#pragma unroll
    for (int e = 0; e < RW; ++e) v[e] = T(0);
    if (!(Rw.f & F_SOLID)) {
      v[0] = Rw.sv0;
      v[1] = Rw.sv1;
      v[2] = Rw.sv2;
      code = 0;
      const int sidx[2] = {(o & 1), (o >> 1) & 1}, sg[2] = {s0, s1}, pn[2] = {pin0, pin1};
      const T wv[2] = {Rw.wv0, Rw.wv1};
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const uint32_t fj = Rw.f >> fbit(a, sidx[a]);
        const bool fo = fj & 1u, y1s = fj & 2u, y2s = fj & 4u;
        T c1 = fo ? (y1s ? T(0) : T(1)) : T(2);
        T c2 = fo ? T(0) : T(-0.5);
        T wl = (fo && y1s) ? wv[a] : T(0);
        if (Y2WALL && !fo && y2s) {
          c2 = T(0);
          const int x = k * C + cl;
          wl = T(-0.5) * wall_at_y1(dm, wall, a, sg[a], pn[a], xm(x), ym(rl), 0);
        }
        v[3 + 3 * a] = c1;
        v[4 + 3 * a] = c2;
        v[5 + 3 * a] = wl;
        code |= (fo ? 1u : 0u) << a;
      }
    }
#pragma unroll
    for (int e = 0; e < RW; ++e) rp[e] = v[e];
    code_lds[w][k & 1][lane] = code;
  };

  // ---- the walk ----------------------------------------------------------------
  // cur/prv: the last two columns of each row, per group; b1p: the row below
  // the strip at the previous step's column (row 1's second value below)
  T cur[G][TH], prv[G][TH], b1p[G];
  // images across the x1 wrap: the values row r starts from
  auto left_image = [&](int g, int r, int m) __attribute__((always_inline)) {
    Dom<T> dv = dm;
    return upstream_fluid(dv, hcc, hp, 0, xm(0) - m * s0, ym(min(r, cnt1 - 1)), 0, kofs[g], kmir0[g]);
  };
#pragma unroll
  for (int g = 0; g < G; ++g) {
    b1p[g] = T(0);
#pragma unroll
    for (int r = 0; r < TH; ++r) cur[g][r] = prv[g][r] = T(0);
    cur[g][0] = left_image(g, 0, 1);
    prv[g][0] = left_image(g, 0, 2);
  }
  // the rows below the strip, per hand-over of CH columns, in two buffers by
  // hand-over parity: B1 (the row just below) and B2 (the one below it)
  T hb1[2][CH][G], hb2[2][CH][G];
  const bool ghalo = !lwait;  // from global memory: h of the band below, or the lateral images
  auto ghalo_load = [&](int t0, T (&b1)[CH][G], T (&b2)[CH][G]) __attribute__((always_inline)) {
    if (gwait) {
      const int32_t want = (int32_t)(seq * (uint32_t)n0 + (uint32_t)min(t0 + CH, n0));
      bounded_wait(
          [&] {
            const int32_t got = __hip_atomic_load(wait_on, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return (int32_t)(got - want) >= 0;
          },
          1);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no load below is moved above the poll
    }
    // columns past the domain re-read its last one (their results are never stored)
    const int yb = s1 > 0 ? lo1 : n1 - 1 - lo1;  // memory row of strip row 0
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int x = xm(min(t0 + u, n0 - 1));
#pragma unroll
      for (int g = 0; g < G; ++g) {
        b1[u][g] = *upstream_addr(dm, hcc, hp, 1, x, yb - s1, kofs[g], kmir1[g]);
        b2[u][g] = *upstream_addr(dm, hcc, hp, 1, x, yb - 2 * s1, kofs[g], kmir1[g]);
      }
    }
  };
  auto lhalo_read = [&](int t0, T (&b1)[CH][G], T (&b2)[CH][G]) __attribute__((always_inline)) {
    lds_wait(&made[w - 1], min(t0 + CH, n0));
#pragma unroll
    for (int u = 0; u < CH; ++u)
#pragma unroll
      for (int g = 0; g < G; ++g) {
        b1[u][g] = ring[w - 1][(t0 + u) & (R - 1)][0][g][lane];
        b2[u][g] = ring[w - 1][(t0 + u) & (R - 1)][1][g][lane];
      }
  };

  const int nsteps = n0 + TH - 1;
  const int nchunks = (nsteps + C - 1) / C;
  Raw raw;
  fetch(0, raw);
  stage(0, raw);
  // global rows below are loaded one hand-over ahead
  if (ghalo) ghalo_load(0, hb1[0], hb2[0]);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  auto chunk = [&](int k, auto is_first) __attribute__((always_inline)) {
    constexpr bool FIRST = decltype(is_first)::value;
    const T *rec_cur = &rec_lds[w][k & 1][0];
    const T *rec_old = &rec_lds[w][(k + 1) & 1][0];
    const uint32_t *code_cur = &code_lds[w][k & 1][0];
    const uint32_t *code_old = &code_lds[w][(k + 1) & 1][0];
    uint32_t cws[CH][TH];
    static_for<0, C>([&](auto ic) __attribute__((always_inline)) {
      constexpr int i = decltype(ic)::value;
      const int t = k * C + i;
      constexpr int u = i % CH, hbp = (i / CH) & 1;  // column in the hand-over, buffer parity
      if constexpr (u == 0) {
        if (ghalo) ghalo_load(t + CH, hb1[hbp ^ 1], hb2[hbp ^ 1]);
        else lhalo_read(t, hb1[hbp], hb2[hbp]);
        if (lmake) lds_wait(&used[w + 1], t + CH - TH + 2 - R);  // ring slots free
        // the next chunk's raw data, in flight during the chunk's last hand-over
        if constexpr (i == C - CH) fetch(min(k + 1, nchunks), raw);
      }
      // this hand-over's voxel codes, read at its start (row r of step i + v
      // holds column t + v - r: this chunk's buffer, or the previous chunk's
      // for the rows still behind the chunk boundary)
      if constexpr (u == 0) {
        static_for<0, CH>([&](auto vc) __attribute__((always_inline)) {
          constexpr int v = decltype(vc)::value;
#pragma unroll
          for (int r = 0; r < TH; ++r) {
            const bool here = i + v >= r;
            const int slot = here ? (i + v - r) * TH + r : (C + i + v - r) * TH + r;
            cws[v][r] = __builtin_amdgcn_readfirstlane((here ? code_cur : code_old)[slot]);
          }
        });
      }
      T nw[G][TH];
#pragma unroll
      for (int r = 0; r < TH; ++r) {
        const bool here = i >= r;
        const int slot = here ? (i - r) * TH + r : (C + i - r) * TH + r;
        const T *rp = (here ? rec_cur : rec_old) + slot * RW;
        const uint32_t code = cws[u][r];
        const T *rd = &rd_lds[code & 3u][0][lane];
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const T x1a = cur[g][r], x1b = prv[g][r];
          const T x2a = r == 0 ? hb1[hbp][u][g] : cur[g][r >= 1 ? r - 1 : 0];
          const T x2b = r == 0 ? hb2[hbp][u][g] : (r == 1 ? b1p[g] : prv[g][r >= 2 ? r - 2 : 0]);
          T num = fma(rp[1], vv0[g], rp[0]);
          num = fma(rp[2], vv1[g], num);
          num = fma(aa0[g], fma(rp[3], x1a, fma(rp[4], x1b, rp[5])), num);
          num = fma(aa1[g], fma(rp[6], x2a, fma(rp[7], x2b, rp[8])), num);
          nw[g][r] = num * rd[g * kWave];
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        b1p[g] = hb1[hbp][u][g];
#pragma unroll
        for (int r = 0; r < TH; ++r) {
          prv[g][r] = cur[g][r];
          cur[g][r] = nw[g][r];
        }
      }
      // stores: row r holds column t - r (branch-free, see rowrs)
#pragma unroll
      for (int r = 0; r < TH; ++r) {
        if (FIRST && i < r) continue;  // the columns before the strip's start
        const int x = t - r;
        const bool ok = !(cws[u][r] & R_SKIP) && r < cnt1 && x < n0;
        const uint32_t at = ok ? (uint32_t)xm(x) * colb : kDrop;
#pragma unroll
        for (int g = 0; g < G; ++g) buffer_store(nw[g][r], rowrs[r], kst[g] + at, 0u);
      }
      // the next row's start: inject its images before its first column
      if constexpr (FIRST && i + 1 < TH) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          cur[g][i + 1] = left_image(g, i + 1, 1);
          prv[g][i + 1] = left_image(g, i + 1, 2);
        }
      }
      // hand the top two rows on: column t - TH + 1 of row TH - 1, column
      // t - TH + 2 of row TH - 2 (the slot of a column before the strip's
      // start is rewritten with its real value before the consumer reads it)
#pragma unroll
      for (int g = 0; g < G; ++g) {
        ring[w][(t - TH + 1) & (R - 1)][0][g][lane] = nw[g][TH - 1];
        ring[w][(t - TH + 2) & (R - 1)][1][g][lane] = nw[g][TH - 2];
      }
      if constexpr (u == CH - 1) {
        const int done = min(max(t - TH + 2, 0), n0);  // columns whose two top rows are complete
        if (lmake) lds_post(&made[w], done);
        if (lwait) lds_post(&used[w], t + 1);
        if (gmake) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
          __builtin_amdgcn_s_waitcnt(0);  // every store of the wavefront has reached the L2
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
          if (lane == 0)
            __hip_atomic_store(publish, (int32_t)(seq * (uint32_t)n0 + (uint32_t)done), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    });
    // the next chunk's records; the buffer is the one of chunk k - 1, no
    // longer read
    stage(k + 1, raw);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  chunk(0, std::true_type{});
  for (int k = 1; k < nchunks; ++k) chunk(k, std::false_type{});
}

}  // namespace

template <typename T, int TH, int G, int NW>
void launch_strips_as(const Batch<T> &B, hipStream_t st, const Scratch &scr) {
  const dim3 grid((unsigned)B.h_strip_off[B.nprob]);
  if (B.y2wall)
    hipLaunchKernelGGL((sweep_strips_kernel<T, TH, G, NW, true>), grid, dim3(kWave * NW), 0, st, B.d_geo,
                       B.d_strip_off, B.nprob, B.strip_stride, scr.progress, scr.xcc);
  else
    hipLaunchKernelGGL((sweep_strips_kernel<T, TH, G, NW, false>), grid, dim3(kWave * NW), 0, st, B.d_geo,
                       B.d_strip_off, B.nprob, B.strip_stride, scr.progress, scr.xcc);
}

template <typename T>
hipError_t launch_sweep_strips(const Batch<T> &B, hipStream_t st, const Scratch &scr) {
  switch (B.strip_shape) {
    case kStrip4x2: launch_strips_as<T, 4, 2, 4>(B, st, scr); break;
    case kStrip4x1: launch_strips_as<T, 4, 1, 8>(B, st, scr); break;
    case kStrip2x2: launch_strips_as<T, 2, 2, 4>(B, st, scr); break;
    default: launch_strips_as<T, 2, 1, 8>(B, st, scr); break;
  }
  return hipGetLastError();
}

}  // namespace pdvm
