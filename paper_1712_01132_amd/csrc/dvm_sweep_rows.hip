// Step (i) of the iteration (Sec. 3.1, Algorithm 1) on gfx950 for 2D problems
// as one launch: the row pipeline of tile rows, and the XCD placement probe.
#include "dvm_device.h"

namespace pdvm {
namespace {

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
    sweep_rows_kernel(const Geo<T> *__restrict__ G, const int *__restrict__ row_off, int nprob, int stride,
                      int32_t *__restrict__ prog_scr, uint8_t *__restrict__ xcc_scr) {
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
  const int row0 = nprob > 1 ? row_off[p] : 0;
  // counters and XCD records: the problem's own, or its range of a scratch region
  const gptr<int32_t> progress = as_global(prog_scr ? prog_scr + row0 : G_.progress);
  const gptr<int32_t> fault = as_global(&G_.ctl->fault);
  const uint32_t seq = (uint32_t)G_.seq;
  const int n0 = dm.n[0], n1 = dm.n[1];
  const int nchains = ngroups << DIM;
  // block = row_off[p] + band * stride + c; stride and row_off[p] are
  // multiples of 8, so chain c of every band runs on XCD (c mod 8) under
  // round-robin placement
  const int local_b = blockIdx.x - (nprob > 1 ? row_off[p] : 0);
  const int c = local_b % stride;
  const int band = local_b / stride;
  if (c >= nchains) return;  // padding of the band to a multiple of 8 blocks
  if (LOCAL && threadIdx.x == 0) {
    // the XCD this block runs on: the reduction kernel discards the iterate
    // unless every block of this chain ran on one XCD (the LOCAL protocol's premise)
    uint32_t xcc;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
    as_global(xcc_scr ? xcc_scr + row0 : G_.xcc_seen)[local_b] = (uint8_t)(xcc & 0xFFu);
  }
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
  // wall clock (checked every 64 polls) it flags ctl->fault and gives up. A
  // fault already flagged by any wavefront ends the wait at the next check:
  // the iterate is discarded anyway, so every wavefront runs to its end fast.
  auto bounded_wait = [&](auto ready, int sleep2) __attribute__((always_inline)) {
    int n = 0;
    int64_t t0 = 0;
    while (!ready()) {
      if ((++n & 63) == 0) {
        const int64_t t = wall_clock64();
        if (__hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
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
    for (int k = 0; k < TT; ++k)
      hrow[k] = (gptr<char>)(hz + (int64_t)((uint64_t)(uint32_t)((ys + k * s[1]) * n0 + xs) * (uint32_t)Kp));
    const int64_t colb = (int64_t)s[0] * Kp * (int64_t)sizeof(T);  // bytes from one column to the next
    // a whole tile is stored through one buffer resource based at its
    // lowest-addressed voxel, with wavefront-constant row and column offsets
    const __amdgpu_buffer_rsrc_t tile_rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(T *)(hz + (int64_t)((uint64_t)(uint32_t)(ylo * n0 + (s[0] > 0 ? xs : xs - (TT - 1))) * (uint32_t)Kp)),
        (short)0, -1, kBufferFlags);

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

}  // namespace

template <typename T, bool LOCAL>
void launch_rows_local(const Batch<T> &B, dim3 grid, hipStream_t st, const Scratch &scr) {
#define PDVM_ROWS(TTV, Y2, E)                                                                   \
  hipLaunchKernelGGL((sweep_rows_kernel<T, TTV, Y2, LOCAL, band_waves(TTV), E>), grid,         \
                     dim3(kWave * band_waves(TTV)), 0, st, B.d_geo, B.d_row_off, B.nprob, B.row_stride, \
                     scr.progress, scr.xcc)
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
hipError_t launch_sweep_rows(const Batch<T> &B, bool local, hipStream_t st, const Scratch &scr) {
  const dim3 grid((unsigned)B.h_row_off[B.nprob]);
  if (local) launch_rows_local<T, true>(B, grid, st, scr);
  else launch_rows_local<T, false>(B, grid, st, scr);
  return hipGetLastError();
}

namespace {
template <typename T>
__global__ void progress_reset_kernel(const Geo<T> *__restrict__ G, const int *__restrict__ off, int strips,
                                      int32_t *prog) {
  const int p = blockIdx.x;
  const uint32_t per = strips ? (uint32_t)G[p].n[0] : (uint32_t)G[p].ntile[0];
  const int32_t below = (int32_t)((uint32_t)G[p].seq * per);
  for (int i = off[p] + threadIdx.x; i < off[p + 1]; i += blockDim.x) prog[i] = below;
}
}  // namespace

template <typename T>
hipError_t launch_progress_reset(const Batch<T> &B, const int *d_off, bool strips, int32_t *progress, hipStream_t st) {
  hipLaunchKernelGGL((progress_reset_kernel<T>), dim3((unsigned)B.nprob), dim3(256), 0, st, B.d_geo, d_off,
                     strips ? 1 : 0, progress);
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

template hipError_t launch_sweep_rows<double>(const Batch<double> &, bool, hipStream_t, const Scratch &);
template hipError_t launch_sweep_rows<float>(const Batch<float> &, bool, hipStream_t, const Scratch &);
template hipError_t launch_progress_reset<double>(const Batch<double> &, const int *, bool, int32_t *, hipStream_t);
template hipError_t launch_progress_reset<float>(const Batch<float> &, const int *, bool, int32_t *, hipStream_t);

}  // namespace pdvm
