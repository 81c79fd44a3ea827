// Step (i) of the iteration (Sec. 3.1, Algorithm 1) on gfx950: the upwind sweep
// (Eq. numerical stencil, Eq. Discretised_linearised_Boltzmann_equations) as one
// launch per diagonal of sweep tiles, for 2D and 3D problems and batches.
#include "dvm_device.h"

namespace pdvm {
namespace {

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
// EXT bit 0 (PSI, 2D): slots of h and of psi; bit 1 (SH): the Shakhov
// heat-flux source, whose per-voxel values nu (4/5)(1 - Pr) q_j end the record;
// bit 2 (MW): Maxwell walls. A voxel whose axis-j stencil meets a wall (code
// bit 4 + j) adds a_j (1 - alpha) times its own previous-iteration value of
// the velocity mirrored in e_j; the record's wall term is alpha rho_w.
// h at an upstream node (x, y, z) along axis j, as upstream_fluid but without
// the jump across the x1 wrap (the caller adds it where the value is used, so
// nothing waits for the load early) and with no branch: the buffer, the node
// and the velocity slot are selected (uniform values), so the load is issued
// whatever the case and many can be in flight before the first wait.
// The node's offset is formed in 32 bits (a problem has under 2^31 / 6
// voxels) and scaled by the voxel's bytes colb in one 32 x 32 -> 64 bit
// product: these are scalar instructions, a dozen per halo value fewer than
// with 64-bit index arithmetic.
template <typename T>
__device__ __forceinline__ T upstream_sel(const Dom<T> &g, gptr<const T> hc, gptr<const T> hp, int j, int x, int y,
                                          int z, int kofs, int kmir, uint32_t colb) {
  int c[3] = {x, y, z};
  const bool in = c[j] >= 0 && c[j] < g.n[j];
  const Img im = image_of(j, c[j], g.n[j], g.latp);
  c[j] = in ? c[j] : im.r;
  const int k = (!in && im.mir) ? kmir : kofs;
  const uint32_t cell = (uint32_t)(c[0] + g.n[0] * (c[1] + g.n[1] * c[2]));
  const gptr<const char> b = (gptr<const char>)(in ? hc : hp) + (uint64_t)cell * colb;
  return ((gptr<const T>)b)[k];
}
// The jump that upstream_sel leaves out at x1 = x (images across the wrap).
template <typename T>
__device__ __forceinline__ T wrap_jump(const Dom<T> &g, int x) {
  return (x < 0 ? T(1) : (x >= g.n[0] ? T(-1) : T(0))) * g.jump;
}

// LDS of one tile wavefront: the reciprocal denominators of its 64
// velocities and the records of up to PZ planes (128 voxels in 3D).
template <typename T, int DIM, int TT, int EXT>
struct TileLds {
  static constexpr int NC = TT * TT;
  // a record: src (4), nu tau, per axis (c1, c2, w), [q]; its stride RW is
  // padded to 16 bytes, so that a voxel's record is read with 16-byte loads
  static constexpr int RW0 = 5 + 3 * DIM + ((EXT & 2) ? DIM : 0);
  static constexpr int RW = (RW0 * (int)sizeof(T) + 15) / 16 * 16 / (int)sizeof(T);
  static constexpr int PZ = DIM == 3 ? 128 / NC : 1;
  // 3D with 4 x 4 tiles: the two x3-upstream planes of the tile's voxels are
  // carried in registers, ZN values each (one unused value otherwise)
  static constexpr bool ZREG = DIM == 3 && TT == 4;
  static constexpr int ZN = ZREG ? NC : 1;
  T rd[8 * kWave];
  alignas(16) T rec[PZ * NC * RW];
  uint32_t rcode[PZ * NC];
};

// The sweep of one tile (physical tile coordinates tpos) for the 64 velocities
// of group grp in sign octant o; every value it reads outside the tile is final.
// `before` runs once the tile's first records are being loaded and before any
// value outside the tile is read (the queue sweep waits for its upstream tiles
// there). CARRY (3D, 4 x 4 tiles): zc holds the tile's x3-upstream planes
// one and two back (zc[0 .. ZN), zc[ZN .. 2 ZN)) as the caller carries them
// over from the tile below in the same column, unless zload asks for them to
// be loaded from h; it leaves holding the tile's last two planes.
template <typename T, int DIM, int TT, bool Y2WALL, int EXT, bool CARRY = false, typename Before>
__device__ __forceinline__ void sweep_tile(const Geo<T> &G_, int o, int grp, const int (&tpos)[3],
                                           TileLds<T, DIM, TT, EXT> &L, Before &&before, T *zc = nullptr,
                                           bool zload = true) {
  constexpr bool PSI = (EXT & 1) != 0, SH = (EXT & 2) != 0, MW = (EXT & 4) != 0;
  static_assert(!(MW && Y2WALL), "Maxwell walls need stencil rule 1");
  constexpr int NC = TT * TT;
  constexpr int RW = TileLds<T, DIM, TT, EXT>::RW;
  // 3D: the records of PZ planes (128 voxels) are staged at once, before any
  // store of them; KV voxels per lane
  constexpr int PZ = TileLds<T, DIM, TT, EXT>::PZ, KV = (PZ * NC + kWave - 1) / kWave;
  T *const rd_lds = L.rd;
  T *const rec = L.rec;
  uint32_t *const rcode = L.rcode;
  // every per-problem value is read once here; the loops below see registers
  const Dom<T> dm = dom_of(G_);
  const int Ko = G_.Ko, Ko_pad = G_.Ko_pad, tau_fb = G_.tau_fb;
  const int tile[3] = {G_.tile[0], G_.tile[1], G_.tile[2]};
  const gptr<const T> absv = as_global(G_.absv), avv = as_global(G_.av), rden = as_global(G_.rden),
                      vsq = as_global(G_.vsqm);
  const gptr<T> hc = as_global(G_.hcur);
  const gptr<const T> hcc = hc;
  const gptr<const T> hp = as_global(G_.hprev);
  const gptr<const T> src = as_global(G_.srccur);
  const gptr<const T> srct = as_global(G_.srctcur);
  const gptr<const T> srcq = as_global(G_.srcqcur);
  const gptr<const T> wall = as_global(G_.wallcur);
  const gptr<const uint32_t> flags = as_global(G_.flags);
  const int n0 = dm.n[0], n1 = dm.n[1];
  const int lane = threadIdx.x;
  const int q = grp * kWave + lane;
  const bool active = q < Ko;
  // a lane past the octant (last group only) reads the octant's last slot,
  // which its own wavefront owns: it touches no other wavefront's lines
  const int qq = active ? q : Ko - 1;
  const uint32_t colb = (uint32_t)(G_.Kpad * (int64_t)sizeof(T));  // bytes per voxel
  constexpr uint32_t kDrop = 0x40000000u;  // past any row's range; two of them do not wrap
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
  T rdv[1 << DIM];  // written to LDS after the first records' loads are issued
#pragma unroll
  for (int c = 0; c < (1 << DIM); ++c) rdv[c] = rden[c * Ko_pad + qq];
  const T vsqm = tau_fb ? vsq[qq] : T(0);
  const int kofs = o * Ko_pad + qq;
  const uint32_t kst = active ? (uint32_t)kofs * (uint32_t)sizeof(T) : kDrop;  // the lane's byte offset in a voxel
  int kmir[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) kmir[j] = (o ^ (1 << j)) * Ko_pad + qq;

  int lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    lo[j] = tpos[j] * tile[j];
    cnt[j] = min(tile[j], dm.n[j] - lo[j]);
  }
  const int xs = s[0] > 0 ? lo[0] : lo[0] + cnt[0] - 1;
  const int ys = s[1] > 0 ? lo[1] : lo[1] + cnt[1] - 1;
  // 3D with 4 x 4 tiles: the two planes upstream along x3 of every voxel of
  // the tile's plane, ZA one plane back, ZB two, are loaded from h (or the
  // images) for the tile's first plane (or come with the column) and then
  // carried in registers from plane to plane (each voxel's new value replaces
  // ZA, whose value moves to ZB). 8 x 8 tiles read them from h per
  // anti-diagonal (128 more registers would cost them their occupancy).
  constexpr bool ZREG = TileLds<T, DIM, TT, EXT>::ZREG;
  constexpr int ZN = TileLds<T, DIM, TT, EXT>::ZN;
  T ZAl[ZN], ZBl[ZN];
  T *const ZA = CARRY ? zc : ZAl;
  T *const ZB = CARRY ? zc + ZN : ZBl;
  const int64_t Kp = dm.Kpad;
  auto zof = [&](int c3) { return s[2] > 0 ? lo[2] + c3 : lo[2] + cnt[2] - 1 - c3; };
  // the halos of plane z (the current sweep, or the images of the previous
  // iterate outside the domain). Rows and columns past a ragged tile re-read
  // its last one: only voxels outside the tile, which are never stored, see them.
  auto load_halo = [&](int z, T(&L1)[TT], T(&L2)[TT], T(&B1)[TT], T(&B2)[TT]) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < TT; ++k) {
      const int y = ys + min(k, cnt[1] - 1) * s[1], x = xs + min(k, cnt[0] - 1) * s[0];
      L1[k] = upstream_sel(dv, hcc, hp, 0, xs - s[0], y, z, kofs, kmir[0], colb);
      L2[k] = upstream_sel(dv, hcc, hp, 0, xs - 2 * s[0], y, z, kofs, kmir[0], colb);
      B1[k] = upstream_sel(dv, hcc, hp, 1, x, ys - s[1], z, kofs, kmir[1], colb);
      B2[k] = upstream_sel(dv, hcc, hp, 1, x, ys - 2 * s[1], z, kofs, kmir[1], colb);
    }
  };
  // records of the voxels of planes c0 .. c0 + np - 1 (lane l takes voxels
  // l, l + 64, ...). The voxel's sources and wall values are loaded together
  // with its flags (valid addresses whatever the flags say) and every record
  // value is selected, not branched on, so one round trip serves them all.
  // `before` runs between the loads and the LDS writes (the queue sweep polls
  // its upstream tiles there, so the polls and these loads share a round trip)
  auto stage = [&](int c0, int np, auto &&before) __attribute__((always_inline)) {
    uint32_t f[KV];
    T sv[KV][5], wv[KV][DIM], qv[KV][DIM];
    int xy[KV][3];
#pragma unroll
    for (int kv = 0; kv < KV; ++kv) {
      const int v = lane + kv * kWave;
      const int pz = min(v / NC, np - 1), i = v % TT, r = (v / TT) % TT;
      const int x = xs + min(i, cnt[0] - 1) * s[0], y = ys + min(r, cnt[1] - 1) * s[1];
      const int z = zof(c0 + pz);
      xy[kv][0] = x;
      xy[kv][1] = y;
      xy[kv][2] = z;
      const int c = (y + n1 * z) * n0 + x;
      f[kv] = flags[c];
      const gptr<const T> sp = src + c * kSrcStride;
      sv[kv][0] = sp[0];
      sv[kv][1] = sp[1];
      sv[kv][2] = sp[2];
      sv[kv][3] = DIM == 3 ? sp[3] : T(0);
      sv[kv][4] = tau_fb ? srct[c] : T(0);
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        wv[kv][j] = wall[c * 6 + 2 * j + pin[j]];
        qv[kv][j] = SH ? srcq[c * 4 + j] : T(0);
      }
    }
    before();
#pragma unroll
    for (int kv = 0; kv < KV; ++kv) {
      const int v = lane + kv * kWave;
      if (KV * kWave > PZ * NC && v >= PZ * NC) break;
      const int pz = v / NC, i = v % TT, r = (v / TT) % TT;
      const bool in = pz < np && i < cnt[0] && r < cnt[1];
      const bool fl = in && !(f[kv] & F_SOLID);
      T *rp = rec + v * RW;
#pragma unroll
      for (int k = 0; k < 5; ++k) rp[k] = fl ? sv[kv][k] : T(0);  // a skipped voxel's record is 0: it computes 0
      if (SH) {
#pragma unroll
        for (int j = 0; j < DIM; ++j) rp[5 + 3 * DIM + j] = fl ? qv[kv][j] : T(0);
      }
      uint32_t code = 0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        const uint32_t fj = f[kv] >> fbit(j, sidx[j]);
        const bool first = fj & 1u, y1s = fj & 2u, y2s = fj & 4u;
        T c1 = first ? (y1s ? T(0) : T(1)) : T(2);
        T c2 = first ? T(0) : T(-0.5);
        T w = (first && y1s) ? (MW ? alpha * wv[kv][j] : wv[kv][j]) : T(0);
        if (Y2WALL && fl && !first && y2s) {
          c2 = T(0);
          w = T(-0.5) * wall_at_y1(dm, wall, j, s[j], pin[j], xy[kv][0], xy[kv][1], xy[kv][2]);
        }
        rp[5 + 3 * j] = fl ? c1 : T(0);
        rp[6 + 3 * j] = fl ? c2 : T(0);
        rp[7 + 3 * j] = fl ? w : T(0);
        code |= (first ? 1u : 0u) << j;
        if (MW && first && y1s) code |= 16u << j;
      }
      rcode[v] = fl ? code : R_SKIP;
    }
  };

  const T jx1 = wrap_jump(dv, xs - s[0]), jx2 = wrap_jump(dv, xs - 2 * s[0]);  // the same for every plane
  // the tile's first plane: records, halos and (4 x 4 tiles in 3D) the two
  // planes below, all issued before any wait
  T L1[TT], L2[TT], B1[TT], B2[TT];
  stage(0, min(PZ, cnt[2]), before);
#pragma unroll
  for (int c = 0; c < (1 << DIM); ++c) rd_lds[c * kWave + lane] = rdv[c];
  load_halo(zof(0), L1, L2, B1, B2);
  if (ZREG && (!CARRY || zload)) {
    const int z = zof(0);
#pragma unroll
    for (int v = 0; v < (ZREG ? NC : 0); ++v) {
      const int x = xs + min(v % TT, cnt[0] - 1) * s[0], y = ys + min(v / TT, cnt[1] - 1) * s[1];
      ZA[v] = upstream_sel(dv, hcc, hp, 2, x, y, z - s[2], kofs, kmir[2], colb);
      ZB[v] = upstream_sel(dv, hcc, hp, 2, x, y, z - 2 * s[2], kofs, kmir[2], colb);
    }
  }
  __syncthreads();
  // one plane; the first is peeled off the loop, so that the loop is entered,
  // as it is re-entered, right after a plane's stores: its waits for the
  // halos loaded ahead then never cover those stores. The last is peeled too:
  // it loads no halos ahead (one-plane tiles, rare, reload their own)
  auto plane = [&](int c3, auto next) __attribute__((always_inline)) {
    constexpr bool NEXT = decltype(next)::value;  // a plane follows in this tile
    const int z = zof(c3);
    const int pz = c3 % PZ;
    if (c3 > 0 && pz == 0) {  // the next chunk of records (only LDS is written here)
      __syncthreads();
      stage(c3, min(PZ, cnt[2] - c3), [] {});
      __syncthreads();
    }
    // the next plane's halos, issued before this plane's stores: waiting for
    // them then does not wait for the stores
    T L1n[TT], L2n[TT], B1n[TT], B2n[TT];
    if (DIM == 3 && NEXT) load_halo(zof(min(c3 + 1, cnt[2] - 1)), L1n, L2n, B1n, B2n);
    const T *recp = rec + pz * NC * RW;
    const uint32_t *rcodep = rcode + pz * NC;
    // stores: one buffer resource per row of the tile (a row of h spans below
    // 1 GiB, checked by the host); a voxel that is not stored (solid, past a
    // ragged tile) or a lane past the octant gets an offset past the
    // resource's range, which the hardware drops. No branch around the
    // stores, so the wait counts stay exact and a wait for the next plane's
    // halos never waits for this plane's stores.
    __amdgpu_buffer_rsrc_t rowrs[TT];
#pragma unroll
    for (int k = 0; k < TT; ++k)
      rowrs[k] = __builtin_amdgcn_make_buffer_rsrc(
          (void *)((gptr<char>)hc + (uint64_t)(uint32_t)((n1 * z + ys + min(k, cnt[1] - 1) * s[1]) * n0) * colb),
          (short)0, (int)(colb * (uint32_t)n0), kBufferFlags);
    // --- the plane's anti-diagonals ---------------------------------------
    T D1[TT], D2[TT];
#pragma unroll
    for (int k = 0; k < TT; ++k) D1[k] = D2[k] = T(0);
#pragma unroll
    for (int d = 0; d < 2 * TT - 1; ++d) {
      T Nw[TT];
      uint32_t Nc[TT];
      T Z1[TT], Z2[TT];  // 8 x 8 tiles in 3D: the x3-upstream values from h
#pragma unroll
      for (int r = 0; r < TT; ++r) {
        Nw[r] = T(0);
        Nc[r] = R_SKIP;
        Z1[r] = Z2[r] = T(0);
        const int i = d - r;
        if (DIM == 3 && !ZREG && i >= 0 && i < TT) {
          const int x = xs + min(i, cnt[0] - 1) * s[0], y = ys + min(r, cnt[1] - 1) * s[1];
          Z1[r] = upstream_sel(dv, hcc, hp, 2, x, y, z - s[2], kofs, kmir[2], colb);
          Z2[r] = upstream_sel(dv, hcc, hp, 2, x, y, z - 2 * s[2], kofs, kmir[2], colb);
        }
      }
#pragma unroll
      for (int r = 0; r < TT; ++r) {
        const int i = d - r;
        if (i < 0 || i >= TT) continue;
        // no branch before the store: the loads of all voxels of the
        // anti-diagonal can be issued together (a skipped voxel's record is 0)
        const uint32_t code = __builtin_amdgcn_readfirstlane(rcodep[i + TT * r]);
        const T *rp = recp + (i + TT * r) * RW;
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
          const gptr<const T> hv_prev =
              hp + (int64_t)((n1 * z + ys + r * s[1]) * n0 + xs + i * s[0]) * Kp;
#pragma unroll
          for (int j = 0; j < DIM; ++j)
            if (code & (16u << j)) num = fma(am[j], hv_prev[kmir[j]], num);
        }
        const T x1a = i >= 1 ? D1[r] : L1[r] + jx1;
        const T x1b = i >= 2 ? D2[r] : (i == 1 ? L1[r] + jx1 : L2[r] + jx2);
        const T x2a = r >= 1 ? D1[r >= 1 ? r - 1 : 0] : B1[i];
        const T x2b = r >= 2 ? D2[r >= 2 ? r - 2 : 0] : (r == 1 ? B1[i] : B2[i]);
        num = fma(aa[0], fma(rp[5], x1a, fma(rp[6], x1b, PSI ? rp[7] * ph : rp[7])), num);
        num = fma(aa[1], fma(rp[8], x2a, fma(rp[9], x2b, PSI ? rp[10] * ph : rp[10])), num);
        if (DIM == 3) {
          const T za = ZREG ? ZA[ZREG ? i + TT * r : 0] : Z1[r], zb = ZREG ? ZB[ZREG ? i + TT * r : 0] : Z2[r];
          num = fma(aa[2], fma(rp[11], za, fma(rp[12], zb, rp[13])), num);
        }
        Nw[r] = num * rd_lds[(code & 7u) * kWave + lane];
        Nc[r] = code;
        if (ZREG) {  // this plane's value is the next plane's one-back, its one-back the two-back
          ZB[ZREG ? i + TT * r : 0] = ZA[ZREG ? i + TT * r : 0];
          ZA[ZREG ? i + TT * r : 0] = Nw[r];
        }
      }
      // the stores after the whole anti-diagonal: the loop above stays free
      // of control flow, so its loads and FMA chains interleave
#pragma unroll
      for (int r = 0; r < TT; ++r) {
        const int i = d - r;
        if (i < 0 || i >= TT) continue;
        const uint32_t at = (Nc[r] & R_SKIP) ? kDrop : (uint32_t)(xs + i * s[0]) * colb;
        buffer_store(Nw[r], rowrs[r], kst + at, 0u);
      }
#pragma unroll
      for (int r = 0; r < TT; ++r) {
        D2[r] = D1[r];
        D1[r] = Nw[r];
      }
    }
    if (DIM == 3 && NEXT) {
#pragma unroll
      for (int k = 0; k < TT; ++k) {
        L1[k] = L1n[k];
        L2[k] = L2n[k];
        B1[k] = B1n[k];
        B2[k] = B2n[k];
      }
    }
  };
  plane(0, std::true_type{});
  for (int c3 = 1; c3 < cnt[2] - 1; ++c3) plane(c3, std::true_type{});
  if (cnt[2] > 1) plane(cnt[2] - 1, std::false_type{});
}

// Step (i) for one diagonal of tiles: block = (octant, group, tile of the
// diagonal). In 2D the tiles (a, b) with a + b = diag are computed, the same
// for every octant; in 3D they come per octant from the table of tiles
// holding fluid.
template <typename T, int DIM, int TT, bool Y2WALL, int EXT>
__global__ void __launch_bounds__(kWave)
    sweep_kernel(const Geo<T> *__restrict__ G, const int *__restrict__ item_off, int nprob, int diag) {
  __shared__ TileLds<T, DIM, TT, EXT> L;
  const int p = nprob > 1 ? owner_of(item_off, nprob, blockIdx.x) : 0;
  const Geo<T> &G_ = G[p];
  if (!G_.run) return;  // converged problems retire
  const int ngroups = G_.ngroups;
  int item = nprob > 1 ? blockIdx.x - item_off[p] : blockIdx.x;
  int t, grp, o, tpos[3] = {0, 0, 0};
  if (DIM == 2) {
    const int amin = max(0, diag - (G_.ntile[1] - 1)), amax = min(diag, G_.ntile[0] - 1);
    const int ntd = amax - amin + 1;
    t = item % ntd;
    item /= ntd;
    grp = item % ngroups;
    o = item / ngroups;
    tpos[0] = amin + t;
    tpos[1] = diag - tpos[0];
#pragma unroll
    for (int j = 0; j < 2; ++j)
      if ((o >> j) & 1) tpos[j] = G_.ntile[j] - 1 - tpos[j];
  } else {
    const gptr<const int32_t> diag_off = as_global(G_.diag_off) + diag * 8;
    const int base = diag_off[0];
    o = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k)
      if (item >= (diag_off[k] - base) * ngroups) o = k;
    const int d0 = diag_off[o], ntd = diag_off[o + 1] - d0;
    item -= (d0 - base) * ngroups;
    t = item % ntd;
    grp = item / ntd;
    const gptr<const int32_t> diag_tiles = as_global(G_.diag_tiles);
#pragma unroll
    for (int j = 0; j < 3; ++j) tpos[j] = diag_tiles[(d0 + t) * 4 + j];
  }
  sweep_tile<T, DIM, TT, Y2WALL, EXT>(G_, o, grp, tpos, L, [] {});
}

// Step (i) as one launch: per XCD, kQueueSub queues of packed tile items (the
// velocity chains, i.e. problem x octant x group, are dealt to the XCDs and
// their sub-queues, each chain to one), ordered by tile diagonal. Every block
// takes items from the queues of the XCD it runs on (one claim ahead: the
// next item's counter update is in flight during a tile, and a claim only
// ever waits on items claimed before it); before a tile it waits for the done flags of
// its upstream tiles along each axis (same chain, so the same queue and XCD),
// and after it drains its stores into the L2 and stamps the tile's flag with
// the iteration's seq (flags are never reset). A wait only ever concerns an
// item taken earlier by a running wavefront, so the queue cannot deadlock.
// Producer and consumer share the XCD's L2: relaxed agent-scope flag stores
// and polls, no cache write-back or invalidation; the consumer's L1 holds no
// line of the tile before the flag (a chain's lines are read only by its own
// downstream tiles, and lanes past the octant read their own group's slot).
// Waits are bounded (Geo::wait_ticks) and flag ctl->fault; the blocks count
// the items they handled, and the reduction discards an iterate whose count
// falls short (a queue without blocks on its XCD).
// Item: bits 0-23 tile index (x1 fastest), 24-26 octant, 27-31 group,
// 32-47 problem, 48-53 waits: bit 2 j + k - 1 = wait for the k-th tile
// upstream along axis j (k = 2 where the first is one voxel thick).
// COL (3D): an item is a segment of Geo::col_tiles tiles of a column along x3
// (bits 0-23 the column's x1 + nt0 x2 tile index, 48-63 the segment), ordered
// by the diagonal of its first tile; one wavefront sweeps its tiles in turn,
// each with the waits of Geo::qtinfo and its own flag, keeping the
// x3-upstream planes in registers from tile to tile (no x3 halo loads but at
// the segment's start).
// Occupancy (FP32): 4 wavefronts per SIMD in 2D (the 64-problem batch sweeps in
// 2.21 ms instead of 2.29 with 3), 3 in 3D (at 4 the 4x4 tile spills its x3
// planes: 5.8 ms on the 96^3 pack instead of 4.3).
template <typename T, int DIM, int TT, bool Y2WALL, int EXT, bool COL>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? (DIM == 2 ? 4 : 3) : 1)))
    sweep_queue_kernel(const Geo<T> *__restrict__ G, const uint64_t *__restrict__ items,
                       const int32_t *__restrict__ q_off, int32_t *__restrict__ qctr, int32_t *__restrict__ qflags,
                       int nprob) {
  __shared__ TileLds<T, DIM, TT, EXT> L;
  if (nprob == 1 && !G[0].run) return;  // a stopped problem (its reduction checks nothing)
  uint32_t xcc;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
  xcc &= 7u;
  const int lane = threadIdx.x;
  int handled = 0;
  // the XCD's sub-queues holding items (the host fills them from the first
  // on), starting with one picked by the block index; a block that finds one
  // drained moves on to the next
  const int *const xo = q_off + xcc * kQueueSub;
  int used = 0;
  for (int i = 0; i < kQueueSub; ++i) used += xo[i + 1] > xo[i];
  const int sub0 = used ? (int)((blockIdx.x >> 3) % used) : 0;
  for (int si = 0; si < used; ++si) {
    const int qi = (int)xcc * kQueueSub + (sub0 + si) % used;
    const int qb = q_off[qi], qn = q_off[qi + 1] - qb;
    int32_t *const ctr = &qctr[qi * kCtrPad];
    // claims run two ahead: the item word of the next claim is loaded, and the
    // claim after it is in flight, while a tile runs
    auto claim = [&]() __attribute__((always_inline)) {
      int c = 0;
      if (lane == 0) c = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return c;
    };
    int k = __builtin_amdgcn_readfirstlane(claim());
    int kn = claim();
    uint64_t it = k < qn ? items[qb + k] : 0;
    while (k < qn) {
      kn = __builtin_amdgcn_readfirstlane(kn);
      const uint64_t itn = kn < qn ? items[qb + kn] : 0;
      const int knn = claim();
      ++handled;
      const int tile = (int)(it & 0xFFFFFFu), o = (int)((it >> 24) & 7u), grp = (int)((it >> 27) & 31u);
      const int p = (int)((it >> 32) & 0xFFFFu), wm = (int)((it >> 48) & 63u);
      const Geo<T> &G_ = G[p];
      if (G_.run) {
        const int32_t stamp = G_.seq;
        const int nt0 = G_.ntile[0], nt1 = G_.ntile[1];
        int32_t *const fl = qflags + G_.qflag_off + (int64_t)(o * G_.ngroups + grp) * G_.ntiles_all;
        // the upstream tiles' flags of tile wt with waits ww, polled by lane
        // b < 2 DIM for wait b, all at once, while the tile's first records
        // are being loaded
        int wt = tile, ww = wm;
        auto wait_upstream = [&]() __attribute__((always_inline)) {
          if (!ww) return;
          const int j = lane >> 1, kk = (lane & 1) + 1;
          const bool mine = lane < 2 * DIM && ((ww >> lane) & 1);
          const int stride = j == 0 ? 1 : (j == 1 ? nt0 : nt0 * nt1);
          const int up = mine ? wt - (((o >> j) & 1) ? -kk : kk) * stride : wt;
          int32_t *const fault = &G_.ctl->fault;
          const int64_t wait_ticks = G_.wait_ticks;
          int n = 0;
          int64_t t0 = 0;
          for (;;) {
            const bool ok = !mine || __hip_atomic_load(&fl[up], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == stamp;
            if (__all(ok)) break;
            if ((++n & 63) == 0) {
              const int64_t tn = wall_clock64();
              if (__hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
              if (n == 64) {
                t0 = tn;
              } else if (tn - t0 > wait_ticks) {
                if (lane == 0) __hip_atomic_store(fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
              }
            }
            __builtin_amdgcn_s_sleep(1);
          }
          __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no load outside the tile is moved above the polls
        };
        // after a tile: its stores drained into the L2, then its flag stamped
        auto publish = [&](int t) __attribute__((always_inline)) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
          __builtin_amdgcn_s_waitcnt(0);  // every store of the tile has reached the L2
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
          if (lane == 0) __hip_atomic_store(&fl[t], stamp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();  // the next tile's records overwrite this tile's
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        if constexpr (!COL) {
          const int tpos[3] = {tile % nt0, (tile / nt0) % nt1, tile / (nt0 * nt1)};
          sweep_tile<T, DIM, TT, Y2WALL, EXT>(G_, o, grp, tpos, L, wait_upstream);
          publish(tile);
        } else {
          // a column (tile = x1 + nt0 x2 tile index), or the segment wm of
          // col_tiles tiles of it: its tiles holding fluid in the octant's x3
          // order; the planes below a tile come in registers from the tile
          // before it, and are loaded from h at the segment's start and after
          // a tile without fluid (which is skipped, its flag never stamped).
          // Waits along x3 only where the tile below is another segment's.
          const int nt2 = G_.ntile[2], ncol = nt0 * nt1, S = G_.col_tiles;
          const int seg = (int)((it >> 48) & 0xFFFFu);
          const int cb0 = seg * S, cb1 = min(nt2, cb0 + S);
          const bool down = (o >> 2) & 1;
          const gptr<const int32_t> info = as_global(G_.qtinfo) + (int64_t)o * G_.ntiles_all;
          T zc[2 * TileLds<T, DIM, TT, EXT>::ZN];
          bool zload = true;
          int t = tile + (down ? nt2 - 1 - cb0 : cb0) * ncol;
          int inf = info[t];
          for (int cb = cb0; cb < cb1; ++cb) {
            const int tn = t + (down ? -ncol : ncol);
            const int infn = info[cb + 1 < cb1 ? tn : t];  // the next tile's, loaded ahead
            if (inf & 128) {
              const int tpos[3] = {tile % nt0, tile / nt0, t / ncol};
              wt = t;
              ww = inf & (15 | (cb == cb0 ? 48 : (cb == cb0 + 1 ? 32 : 0)));
              sweep_tile<T, DIM, TT, Y2WALL, EXT, true>(G_, o, grp, tpos, L, wait_upstream, zc, zload);
              publish(t);
              zload = false;
            } else {
              zload = true;
            }
            t = tn;
            inf = infn;
          }
        }
      }
      k = kn;
      kn = knn;
      it = itn;
    }
  }
  if (lane == 0)
    __hip_atomic_fetch_add(&qctr[(8 * kQueueSub + xcc) * kCtrPad], handled, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// The queue counters (taken per sub-queue, handled per XCD) before a queue
// sweep: a fill kernel, so that a captured graph holds no memset node.
__global__ void queue_reset_kernel(int32_t *qctr) {
  for (int i = threadIdx.x; i < kQueueCounters; i += blockDim.x) qctr[i * kCtrPad] = 0;
}

__global__ void fill_i32_kernel(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

}  // namespace

template <typename T, bool Y2WALL>
void launch_queue_rule(const Batch<T> &B, hipStream_t st, int32_t *qctr, int32_t *qflags) {
  hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(128), 0, st, qctr);
  const dim3 grid(kQueueBlocks);
#define PDVM_QUEUE_C(D, X, E, C)                                                                             \
  hipLaunchKernelGGL((sweep_queue_kernel<T, D, X, Y2WALL, E, C>), grid, dim3(kWave), 0, st, B.d_geo, B.d_qitems, \
                     B.d_q_off, qctr, qflags, B.nprob)
#define PDVM_QUEUE_E(D, X, E)                                   \
  if (D == 3 && B.use_columns) PDVM_QUEUE_C(D, X, E, D == 3); \
  else PDVM_QUEUE_C(D, X, E, false)
#define PDVM_QUEUE_T(D, E)                          \
  if (B.tile_edge <= 4) PDVM_QUEUE_E(D, 4, E);      \
  else PDVM_QUEUE_E(D, 8, E)
  if constexpr (!Y2WALL) {
    if (B.maxwell) {
      if (B.dim == 2) {
        if (B.shakhov) { PDVM_QUEUE_T(2, 7); }
        else if (B.psi) { PDVM_QUEUE_T(2, 5); }
        else { PDVM_QUEUE_T(2, 4); }
      } else {
        if (B.shakhov) { PDVM_QUEUE_T(3, 6); }
        else { PDVM_QUEUE_T(3, 4); }
      }
      return;
    }
  }
  if (B.dim == 2) {
    if (B.shakhov) { PDVM_QUEUE_T(2, 3); }
    else if (B.psi) { PDVM_QUEUE_T(2, 1); }
    else { PDVM_QUEUE_T(2, 0); }
  } else {
    if (B.shakhov) { PDVM_QUEUE_T(3, 2); }
    else { PDVM_QUEUE_T(3, 0); }
  }
#undef PDVM_QUEUE_T
#undef PDVM_QUEUE_E
#undef PDVM_QUEUE_C
}

template <typename T>
hipError_t launch_sweep_queue(const Batch<T> &B, hipStream_t st, const Scratch &scr) {
  int32_t *qctr = scr.qctr ? scr.qctr : B.d_qctr;
  int32_t *qflags = scr.qflags ? scr.qflags : B.d_qflags;
  if (B.y2wall) launch_queue_rule<T, true>(B, st, qctr, qflags);
  else launch_queue_rule<T, false>(B, st, qctr, qflags);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

template hipError_t launch_sweep_queue<double>(const Batch<double> &, hipStream_t, const Scratch &);
template hipError_t launch_sweep_queue<float>(const Batch<float> &, hipStream_t, const Scratch &);

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

template hipError_t launch_sweep<double>(const Batch<double> &, int, hipStream_t);
template hipError_t launch_sweep<float>(const Batch<float> &, int, hipStream_t);

}  // namespace pdvm
