// Internal declarations shared by the HIP kernels and the host library.
// Not part of the public C ABI (include/poredvm.h).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace pdvm {

constexpr int kWave = 64;     // CDNA wavefront width: one discrete velocity per lane
// Tile rows (one wavefront each) per block of the 2D row-pipeline sweep, by
// compiled tile edge: the LDS ring between them fits twice in one CU's LDS.
constexpr int band_waves(int tile_edge) { return tile_edge == 4 ? 8 : 4; }
constexpr int kRing = 64;     // permeability history kept at multiples of 100 iterations
constexpr int kMomBlock = 256;
constexpr int kSrcStride = 4; // per-voxel source record: nu rho, 2 nu u_1, 2 nu u_2, 2 nu u_3 (0 in 2D)

// Per-voxel flags, computed once on the host from the solid mask (the paper's
// pre-processing of the stencil order, Sec. 2.3). For axis j and upwind sign
// s (sidx = 0 for s = +1, 1 for s = -1): FIRST = use the first-order stencil;
// Y1S = the image of x - s e_j is solid (its wall value is the first upstream
// value); Y2S = second-order stencil whose image of x - 2 s e_j is solid
// (wall value there).
constexpr uint32_t F_SOLID = 1u;
__host__ __device__ constexpr int fbit(int j, int sidx) { return 1 + 3 * (2 * j + sidx); }
__host__ __device__ constexpr uint32_t f_first(int j, int sidx) { return 1u << fbit(j, sidx); }
__host__ __device__ constexpr uint32_t f_y1s(int j, int sidx) { return 1u << (fbit(j, sidx) + 1); }
__host__ __device__ constexpr uint32_t f_y2s(int j, int sidx) { return 1u << (fbit(j, sidx) + 2); }

// Device-resident control block. `par` selects which of the two buffers of
// every iterated array holds the last completed iteration; the reduction
// kernel flips it only when the new iterate is finite, so a failing
// iteration leaves the previous state intact. Every kernel returns at once
// while `stop` is set, so graph replays past convergence cost no work.
struct Ctl {
  int32_t par;
  int32_t stop;
  int32_t status;       // 0 running, 1 converged, 2 budget reached, -4 non-finite,
                        // -3 sweep abandoned (see fault)
  int32_t mode;         // 0 field residual, 1 paper Err(l)
  int32_t fault;        // a pipelined sweep was abandoned: 1 a wait gave up, 2 the
                        // blocks of a velocity chain ran on different XCDs (row and
                        // strip pipelines) or a queue sweep left tiles unswept. The iterate
                        // is discarded (par kept); only the host clears it
                        // (set_initial / set_state), so a poisoned problem stays stopped
  int32_t pad_;
  int64_t iter;         // iterations since the initial state
  int64_t iter_limit;   // stop (status 2) when iter reaches this
  double tol;
  double r, err, k, gp;
  double kn_coef;       // (2/sqrt(pi)) Kn
  double kring[kRing];  // k at iterations 100, 200, ... (cyclic)
};

template <typename T>
struct Geo {
  int32_t dim, n[3];
  int64_t N;
  int32_t Ko, Ko_pad, Kpad, ngroups;  // velocities per sign octant, padded, per voxel, 64-groups per octant
  int32_t lateral_periodic, tau_fb;
  int32_t psi;             // 2D with tau_fb: octant slots [Ko/2, Ko) hold psi of velocity q - Ko/2
  int32_t shakhov;         // the heat flux is fed back (Shakhov model)
  double sh_coef;          // (4/5)(1 - Pr)
  int32_t maxwell;         // Maxwell walls: a wall value is alpha (diffuse) + spec (mirrored previous h)
  T spec, alpha;           // 1 - alpha, alpha
  int32_t y2wall;          // stencil rule 0: a solid second image enters the second-order stencil
  T jump;                  // the jump the sweep adds across the x1 wrap (0 in the offset form)
  // Offset form (every problem without Maxwell walls): h is stored as its
  // deviation from the linear density ramp rho_r = J (1/2 - (x1 + 1/2) / n1),
  // which carries the jump of Eq. periodic_BC, so the stored values are of the
  // size of u and rho - rho_r rather than of J. The sweep is unchanged: the
  // ramp enters only through the records (see moments_kernel) and the jump
  // across the wrap is 0.
  int32_t dev;
  double ramp;             // J
  double w0, we;           // 2^dim sums over the slots of h of the rho and energy weights
  double nu, D[3];
  const uint32_t *flags;   // [N]
  const T *absv;           // [3][Ko_pad]   |v_j| of octant slot q
  const T *av;             // [3][Ko_pad]   |v_j| / dx
  const T *vsqm;           // [Ko_pad]      temperature-source factor: |v|^2 - 3/2 (3D),
                           //               v1^2 + v2^2 - 1 (2D), 1/2 (psi slots)
  const T *phm;            // [Ko_pad]      1 for a slot of h, 0 for a psi slot (no rho, u, wall or jump terms)
  const T *qsf;            // [Ko_pad]      Shakhov source factor of q.v: |v|^2 - 5/2 (2D: v1^2 + v2^2 - 2; psi 1/2)
  const T *rden;           // [8][Ko_pad]   1 / (nu + sum_j a_j (1 or 3/2)), bit j = first order on axis j
  const double *wq;        // [8][Ko_pad]   W, W|v1|, W|v2|, W|v3|, W |v|^2 (2D: + W/2), then the heat
                           //               flux's W |v_j| (|v|^2 - 5/2) (2D: v1^2 + v2^2 - 2);
                           //               psi slots: 0 except W in the energy row and W |v_j| for q
  T *h[2];                 // [N][Kpad]     distribution, voxel-major, velocity fastest
  T *src[2];               // [N][kSrcStride]
  T *srct[2];              // [N] nu tau (only with the temperature term fed back)
  T *srcq[2];              // [N][4] nu sh_coef q_j (Shakhov only, else null)
  T *wall[2];              // [N][6]        Phi_j^p / D_j  (p = 0: v_j > 0 half, 1: v_j < 0)
  double *rho[2];          // [N]
  double *u[2];            // [3][N]
  Ctl *ctl;
  double *part;            // [mom_blocks][4] per-block residual / flux partials
  int32_t mom_blocks;
  const int32_t *fluid_idx;  // [nfluid] the fluid voxels in index order (moment kernel's work list)
  int64_t nfluid;
  int32_t tile[3], ntile[3];
  // 2D: the tiles of each diagonal, as oriented coordinates (x1, x2, 0, pad),
  // diag_off [ndiag + 1]. 3D: per diagonal and sign octant (list d * 8 + o),
  // the physical coordinates (x1, x2, x3, pad) of the tiles holding fluid,
  // diag_off [ndiag * 8 + 1].
  const int32_t *diag_tiles;
  const int32_t *diag_off;
  int32_t ndiag;
  // Resolved for the next iteration by the kernels that change the state
  // (arm: from the control block; reduce: after its parity decision), so that
  // a sweep or moment launch needs one descriptor read and no control-block
  // read before its data loads.
  int32_t run = 0;            // 0 once the problem stopped (converged, budget, non-finite)
  int32_t cpar = 0;           // the control block's `par`
  T *hcur = nullptr;          // h being swept this iteration: h[par ^ 1]
  const T *hprev = nullptr;   // h of the previous iteration: h[par]
  const T *srccur = nullptr, *srctcur = nullptr, *wallcur = nullptr;  // src, srct, wall [par]
  const T *srcqcur = nullptr;  // srcq [par]
  int32_t seq = 0;            // advanced by every arm and reduction: stamps of the row pipeline
  int32_t *progress = nullptr;  // [bands][chains] tiles completed per band (row-pipeline sweep)
  int64_t wait_ticks = 0;       // a row-pipeline wait gives up after this many wall-clock ticks (2 s)
  // XCD-local row pipeline only (else null): every block records the XCD it ran
  // on, [row_blocks] bytes (block = band * row_stride + chain); the reduction
  // kernel discards the iterate unless all blocks of each chain agree
  uint8_t *xcc_seen = nullptr;
  int32_t row_blocks = 0, row_stride = 0, row_sets = 0;  // blocks, blocks per band, real ones per band
  // queue sweep: the done flag of tile t of chain c = o * ngroups + group is
  // qflags[qflag_off + c * ntiles_all + t] (qflags: the batch's flag array)
  int64_t qflag_off = 0;
  int32_t ntiles_all = 0;
  // queue of tile columns (3D): per sign octant and tile (physical index),
  // qtinfo[o * ntiles_all + t] = 128 if the tile holds fluid, plus its waits
  // in bits 0-5 as in a queue item (null for tile items)
  const int32_t *qtinfo = nullptr;
  int32_t col_tiles = 0;  // tiles per column item (its bits 48-63: which segment of the column)
};

// Square sweep tile edges in (x1, x2) compiled into the kernel; the host
// rounds a requested edge up to one of them.
constexpr int kTileEdge[2] = {4, 8};

// A batch of problems sharing dimension, precision, velocity grid, tile edge
// and stencil rule (sizes, geometries and Kn may differ). The hot kernels take
// the device array of descriptors and locate their problem from per-launch
// block offsets; a single problem is a batch of one.
template <typename T>
struct Batch {
  int nprob = 0, dim = 2, Ko = 0, tile_edge = 8, y2wall = 0, tau_fb = 0, psi = 0, shakhov = 0, maxwell = 0, ndiag_max = 0;
  const Geo<T> *d_geo = nullptr;
  const int *d_item_off = nullptr;   // [ndiag_max][nprob + 1] sweep blocks per diagonal
  const int *d_blk_off = nullptr;    // [nprob + 1] moment-kernel blocks
  const int *h_item_off = nullptr;   // host copies
  const int *h_blk_off = nullptr;
  // row-pipeline sweep: problem p owns blocks [row_off[p], row_off[p + 1]),
  // its tile rows times row_stride (the chain count rounded up to 8); both
  // multiples of 8
  const int *d_row_off = nullptr;
  const int *h_row_off = nullptr;
  int row_stride = 8;
  // strip pipeline (2D): problem p owns blocks [strip_off[p], strip_off[p + 1]),
  // its bands times strip_stride (chain sets rounded up to 8); strip_shape is
  // one of kStrip* (rows per strip, velocity groups per wavefront, strips per block)
  const int *d_strip_off = nullptr;
  const int *h_strip_off = nullptr;
  int strip_stride = 8, strip_shape = 0;
  int use_strips = 0;  // the sweep is the strip pipeline (its block offsets locate the XCD records)
  // queue sweep: per-XCD sub-queues of packed tile items, sub-queue
  // x * kQueueSub + i at qitems[q_off[.] .. q_off[. + 1]); the batch's
  // counters [kQueueCounterInts] and done flags (scratch); q_total items in all
  // use_columns: an item is a column of tiles along x3 (3D), walked by one
  // wavefront in the octant's x3 order
  int use_queue = 0, q_total = 0, use_columns = 0;
  const uint64_t *d_qitems = nullptr;
  const int32_t *d_q_off = nullptr;
  int32_t *d_qctr = nullptr;
  int32_t *d_qflags = nullptr;
};

// Blocks of a queue-sweep launch: more than the 256 CUs of the GPU can hold at
// once; blocks that start late find the queues empty and end. Sub-queues per
// XCD (each with its own counter: one counter per XCD serialised the claims);
// counters: taken per sub-queue, then handled per XCD.
constexpr int kQueueBlocks = 4096;
constexpr int kQueueSub = 16;
constexpr int kQueueCounters = 8 * kQueueSub + 8;
// counter c at qctr[c * kCtrPad]: one 128-byte line each (claims on a shared
// line serialise: with 8 counters per line the claims alone took 2.9 ms per
// sweep of the 64-problem batch)
constexpr int kCtrPad = 32;
constexpr int kQueueCounterInts = kQueueCounters * kCtrPad;
// Tiles per item of the column queue (3D). Measured on the 96^3 pack (FP32,
// 4x4x4 tiles): 1: 4.34 ms per sweep, 2: 4.24, 3: 4.34, 4: 4.43, whole
// columns of 24: 5.21 (a long item started last holds up the end of the
// sweep); tile items 4.30.
constexpr int kColumnTiles = 2;

// Shapes of the strip pipeline: rows per strip TH x velocity groups per
// wavefront G, with the strips per block NW that each is compiled with.
enum { kStrip4x2 = 0, kStrip4x1 = 1, kStrip2x2 = 2, kStrip2x1 = 3, kStripShapes = 4 };
constexpr int strip_th(int shape) { return shape == kStrip4x2 || shape == kStrip4x1 ? 4 : 2; }
constexpr int strip_g(int shape) { return shape == kStrip4x2 || shape == kStrip2x2 ? 2 : 1; }
constexpr int strip_nw(int shape) { return strip_g(shape) == 2 ? 4 : 8; }

// Scratch memory of the iteration's kernels: the moment kernel's per-block
// partial sums, the row pipeline's progress counters and per-block XCD
// records. A null member means each problem's own, in its workspace
// (Geo::part, progress, xcc_seen). Otherwise it is one region for the whole
// batch: problem p's partial sums at part + 4 blk_off[p], its counters and XCD
// records at progress + row_off[p] and xcc + row_off[p].
struct Scratch {
  double *part = nullptr;
  int32_t *progress = nullptr;
  uint8_t *xcc = nullptr;
  int32_t *qctr = nullptr;    // queue sweep: counters [kQueueCounterInts]
  int32_t *qflags = nullptr;  // queue sweep: done flags
};

// Kernel launchers (dvm_sweep_diag.hip, dvm_sweep_rows.hip, dvm_iter.hip).
// All enqueue on `st`.
template <typename T>
hipError_t launch_sweep(const Batch<T> &B, int diag, hipStream_t st);
// The whole 2D sweep of every problem of the batch as one row-pipeline launch
// of bands of band_waves(tile edge) tile rows per block; `local`: every
// chain's bands run on one XCD (checked with launch_xcd_probe).
template <typename T>
hipError_t launch_sweep_rows(const Batch<T> &B, bool local, hipStream_t st, const Scratch &scr = Scratch{});
// The strip pipeline (2D, one launch for all problems of the batch).
template <typename T>
hipError_t launch_sweep_strips(const Batch<T> &B, hipStream_t st, const Scratch &scr = Scratch{});
// The tile sweep of every problem of the batch as one launch fed by per-XCD
// queues (after a fill kernel that clears the queue counters).
template <typename T>
hipError_t launch_sweep_queue(const Batch<T> &B, hipStream_t st, const Scratch &scr = Scratch{});
// The pipeline's progress counters of a batch-wide scratch region (blocks
// off[p] .. off[p + 1] of problem p), set below every stamp the next sweep of
// each problem publishes: seq * ntile0 for the row pipeline, seq * n0 for the
// strips; a fill kernel (no memset node when the caller captures a graph).
template <typename T>
hipError_t launch_progress_reset(const Batch<T> &B, const int *d_off, bool strips, int32_t *progress, hipStream_t st);
// p[0 .. n) = v (a fill kernel).
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
// out[b] = the XCD that block b of a `blocks`-block grid runs on.
hipError_t launch_xcd_probe(uint32_t *out, int blocks, int threads, hipStream_t st);
template <typename T>
hipError_t launch_moments(const Batch<T> &B, hipStream_t st, const Scratch &scr = Scratch{});
template <typename T>
hipError_t launch_reduce(const Batch<T> &B, hipStream_t st, const Scratch &scr = Scratch{});
template <typename T>
hipError_t launch_arm(const Batch<T> &B, double tol, int mode, int64_t max_iters, hipStream_t st);
template <typename T>
hipError_t launch_ctl_gather(const Batch<T> &B, Ctl *out, hipStream_t st);
template <typename T>
hipError_t launch_init_state(const Geo<T> &g, const double *rho, const double *u, hipStream_t st);
template <typename T>
hipError_t launch_diagnostics(const Geo<T> &g, double *tau, double *q, hipStream_t st);
template <typename T>
hipError_t launch_face_copy(const Geo<T> &g, int axis, int r, T *buf, int to_buf, hipStream_t st);

}  // namespace pdvm
