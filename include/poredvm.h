/*
 * poredvm: iterative discrete-velocity solve of the steady linearised BGK
 * equation on a voxelised porous geometry, on one AMD Instinct MI355X (gfx950).
 *
 * Reference: Ho, Zhu, Wu, Wang, Guo, Li, Zhang, "A multi-level parallel solver
 * for rarefied gas flows in porous media", arXiv:1712.01132.
 *   model and boundary conditions ......... Sec. 2.1, Eqs. linearised_Boltzmann_equation,
 *                                           diffusive-specular_BC (alpha = 1), wall_density,
 *                                           periodic_BC, symmetric_BC
 *   velocity grid ......................... Sec. 2.2 (half-range Gauss-Hermite, Cartesian)
 *   upwind stencil ........................ Sec. 2.3, Eq. numerical stencil
 *   iteration (sweep, BC, moments) ........ Sec. 3.1 steps (i)-(iii), Algorithm 1
 *   permeability and convergence .......... Eq. k_Gp, Sec. 3.1 steps (iv)-(v),
 *                                           Eq. convergence_criterion
 *
 * Conventions shared by every entry point:
 *  - Geometry: a voxel image of n[0] x n[1] (x n[2]) cubic voxels, index
 *    i + n0 * (j + n1 * l), x1 = the flow axis = the fastest index. Nodes sit at
 *    voxel centres; lengths are scaled by L = n[0] voxels (so dx = 1/n0) and
 *    Kn is referenced to that L.
 *  - The flow is driven by the periodic pressure jump along x1: molecules
 *    entering at the inlet carry h(outlet) + jump (Eq. periodic_BC); the
 *    paper's value is jump = 1. Lateral faces are specular (Eq. symmetric_BC,
 *    mirror plane = the outer voxel face) or, optionally, periodic.
 *  - The velocity grid is the tensor product of per-axis 1D lists that are
 *    symmetric about 0, even-sized and free of 0, with normalised weights
 *    (sum 1 per axis; they absorb exp(-v^2)/sqrt(pi)). In 2D the distribution
 *    is the reduced one with v3 integrated out.
 *  - Status codes are returned, never thrown; a message is kept per handle and
 *    per thread (pdvm_last_error).
 *  - All device work is enqueued on the stream given at creation; calls that
 *    return host data synchronise that stream first.
 *  - A handle may be used by one host thread at a time.
 */
#ifndef POREDVM_H
#define POREDVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PDVM_OK = 0,
  PDVM_NOT_CONVERGED = 1,   /* iteration budget used up; state valid and resumable */
  PDVM_E_INVAL = -1,        /* invalid argument or configuration */
  PDVM_E_NOMEM = -2,        /* allocation failed or workspace too small */
  PDVM_E_HIP = -3,          /* a HIP runtime call failed */
  PDVM_E_NONFINITE = -4,    /* r or k became NaN/Inf; the last good state is kept */
  PDVM_E_STATE = -5,        /* checkpoint buffer of the wrong size or problem; or iterating a
                               solver whose earlier sweep was abandoned (see pdvm_set_wait_limit) */
  PDVM_E_UNSUPPORTED = -6   /* valid but not implemented (e.g. the row pipeline in 3D) */
};

enum { PDVM_FP64 = 0, PDVM_FP32 = 1 };                       /* sweep + h storage precision */
enum { PDVM_LATERAL_SPECULAR = 0, PDVM_LATERAL_PERIODIC = 1 };
enum { PDVM_STOP_FIELD = 0, PDVM_STOP_PAPER_ERR = 1 };
/* Sweep schedules (results are bitwise identical between them):
 * DIAGONALS: one launch per diagonal of sweep tiles (all octants, velocity
 *            groups and problems of a batch in each launch);
 * ROWS:      2D: one launch for all problems of the batch, in which each
 *            wavefront pipelines a row of tiles behind the row below it;
 * ROWS_AGENT: ROWS with agent-scope release/acquire per tile, correct for any
 *            block placement (slower; ROWS uses it when the probe below fails);
 * STRIPS:    2D, isothermal source and diffuse walls: one launch for all
 *            problems of the batch, in which each wavefront walks a strip of
 *            voxel rows along x1 as a skewed front behind the strip below it,
 *            for one or two 64-velocity groups at once; needs every velocity
 *            chain on one XCD (probed at creation, else PDVM_E_UNSUPPORTED);
 *            only on request (slower than ROWS on one problem and than
 *            DIAGONALS on batches, as measured);
 * QUEUE:     one launch for all problems of the batch (2D or 3D): the tiles
 *            of every velocity chain wait in the queue of one XCD, in diagonal
 *            order; a block takes tiles from its own XCD's queue and waits for
 *            each tile's upstream neighbours' done flags (cheap: through that
 *            XCD's L2). Needs blocks on all 8 XCDs (probed at creation, else
 *            PDVM_E_UNSUPPORTED); an iterate whose queues were not all drained
 *            is discarded as for ROWS;
 * COLUMNS:   3D: QUEUE whose items are whole columns of tiles along x3, each
 *            swept by one wavefront tile after tile (the two planes below a
 *            tile stay in registers, and a column runs a tile or so behind its
 *            upstream columns, so the values it reads from them are still in
 *            the L2); the same requirements as QUEUE;
 * AUTO:      for a single 2D problem, ROWS when a probe of the block placement
 *            at creation shows that every velocity chain runs on one XCD (cheap
 *            synchronisation through its L2); for 3D problems and 2D batches,
 *            QUEUE when the probe finds all 8 XCDs; DIAGONALS otherwise. */
enum { PDVM_SCHEDULE_AUTO = 0, PDVM_SCHEDULE_DIAGONALS = 1, PDVM_SCHEDULE_ROWS = 2, PDVM_SCHEDULE_ROWS_AGENT = 3,
       PDVM_SCHEDULE_STRIPS = 4, PDVM_SCHEDULE_QUEUE = 5, PDVM_SCHEDULE_COLUMNS = 6 };

typedef struct pdvm_solver pdvm_solver;

typedef struct {
  int32_t dim;               /* 2 or 3 */
  int32_t n[3];              /* voxels per axis; n[2] ignored (1) in 2D; each >= 2 */
  const uint8_t *solid;      /* host, n0*n1(*n2) bytes, nonzero = solid; copied at create */
  int32_t nv[3];             /* 1D velocity counts per axis (even, >= 2) */
  const double *vnode[3];    /* host, ascending 1D nodes per axis; copied */
  const double *vweight[3];  /* host, 1D weights per axis, > 0, sum 1; copied */
  double kn;                 /* Knudsen number (> 0; +INFINITY = free molecular) */
  double jump;               /* pressure jump added at the x1 wrap (paper: 1.0) */
  int32_t precision;         /* PDVM_FP64 or PDVM_FP32 (moments and reductions stay FP64) */
  int32_t lateral_bc;        /* PDVM_LATERAL_SPECULAR (paper) or PDVM_LATERAL_PERIODIC */
  int32_t tau_feedback;      /* 0 = isothermal source as in the paper's runs; 1 = feed the
                                temperature term back. In 2D this also carries the second
                                v3-reduced function psi = int (v3^2 - 1/2) h dv3 in a second
                                slot per velocity (twice the work and memory; at most 512
                                velocities per sign octant, else PDVM_E_INVAL) */
  int32_t check_every;       /* host polls convergence every this many iterations (0 = 16) */
  int32_t tile[3];           /* sweep tile extent per axis in voxels (0 = default: 8 along
                                x1, x1's value along x2, 8 along x3); x1 and x2 are capped
                                at 8, x3 takes any depth */
  int32_t stencil_rule;      /* when the upwind stencil along an axis drops to first order
                                (Sec. 2.3 says: when the upstream point is a boundary point):
                                1 = when either of the two upstream images is solid;
                                0 = only when the first one is (a solid second image then
                                    enters the second-order stencil with its wall value;
                                    this iteration can diverge on some geometries) */
  int32_t sweep_schedule;    /* PDVM_SCHEDULE_*; ROWS(_AGENT) or STRIPS with dim 3, or COLUMNS
                                with dim 2, is PDVM_E_UNSUPPORTED;
                                a batch takes the first config's schedule */
  double prandtl;            /* 0 = BGK. > 0 (needs tau_feedback = 1): Shakhov model, whose
                                source adds (4/5)(1 - Pr) q.v (|v|^2 - 5/2) with the heat
                                flux q of the previous iteration (2D: reduced over v3, as
                                for tau), so that collisions relax q at Pr nu (a kinetic
                                model the method extends to, Sec. 1 and Sec. 2.1; Pr = 2/3
                                for a monatomic gas). Both sweep schedules carry it */
  double specular_fraction;  /* 1 - alpha of Maxwell walls (Eq. diffusive-specular_BC), in
                                [0, 1); 0 = diffuse walls as in the paper's runs. A solid met
                                by the first-order stencil of fluid node x along e_j emits
                                alpha times the diffuse value plus (1 - alpha) times the
                                previous iteration's h at x for the velocity mirrored in e_j.
                                Needs stencil_rule 1; both sweep schedules carry it; a
                                checkpoint then holds all of h */
} pdvm_config;

typedef struct {
  int64_t iters;             /* iterations completed in this call */
  int64_t total_iters;       /* iterations since the last initial state */
  double r;                  /* field residual max|u^l - u^(l-1)| / max|u^l| (FP64) */
  double err;                /* paper criterion Err(l) at the last multiple of 100, -1 if none */
  double k;                  /* apparent permeability (2/sqrt(pi)) Kn G_p */
  double gp;                 /* G_p = mean of u1 over all cells (solid = 0) */
  double seconds;            /* wall time of the call */
  int32_t converged;         /* 1 if stopped on the tolerance */
} pdvm_stats;

/* Half-range Gauss-Hermite velocity grid (Sec. 2.2): n_total/2 nodes of the
 * Gauss rule for exp(-x^2) on [0, inf), mirrored to both signs; weights
 * normalised to sum 1. nodes/weights: host arrays of n_total doubles (caller
 * owned). n_total even, 2..64. Returns PDVM_OK or PDVM_E_INVAL. */
int pdvm_halfrange_gh(int32_t n_total, double *nodes, double *weights);

/* Device bytes the solver needs for cfg (0 if cfg is invalid). */
size_t pdvm_workspace_bytes(const pdvm_config *cfg);

/* Validate cfg, preprocess the geometry (per-voxel stencil-order flags,
 * percolation check along x1) and upload it (Sec. 2.3, pre-processing of the
 * (C0, C1, C2) choice). dev_workspace: NULL (the library allocates and frees)
 * or a device buffer of at least pdvm_workspace_bytes(cfg) bytes, owned by the
 * caller, that must outlive the solver (the library still allocates a few KB
 * of launch tables). hip_stream: a hipStream_t, or NULL for a private stream
 * of the library. The initial state is rest (all perturbations zero).
 * PDVM_E_INVAL if no pore component winds around x1. */
int pdvm_create(const pdvm_config *cfg, void *dev_workspace, size_t ws_bytes,
                void *hip_stream, pdvm_solver **out);

/* Initial state: the local linearised equilibrium h = rho + 2 u.v of the
 * given host fields (rho: N doubles, u: dim*N doubles component-major; NULL =
 * zero). Resets the iteration counter. */
int pdvm_set_initial(pdvm_solver *s, const double *rho, const double *u);

/* Run up to max_iters iterations (Algorithm 1). stop_mode PDVM_STOP_FIELD:
 * stop when r <= tol; PDVM_STOP_PAPER_ERR: stop when Err(l) < tol at a
 * multiple of 100 iterations (Eq. convergence_criterion). tol <= 0 runs all
 * max_iters. Returns PDVM_OK (converged), PDVM_NOT_CONVERGED, or an error.
 * PDVM_E_HIP when a row-pipeline sweep was abandoned (a wait for the upstream
 * row exceeded its limit, or the blocks of one velocity chain were found on
 * different XCDs): that iterate is discarded, the state is the last completed
 * iteration, and the solver then returns PDVM_E_STATE from every iterate until
 * pdvm_set_initial or pdvm_set_state restores a state. */
int pdvm_iterate(pdvm_solver *s, int64_t max_iters, double tol, int32_t stop_mode,
                 pdvm_stats *out);

/* pdvm_iterate for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * iterations with the same kernels and results, but no HIP graph is built and
 * no device or pinned memory is allocated; the kernels' scratch (per-block
 * partial sums, the row pipeline's progress counters and XCD records) lives in
 * a static array of the library, 4 MiB per GPU, held until the process ends.
 * PDVM_E_NOMEM if the solve needs more of it (a problem needs at most 32 KiB
 * plus 5 bytes per row-pipeline block: about 0.2 MiB at 16384 voxel rows and
 * 1024 velocities). Calls on one GPU share that array: calls that overlap in
 * time on one GPU (several host threads or streams) race and must not be made.
 * Returns and stats as pdvm_iterate. */
int pdvm_iterate_noalloc(pdvm_solver *s, int64_t max_iters, double tol, int32_t stop_mode,
                         pdvm_stats *out);

/* Macroscopic fields of the current state (Eq. perturbed_quantities), host
 * arrays of N (rho, tau) or dim*N (u, q) doubles, solid voxels read 0; NULL
 * skips. tau and q are diagnostics (2D: reduced forms with v3 integrated
 * out); they are computed from the stored distribution on demand. */
int pdvm_get_moments(pdvm_solver *s, double *rho, double *u, double *tau, double *q);

/* G_p, k = (2/sqrt(pi)) Kn G_p (Eq. k_Gp), and optionally the per-section
 * G_p(i) (n[0] doubles, mean of u1 over the cross-section at x1 index i). */
int pdvm_get_flux(pdvm_solver *s, double *gp, double *k, double *gp_section);

/* Checkpoint: everything the next iteration reads (moments, wall data, the
 * boundary layers of the distribution, counters). With buf == NULL, *bytes
 * receives the size. Restoring into a solver created with the same config
 * continues bitwise identically. A checkpoint of the same problem taken at the
 * other precision is accepted and converted value by value (FP32 -> FP64 is
 * exact), so a run can be continued in FP64 after an FP32 phase.
 * PDVM_E_STATE on a size or problem mismatch. */
int pdvm_get_state(pdvm_solver *s, void *buf, size_t *bytes);
int pdvm_set_state(pdvm_solver *s, const void *buf, size_t bytes);

/* Per-kernel timing on the solver's stream with HIP events, over 2*iters
 * iterations: in the first iters, an event pair brackets every launch, giving
 * the average milliseconds per launch of the sweep kernel, of the moment kernel
 * and of the reduction kernel. In the next iters, events bracket the whole
 * sweep sequence and the whole iteration (sweep_ms_per_iter, iter_ms,
 * including launch gaps). Also returns the number of sweep launches per
 * iteration, and the algorithmic bytes per iteration of the sweep (h written
 * once per fluid voxel and velocity) and of the moment kernel (h read once).
 * Runs real iterations (the state advances). */
typedef struct {
  double sweep_ms_per_launch, moments_ms_per_launch, reduce_ms_per_launch;
  double sweep_ms_per_iter, moments_ms_per_iter, iter_ms;
  int32_t sweep_launches_per_iter;
  double sweep_bytes_per_iter, moments_bytes_per_iter;
  double fluid_cells, velocities;
} pdvm_timing;
int pdvm_time_kernels(pdvm_solver *s, int32_t iters, pdvm_timing *out);

/* ---- Batches ------------------------------------------------------------
 * Many problems (geometries of uneven size, Kn values, jumps, lateral
 * conditions) iterated together: each iteration is one replay of a HIP graph
 * whose sweep launches cover the tiles of every problem on a tile diagonal,
 * followed by one moment launch and one reduction launch over all problems.
 * Problems that reach their stop condition retire: their kernels return at
 * once while the others continue. All configs of a batch share dim,
 * precision, velocity grid, stencil rule and tau feedback (else
 * PDVM_E_INVAL); the library allocates each problem's workspace.
 * The single-problem calls above need a solver of one problem; a batch of
 * one is an ordinary solver. */
int pdvm_batch_create(int32_t n, const pdvm_config *cfgs, void *hip_stream, pdvm_solver **out);
int32_t pdvm_batch_size(const pdvm_solver *s);
int pdvm_batch_set_initial(pdvm_solver *s, int32_t i, const double *rho, const double *u);
/* out: n entries (NULL allowed). Returns PDVM_OK when every problem met the
 * tolerance, PDVM_NOT_CONVERGED if any did not, PDVM_E_NONFINITE if any
 * diverged (its previous state is kept). */
int pdvm_batch_iterate(pdvm_solver *s, int64_t max_iters, double tol, int32_t stop_mode, pdvm_stats *out);
int pdvm_batch_get_moments(pdvm_solver *s, int32_t i, double *rho, double *u, double *tau, double *q);
int pdvm_batch_get_flux(pdvm_solver *s, int32_t i, double *gp, double *k, double *gp_section);

/* The sweep schedule in use: 0 tile diagonals; 1 row pipeline with
 * agent-scope synchronisation; 2 row pipeline with every velocity chain on one
 * XCD (chosen only after a probe of the block placement confirms it); 3 strip
 * pipeline; 4 per-XCD tile queues; 5 per-XCD queues of tile columns; -1 for
 * NULL. */
int32_t pdvm_sweep_schedule(const pdvm_solver *s);

/* Wall-clock bound on each wait of the row-pipeline sweep for its upstream row
 * (default 2 s; seconds in [0, 3600]). A wait that exceeds it abandons the
 * sweep as described at pdvm_iterate; every kernel still runs to its end. For
 * callers that want a tighter bound, and for tests of the fault path (0 gives
 * up at the first check, after 128 polls). PDVM_E_INVAL outside the range. */
int pdvm_set_wait_limit(pdvm_solver *s, double seconds);

void pdvm_destroy(pdvm_solver *s);

/* Last error message of the handle, or of the calling thread if s is NULL. */
const char *pdvm_last_error(const pdvm_solver *s);

#ifdef __cplusplus
}
#endif
#endif /* POREDVM_H */
