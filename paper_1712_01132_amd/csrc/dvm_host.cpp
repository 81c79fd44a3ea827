// Host side of libporedvm: the C ABI of include/poredvm.h.
//
//  * validation and one-time preprocessing of the voxel image (per-voxel
//    stencil-order flags, percolation along x1) -- the paper's pre-processing
//    of the stencil coefficients (Sec. 2.3);
//  * the half-range Gauss-Hermite velocity grid (Sec. 2.2);
//  * device layout, upload and the iteration driver (Sec. 3.1, Algorithm 1):
//    one iteration = the sweep over all tile diagonals, the moment kernel and
//    the FP64 reduction, captured once as a HIP graph and replayed; the host
//    polls a 16-byte status every few iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/poredvm.h"
#include "dvm_internal.h"

using namespace pdvm;

// Static device scratch of pdvm_iterate_noalloc (callers that cannot
// allocate): the moment kernel's per-block partial sums, the row pipeline's
// progress counters and XCD records, for one solve at a time per GPU. Each GPU
// holds its own copy until the process ends. The array's name is a host-side
// stand-in, not a device address: host code uses only the address that
// hipGetSymbolAddress returns for the current device (scratch_address).
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_thread_error;

// The device address of `scratch` on device `dev` (that device current), taken
// once per device; the result (address or error) is kept for later calls.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
bool g_scratch_done[kMaxDevices];

hipError_t scratch_address(int dev, void **out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_err[dev] = e;
    g_scratch_ptr[dev] = e == hipSuccess ? ptr : nullptr;
    g_scratch_done[dev] = true;
  }
  *out = g_scratch_ptr[dev];
  return g_scratch_err[dev];
}

void set_thread_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_thread_error = buf;
}

// ---------------------------------------------------------------------------
// Half-range Gauss-Hermite rule in extended precision: the recurrence of the
// orthogonal polynomials for exp(-x^2) on [0, inf) by the discretised
// Stieltjes procedure (composite Gauss-Legendre on [0, 14]); the nodes are
// the eigenvalues of the recurrence's Jacobi matrix (Golub-Welsch), the
// weights the Christoffel numbers 1 / sum_j p_j(x)^2 of the orthonormal
// polynomials at each node (a sum of positive terms: full relative accuracy
// also for the smallest weights).

// Eigenvalues of the symmetric tridiagonal matrix with diagonal `diag` and
// off-diagonal `off` (off[i] couples i and i + 1), by cyclic Jacobi
// rotations on the dense matrix: each rotation in the (p, q) plane makes the
// (p, q) entry zero, with the tangent of the smaller rotation angle taken
// from tau = (a_qq - a_pp) / (2 a_pq), t = sign(tau) / (|tau| + sqrt(1 +
// tau^2)). Sweeps over all pairs repeat until the off-diagonal mass is at
// rounding level (quadratic convergence; the matrices here have at most 32
// rows).
bool symtri_eigen(const std::vector<long double> &diag, const std::vector<long double> &off,
                  std::vector<long double> &val) {
  const int n = (int)diag.size();
  std::vector<long double> A((size_t)n * n, 0);
  auto at = [&A, n](int r, int c) -> long double & { return A[(size_t)r * n + c]; };
  for (int i = 0; i < n; ++i) at(i, i) = diag[i];
  for (int i = 0; i + 1 < n; ++i) at(i, i + 1) = at(i + 1, i) = off[i];
  bool done = false;
  for (int sweep = 0; sweep < 60 && !done; ++sweep) {
    long double offd = 0, all = 0;
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) {
        const long double a2 = at(r, c) * at(r, c);
        all += a2;
        if (r != c) offd += a2;
      }
    if (offd <= 1e-36L * all) {
      done = true;
      break;
    }
    for (int p = 0; p + 1 < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const long double apq = at(p, q);
        if (fabsl(apq) <= 1e-24L * (fabsl(at(p, p)) + fabsl(at(q, q)))) {
          at(p, q) = at(q, p) = 0;
          continue;
        }
        const long double tau = (at(q, q) - at(p, p)) / (2 * apq);
        const long double t = (tau >= 0 ? 1.0L : -1.0L) / (fabsl(tau) + sqrtl(1 + tau * tau));
        const long double c = 1 / sqrtl(1 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A J
          const long double akp = at(k, p), akq = at(k, q);
          at(k, p) = c * akp - s * akq;
          at(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^T A
          const long double apk = at(p, k), aqk = at(q, k);
          at(p, k) = c * apk - s * aqk;
          at(q, k) = s * apk + c * aqk;
        }
        at(p, q) = at(q, p) = 0;  // zero by construction; drop the rounding
      }
  }
  if (!done) return false;
  val.assign(n, 0);
  for (int k = 0; k < n; ++k) val[k] = at(k, k);
  return true;
}

// Gauss rule of the three-term recurrence with diagonal `diag`, off-diagonal
// `off` (the square roots of beta_1 ..) and weight-function mass `mass`.
bool gauss_rule(const std::vector<long double> &diag, const std::vector<long double> &off, long double mass,
                std::vector<long double> &x, std::vector<long double> &w) {
  const int n = (int)diag.size();
  if (!symtri_eigen(diag, off, x)) return false;
  w.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    long double pm = 0, pc = 1 / sqrtl(mass), sum = pc * pc;  // p_{j-1}, p_j at x_i
    for (int j = 0; j + 1 < n; ++j) {
      const long double pn = ((x[i] - diag[j]) * pc - (j > 0 ? off[j - 1] * pm : 0)) / off[j];
      pm = pc;
      pc = pn;
      sum += pc * pc;
    }
    w[i] = 1 / sum;
  }
  return true;
}

// m-point Gauss-Legendre rule on [-1, 1]: zero diagonal, off-diagonal
// k / sqrt(4 k^2 - 1), mass 2.
bool gauss_legendre(int m, std::vector<long double> &x, std::vector<long double> &w) {
  std::vector<long double> diag(m, 0), off(m > 1 ? m - 1 : 0);
  for (int k = 1; k < m; ++k) off[k - 1] = k / sqrtl(4.0L * k * k - 1);
  return gauss_rule(diag, off, 2.0L, x, w);
}

// ---------------------------------------------------------------------------
// Percolation along x1: union-find over fluid voxels with the period offset of
// each voxel relative to its root; a component winds around x1 when an edge
// closes a cycle whose offsets disagree.

struct PeriodicUF {
  std::vector<int64_t> parent;
  std::vector<int32_t> off;
  std::vector<uint8_t> winds;
  explicit PeriodicUF(int64_t n) : parent(n), off(n, 0), winds(n, 0) {
    for (int64_t i = 0; i < n; ++i) parent[i] = i;
  }
  int64_t find(int64_t a, int32_t &oa) {
    int32_t acc = 0;
    int64_t r = a;
    while (parent[r] != r) {
      acc += off[r];
      r = parent[r];
    }
    // path compression with offsets
    int32_t rem = acc;
    int64_t c = a;
    while (parent[c] != c) {
      const int64_t nxt = parent[c];
      const int32_t o = off[c];
      parent[c] = r;
      off[c] = rem;
      rem -= o;
      c = nxt;
    }
    oa = acc;
    return r;
  }
  // b's lifted position = a's + d periods
  void unite(int64_t a, int64_t b, int32_t d) {
    int32_t oa, ob;
    const int64_t ra = find(a, oa), rb = find(b, ob);
    if (ra != rb) {
      parent[rb] = ra;
      off[rb] = oa + d - ob;
      winds[ra] |= winds[rb];
    } else if (ob != oa + d) {
      winds[ra] = 1;
    }
  }
};

// ---------------------------------------------------------------------------

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <typename T>
struct Layout {
  size_t ctl, flags, absv, av, vsqm, rden, wq, h[2], src[2], srct[2], srcq[2], wall[2], rho[2], u[2], part, tiles, offs, fidx,
      scratch,
      progress, total;
};

struct Problem {
  int dim = 2;
  int n[3] = {1, 1, 1};
  int64_t N = 0, fluid = 0;
  int hv[3] = {1, 1, 1};      // positive half-node counts
  int Ko = 0, Ko_pad = 0, Kpad = 0, ngroups = 0;
  int tile[3] = {1, 1, 1}, ntile[3] = {1, 1, 1};
  int ndiag = 0;
  int mom_blocks = 0;
  double nu = 0, kn = 0, jump = 1, D[3] = {0, 0, 0};
  int lateral_periodic = 0, tau_fb = 0, precision = 0, check_every = 16, stencil_rule = 1;
  int schedule = 0;  // sweep schedule requested (PDVM_SCHEDULE_*)
  std::vector<uint32_t> flags;
  int psi = 0;       // 2D with tau feedback: octant slots [Ko/2, Ko) hold psi
  double prandtl = 0;  // > 0: Shakhov model
  double spec = 0;     // > 0: Maxwell walls, 1 - alpha
  std::vector<double> absv, wq, vsqm, rden;   // host FP64 tables, [rows][Ko_pad]
  std::vector<int32_t> diag_tiles, diag_off;
  std::vector<uint8_t> live;  // per tile (x1 fastest): holds a fluid voxel
  std::vector<int32_t> fluid_idx;  // fluid voxels in index order
  uint64_t fingerprint = 0;  // hash of everything that defines the problem
};

uint64_t fnv1a(uint64_t h, const void *data, size_t n) {
  const unsigned char *p = (const unsigned char *)data;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

int validate_and_build(const pdvm_config *cfg, Problem &P, std::string &err) {
  if (!cfg) { err = "config is NULL"; return PDVM_E_INVAL; }
  if (cfg->dim != 2 && cfg->dim != 3) { err = "dim must be 2 or 3"; return PDVM_E_INVAL; }
  P.dim = cfg->dim;
  for (int a = 0; a < 3; ++a) {
    P.n[a] = a < P.dim ? cfg->n[a] : 1;
    if (a < P.dim && (P.n[a] < 2 || P.n[a] > (1 << 20))) { err = "each n[a] must be in [2, 2^20]"; return PDVM_E_INVAL; }
  }
  P.N = (int64_t)P.n[0] * P.n[1] * P.n[2];
  if (P.N * 6 >= ((int64_t)1 << 31)) { err = "at most 2^31/6 voxels per problem"; return PDVM_E_INVAL; }
  if (!cfg->solid) { err = "solid mask is NULL"; return PDVM_E_INVAL; }
  if (!(cfg->kn > 0)) { err = "kn must be > 0 (or +inf)"; return PDVM_E_INVAL; }
  if (!std::isfinite(cfg->jump)) { err = "jump must be finite"; return PDVM_E_INVAL; }
  if (cfg->precision != PDVM_FP64 && cfg->precision != PDVM_FP32) { err = "precision must be FP64 or FP32"; return PDVM_E_INVAL; }
  if (cfg->lateral_bc != PDVM_LATERAL_SPECULAR && cfg->lateral_bc != PDVM_LATERAL_PERIODIC) { err = "bad lateral_bc"; return PDVM_E_INVAL; }
  P.kn = cfg->kn;
  P.nu = std::isinf(cfg->kn) ? 0.0 : std::sqrt(M_PI) / (2.0 * cfg->kn);
  P.jump = cfg->jump;
  P.precision = cfg->precision;
  P.lateral_periodic = cfg->lateral_bc == PDVM_LATERAL_PERIODIC;
  P.tau_fb = cfg->tau_feedback ? 1 : 0;
  P.psi = P.dim == 2 && P.tau_fb;
  if (!(cfg->prandtl >= 0) || !std::isfinite(cfg->prandtl)) { err = "prandtl must be >= 0 and finite"; return PDVM_E_INVAL; }
  if (cfg->prandtl > 0 && !P.tau_fb) { err = "the Shakhov model (prandtl > 0) needs tau_feedback"; return PDVM_E_INVAL; }
  P.prandtl = cfg->prandtl;
  if (!(cfg->specular_fraction >= 0 && cfg->specular_fraction < 1)) {
    err = "specular_fraction (1 - alpha) must be in [0, 1)";
    return PDVM_E_INVAL;
  }
  P.spec = cfg->specular_fraction;
  P.check_every = cfg->check_every > 0 ? cfg->check_every : 16;
  if (cfg->sweep_schedule < 0 || cfg->sweep_schedule > 6) { err = "sweep_schedule must be 0..6"; return PDVM_E_INVAL; }
  P.schedule = cfg->sweep_schedule;
  if ((P.schedule == PDVM_SCHEDULE_ROWS || P.schedule == PDVM_SCHEDULE_ROWS_AGENT ||
       P.schedule == PDVM_SCHEDULE_STRIPS) && cfg->dim != 2) {
    err = "the row-pipeline sweep is 2D only";
    return PDVM_E_UNSUPPORTED;
  }
  if (P.schedule == PDVM_SCHEDULE_COLUMNS && cfg->dim != 3) {
    err = "the column-queue sweep is 3D only";
    return PDVM_E_UNSUPPORTED;
  }
  if (cfg->stencil_rule != 0 && cfg->stencil_rule != 1) { err = "stencil_rule must be 0 or 1"; return PDVM_E_INVAL; }
  if (P.spec > 0 && cfg->stencil_rule != 1) { err = "Maxwell walls (specular_fraction > 0) need stencil_rule 1"; return PDVM_E_UNSUPPORTED; }
  P.stencil_rule = cfg->stencil_rule;

  // velocity grid: per axis, symmetric, even, no zero node, weights > 0, sum 1
  std::vector<double> xp[3], wp[3];
  for (int a = 0; a < 3; ++a) {
    if (a >= P.dim) { xp[a] = {0.0}; wp[a] = {1.0}; P.hv[a] = 1; continue; }
    const int m = cfg->nv[a];
    if (m < 2 || m % 2 || m > 512) { err = "nv[a] must be even in [2, 512]"; return PDVM_E_INVAL; }
    if (!cfg->vnode[a] || !cfg->vweight[a]) { err = "velocity node/weight array is NULL"; return PDVM_E_INVAL; }
    const double *x = cfg->vnode[a], *w = cfg->vweight[a];
    double sw = 0;
    for (int i = 0; i < m; ++i) {
      if (!(w[i] > 0) || !std::isfinite(x[i])) { err = "weights must be > 0 and nodes finite"; return PDVM_E_INVAL; }
      if (i > 0 && !(x[i] > x[i - 1])) { err = "nodes must be strictly ascending"; return PDVM_E_INVAL; }
      sw += w[i];
    }
    if (std::fabs(sw - 1.0) > 1e-12) { err = "weights of each axis must sum to 1"; return PDVM_E_INVAL; }
    for (int i = 0; i < m / 2; ++i) {
      const double xl = x[i], xr = x[m - 1 - i];
      if (std::fabs(xl + xr) > 1e-13 * std::max(1.0, std::fabs(xr)) ||
          std::fabs(w[i] - w[m - 1 - i]) > 1e-13 * w[i]) {
        err = "velocity grid must be symmetric about 0";
        return PDVM_E_INVAL;
      }
    }
    if (!(x[m / 2] > 0)) { err = "velocity grid must not contain 0"; return PDVM_E_INVAL; }
    P.hv[a] = m / 2;
    for (int i = 0; i < m / 2; ++i) { xp[a].push_back(x[m / 2 + i]); wp[a].push_back(w[m / 2 + i]); }
  }
  // velocities per sign octant; in 2D with the temperature fed back, each
  // velocity also carries the second reduced function psi, in slot Kv + q
  const int Kv = P.hv[0] * P.hv[1] * P.hv[2];
  P.Ko = P.psi ? 2 * Kv : Kv;
  if (P.Ko > 16 * kWave) {
    err = P.psi ? "at most 512 velocities per sign octant in 2D with tau feedback (psi doubles them)"
                : "at most 1024 velocities per sign octant";
    return PDVM_E_INVAL;
  }
  const int elem = P.precision == PDVM_FP64 ? 8 : 4;
  const int line = 128 / elem;
  P.Ko_pad = (P.Ko + line - 1) / line * line;
  P.Kpad = P.Ko_pad << P.dim;
  P.ngroups = (P.Ko + kWave - 1) / kWave;
  // the sweeps store a row of h (all voxels along x1) through one buffer resource
  if ((int64_t)P.n[0] * P.Kpad * elem >= ((int64_t)1 << 30)) {
    err = "a row of voxels along x1 may hold at most 1 GiB of the distribution";
    return PDVM_E_INVAL;
  }

  // per-slot tables of one octant (slot q <-> positive node indices p_j)
  const double dx_inv = (double)P.n[0];
  P.absv.assign(3 * (size_t)P.Ko_pad, 0.0);
  P.wq.assign(8 * (size_t)P.Ko_pad, 0.0);
  // row 0: temperature-source factor, row 1: 1 = h, 0 = psi, row 2: heat-flux source factor
  P.vsqm.assign(3 * (size_t)P.Ko_pad, 0.0);
  P.rden.assign(8 * (size_t)P.Ko_pad, 0.0);
  for (int q = 0; q < P.Ko; ++q) {
    const int qv = q % Kv;
    const bool ps = q >= Kv;  // a psi slot
    const int p[3] = {qv % P.hv[0], (qv / P.hv[0]) % P.hv[1], qv / (P.hv[0] * P.hv[1])};
    double W = 1, vsq = 0;
    for (int j = 0; j < 3; ++j) {
      W *= wp[j][p[j]];
      if (j < P.dim) { P.absv[j * P.Ko_pad + q] = xp[j][p[j]]; vsq += xp[j][p[j]] * xp[j][p[j]]; }
    }
    // moment weights: psi enters only the energy, as int (v3^2 - 1/2) h = psi
    P.wq[q] = ps ? 0.0 : W;
    for (int j = 0; j < P.dim; ++j) P.wq[(1 + j) * P.Ko_pad + q] = ps ? 0.0 : W * xp[j][p[j]];
    // |v|^2 weight row (2D: the reduced distribution adds <v3^2> = 1/2)
    P.wq[(1 + P.dim) * P.Ko_pad + q] = ps ? W : W * (vsq + (P.dim == 2 ? 0.5 : 0.0));
    // temperature source factor: |v|^2 - 3/2, integrated over v3 in 2D
    // (v1^2 + v2^2 - 1); psi's source is tau / 2
    P.vsqm[q] = ps ? 0.5 : vsq - (P.dim == 2 ? 1.0 : 1.5);
    P.vsqm[P.Ko_pad + q] = ps ? 0.0 : 1.0;
    // Shakhov: the source's q.v factor |v|^2 - 5/2, integrated over v3 in 2D
    // (v1^2 + v2^2 - 2 for h, 1/2 for psi); q's weights W |v_j| (|v|^2 - 5/2)
    // (2D: v1^2 + v2^2 - 2 for h, 1 for psi)
    const double qs = ps ? 0.5 : vsq - (P.dim == 2 ? 2.0 : 2.5);
    const double qw = ps ? 1.0 : vsq - (P.dim == 2 ? 2.0 : 2.5);
    P.vsqm[2 * P.Ko_pad + q] = qs;
    for (int j = 0; j < P.dim; ++j) P.wq[(5 + j) * P.Ko_pad + q] = W * xp[j][p[j]] * qw;
    for (int combo = 0; combo < (1 << P.dim); ++combo) {
      double den = P.nu;
      for (int j = 0; j < P.dim; ++j) den += xp[j][p[j]] * dx_inv * (((combo >> j) & 1) ? 1.0 : 1.5);
      P.rden[combo * P.Ko_pad + q] = 1.0 / den;
    }
  }
  // D_j = sum over all velocities with v_j > 0 of W v_j (2^(dim-1) octants)
  for (int j = 0; j < P.dim; ++j) {
    double d = 0;
    for (int q = 0; q < P.Ko; ++q) d += P.wq[(1 + j) * P.Ko_pad + q];
    P.D[j] = d * (double)(1 << (P.dim - 1));
  }

  // geometry: flags and percolation
  const uint8_t *sm = cfg->solid;
  P.flags.assign(P.N, 0);
  auto is_solid = [&](int x, int y, int z) { return sm[x + (int64_t)P.n[0] * (y + (int64_t)P.n[1] * z)] != 0; };
  auto image = [&](int j, int c) {
    if (j == 0) return c < 0 ? c + P.n[0] : c - P.n[0];
    if (P.lateral_periodic) return c < 0 ? c + P.n[j] : c - P.n[j];
    return c < 0 ? -c - 1 : 2 * P.n[j] - 1 - c;
  };
  int64_t fluid = 0;
  for (int z = 0; z < P.n[2]; ++z)
    for (int y = 0; y < P.n[1]; ++y)
      for (int x = 0; x < P.n[0]; ++x) {
        const int64_t c = x + (int64_t)P.n[0] * (y + (int64_t)P.n[1] * z);
        if (sm[c]) { P.flags[c] = F_SOLID; continue; }
        ++fluid;
        uint32_t f = 0;
        for (int j = 0; j < P.dim; ++j)
          for (int si = 0; si < 2; ++si) {
            const int s = si ? -1 : 1;
            bool sol[3] = {false, false, false};
            for (int m = 1; m <= 2; ++m) {
              int cc[3] = {x, y, z};
              cc[j] -= m * s;
              if (cc[j] < 0 || cc[j] >= P.n[j]) cc[j] = image(j, cc[j]);
              sol[m] = is_solid(cc[0], cc[1], cc[2]);
            }
            const bool first = sol[1] || (P.stencil_rule == 1 && sol[2]);
            if (first) f |= f_first(j, si);
            if (sol[1]) f |= f_y1s(j, si);
            if (!first && sol[2]) f |= f_y2s(j, si);
          }
        P.flags[c] = f;
      }
  P.fluid = fluid;
  P.fluid_idx.clear();
  P.fluid_idx.reserve((size_t)fluid);
  for (int64_t c = 0; c < P.N; ++c)
    if (!(P.flags[c] & F_SOLID)) P.fluid_idx.push_back((int32_t)c);
  if (fluid == 0) { err = "the geometry has no fluid voxel"; return PDVM_E_INVAL; }
  {
    PeriodicUF uf(P.N);
    for (int z = 0; z < P.n[2]; ++z)
      for (int y = 0; y < P.n[1]; ++y)
        for (int x = 0; x < P.n[0]; ++x) {
          const int64_t c = x + (int64_t)P.n[0] * (y + (int64_t)P.n[1] * z);
          if (sm[c]) continue;
          const int xn = x + 1 < P.n[0] ? x + 1 : 0;
          const int64_t cx = xn + (int64_t)P.n[0] * (y + (int64_t)P.n[1] * z);
          if (!sm[cx]) uf.unite(c, cx, x + 1 < P.n[0] ? 0 : 1);
          if (y + 1 < P.n[1]) {
            const int64_t cy = c + P.n[0];
            if (!sm[cy]) uf.unite(c, cy, 0);
          }
          if (z + 1 < P.n[2]) {
            const int64_t cz = c + (int64_t)P.n[0] * P.n[1];
            if (!sm[cz]) uf.unite(c, cz, 0);
          }
        }
    bool any = false;
    for (int64_t c = 0; c < P.N && !any; ++c) {
      if (sm[c]) continue;
      int32_t o;
      const int64_t r = uf.find(c, o);
      any = uf.winds[r] != 0;
    }
    if (!any) { err = "no pore component winds around x1 (no flow path)"; return PDVM_E_INVAL; }
  }

  // sweep tiles and their diagonals (oriented tile coordinates sum to d)
  {
    // (x1, x2): at most the compiled edge (4 or 8) that covers both requested
    // extents (default 8 x 8); x3: any depth
    const int r0 = cfg->tile[0] > 0 ? cfg->tile[0] : 8, r1 = cfg->tile[1] > 0 ? cfg->tile[1] : r0;
    const int e = std::max(r0, r1) <= kTileEdge[0] ? kTileEdge[0] : kTileEdge[1];
    for (int a = 0; a < 3; ++a) {
      int t = 1;
      if (a < 2) t = std::min(a == 0 ? r0 : r1, e);
      else if (P.dim == 3) t = cfg->tile[2] > 0 ? cfg->tile[2] : 8;
      P.tile[a] = std::max(1, std::min(t, P.n[a]));
      P.ntile[a] = (P.n[a] + P.tile[a] - 1) / P.tile[a];
    }
  }
  P.ndiag = P.ntile[0] + P.ntile[1] + P.ntile[2] - 2;
  P.live.assign((size_t)P.ntile[0] * P.ntile[1] * P.ntile[2], 0);
  for (int64_t c = 0; c < P.N; ++c) {
    if (P.flags[c] & F_SOLID) continue;
    const int64_t x = c % P.n[0], y = (c / P.n[0]) % P.n[1], z = c / ((int64_t)P.n[0] * P.n[1]);
    P.live[(x / P.tile[0]) + P.ntile[0] * ((y / P.tile[1]) + (size_t)P.ntile[1] * (z / P.tile[2]))] = 1;
  }
  std::vector<std::vector<int32_t>> per;
  if (P.dim == 2) {
    per.resize(P.ndiag);
    for (int b = 0; b < P.ntile[1]; ++b)
      for (int a = 0; a < P.ntile[0]; ++a) {
        auto &v = per[a + b];
        v.push_back(a); v.push_back(b); v.push_back(0); v.push_back(0);
      }
  } else {
    // 3D: one list per diagonal and sign octant of the physical tiles that
    // hold a fluid voxel (the sweep does nothing in an all-solid tile, whose
    // voxels keep their values); the octant's walk order sets which physical
    // tile sits at oriented coordinates (a, b, c)
    const std::vector<uint8_t> &live = P.live;
    per.resize((size_t)P.ndiag * 8);
    for (int c = 0; c < P.ntile[2]; ++c)
      for (int b = 0; b < P.ntile[1]; ++b)
        for (int a = 0; a < P.ntile[0]; ++a)
          for (int o = 0; o < 8; ++o) {
            const int pa = (o & 1) ? P.ntile[0] - 1 - a : a, pb = (o & 2) ? P.ntile[1] - 1 - b : b,
                      pc = (o & 4) ? P.ntile[2] - 1 - c : c;
            if (!live[pa + P.ntile[0] * (pb + (size_t)P.ntile[1] * pc)]) continue;
            auto &v = per[(size_t)(a + b + c) * 8 + o];
            v.push_back(pa); v.push_back(pb); v.push_back(pc); v.push_back(0);
          }
  }
  P.diag_off.assign(1, 0);
  for (auto &v : per) {
    P.diag_tiles.insert(P.diag_tiles.end(), v.begin(), v.end());
    P.diag_off.push_back((int32_t)(P.diag_tiles.size() / 4));
  }
  // moment kernel: about 16 fluid voxels per wavefront, at most one round of 4096 wavefronts
  P.mom_blocks = (int)std::max<int64_t>(1, std::min<int64_t>((P.fluid + 63) / 64, 1024));
  uint64_t fp = 1469598103934665603ull;
  const double scal[7] = {P.kn, P.jump, (double)P.lateral_periodic, (double)P.tau_fb, (double)P.stencil_rule, P.prandtl,
                          P.spec};
  fp = fnv1a(fp, scal, sizeof(scal));
  fp = fnv1a(fp, P.n, sizeof(P.n));
  fp = fnv1a(fp, P.hv, sizeof(P.hv));
  fp = fnv1a(fp, P.flags.data(), P.flags.size() * 4);
  // the velocity tables without their padding slots, which depend on the precision
  for (size_t r = 0; r < P.absv.size() / P.Ko_pad; ++r) fp = fnv1a(fp, &P.absv[r * P.Ko_pad], (size_t)P.Ko * 8);
  for (size_t r = 0; r < P.wq.size() / P.Ko_pad; ++r) fp = fnv1a(fp, &P.wq[r * P.Ko_pad], (size_t)P.Ko * 8);
  P.fingerprint = fp;
  return PDVM_OK;
}

template <typename T>
Layout<T> make_layout(const Problem &P) {
  Layout<T> L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o += align256(bytes); return at; };
  const size_t N = (size_t)P.N;
  L.ctl = take(sizeof(Ctl));
  L.flags = take(N * 4);
  L.absv = take(3 * (size_t)P.Ko_pad * sizeof(T));
  L.av = take(3 * (size_t)P.Ko_pad * sizeof(T));
  L.vsqm = take(3 * (size_t)P.Ko_pad * sizeof(T));
  L.rden = take(8 * (size_t)P.Ko_pad * sizeof(T));
  L.wq = take(8 * (size_t)P.Ko_pad * 8);
  for (int b = 0; b < 2; ++b) {
    L.h[b] = take(N * (size_t)P.Kpad * sizeof(T));
    L.src[b] = take(N * kSrcStride * sizeof(T));
    L.srct[b] = take(N * sizeof(T));
    L.srcq[b] = take(P.prandtl > 0 ? N * 4 * sizeof(T) : 0);
    L.wall[b] = take(N * 6 * sizeof(T));
    L.rho[b] = take(N * 8);
    L.u[b] = take(3 * N * 8);
  }
  L.part = take((size_t)P.mom_blocks * 4 * 8);
  L.tiles = take(P.diag_tiles.size() * 4);
  L.offs = take(P.diag_off.size() * 4);
  L.fidx = take((size_t)P.fluid * 4);
  L.scratch = take(8 * N * 8);  // tau, q (3), rho, u (3) staging
  // pipeline counters: at most one per (band, chain rounded up to 8) of the
  // row pipeline or the strips
  L.progress = take((size_t)(P.n[1] + 8) * (((P.ngroups << P.dim) + 7) / 8 * 8) * 4);
  L.total = o;
  return L;
}

size_t layout_bytes(const Problem &P) {
  return P.precision == PDVM_FP64 ? make_layout<double>(P).total : make_layout<float>(P).total;
}

int halfrange_gh(int32_t n_total, double *nodes, double *weights) {
  if (n_total < 2 || n_total % 2 || n_total > 64 || !nodes || !weights) {
    set_thread_error("n_total must be even in [2, 64] and outputs non-NULL");
    return PDVM_E_INVAL;
  }
  const int n = n_total / 2;
  // discretise int_0^14 f(x) exp(-x^2) dx by composite Gauss-Legendre
  std::vector<long double> gx, gw;
  if (!gauss_legendre(24, gx, gw)) {
    set_thread_error("eigenvalue iteration did not converge");
    return PDVM_E_INVAL;
  }
  const int panels = 96;
  const long double X = 14.0L, hp = X / panels;
  std::vector<long double> x, w;
  for (int p = 0; p < panels; ++p)
    for (size_t i = 0; i < gx.size(); ++i) {
      const long double t = hp * (p + 0.5L * (gx[i] + 1));
      x.push_back(t);
      w.push_back(0.5L * hp * gw[i] * expl(-t * t));
    }
  // Stieltjes procedure for the recurrence coefficients
  std::vector<long double> alpha(n), beta(n), p0(x.size(), 0), p1(x.size(), 1), p2(x.size());
  long double norm_prev = 1;
  for (int k = 0; k < n; ++k) {
    long double nrm = 0, xn = 0;
    for (size_t i = 0; i < x.size(); ++i) {
      nrm += w[i] * p1[i] * p1[i];
      xn += w[i] * x[i] * p1[i] * p1[i];
    }
    alpha[k] = xn / nrm;
    beta[k] = k == 0 ? nrm : nrm / norm_prev;
    norm_prev = nrm;
    for (size_t i = 0; i < x.size(); ++i) {
      p2[i] = (x[i] - alpha[k]) * p1[i] - (k == 0 ? 0 : beta[k]) * p0[i];
      p0[i] = p1[i];
      p1[i] = p2[i];
    }
  }
  std::vector<long double> off(n > 1 ? n - 1 : 0), d, z;
  for (int i = 0; i + 1 < n; ++i) off[i] = sqrtl(beta[i + 1]);
  if (!gauss_rule(alpha, off, beta[0], d, z)) {
    set_thread_error("eigenvalue iteration did not converge");
    return PDVM_E_INVAL;
  }
  std::vector<std::pair<long double, long double>> nw(n);
  long double tot = 0;
  for (int i = 0; i < n; ++i) {
    nw[i] = {d[i], z[i]};
    tot += nw[i].second;
  }
  std::sort(nw.begin(), nw.end());
  for (int i = 0; i < n; ++i) {
    nodes[n + i] = (double)nw[i].first;
    nodes[n - 1 - i] = -(double)nw[i].first;
    weights[n + i] = (double)(nw[i].second / (2 * tot));
    weights[n - 1 - i] = weights[n + i];
  }
  return PDVM_OK;
}

}  // namespace

// One or more problems driven together (a single problem is a batch of one).
struct ProbDev {
  char *ws = nullptr;
  bool own_ws = false;
  size_t bytes = 0;
  double *scratch = nullptr;
};

struct pdvm_solver {
  std::vector<Problem> P;
  std::vector<ProbDev> D;
  std::vector<Geo<double>> gd;
  std::vector<Geo<float>> gf;
  int precision = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  char *meta = nullptr;            // device: descriptors, offset tables, gathered control blocks
  Ctl *d_ctl_all = nullptr;
  std::vector<int> h_item_off, h_blk_off, h_row_off, h_strip_off;
  Batch<double> bd;
  Batch<float> bf;
  Ctl *host_ctl = nullptr;         // pinned, one per problem
  uint8_t *d_xcc = nullptr;        // device: the XCD of every row-pipeline block (in meta)
  // pdvm_iterate_noalloc: this GPU's static scratch (null if its address could
  // not be taken: scratch_err), the regions the batch needs in it, and room for
  // the per-problem start counters (sized at creation)
  char *scratch_dev = nullptr;
  hipError_t scratch_err = hipSuccess;
  size_t scr_part = 0, scr_prog = 0, scr_xcc = 0, scr_qctr = 0, scr_qflags = 0, scr_need = 0;
  std::vector<int64_t> start_iters;
  hipGraphExec_t graph = nullptr;
  int graph_iters = 0;
  bool rows = false;               // the sweep is one row-pipeline launch (2D, single problem)
  bool rows_local = false;         // ... whose chains each run on one XCD (probed)
  bool strips = false;             // the sweep is one strip-pipeline launch (2D; XCD-local placement probed)
  bool queue = false;              // the sweep is one launch fed by per-XCD tile queues
  bool columns = false;            // ... whose items are columns of tiles along x3 (3D)
  char *qmem = nullptr;            // device: queue items, offsets, counters, done flags
  size_t qflag_ints = 0;           // done flags of the whole batch
  std::string err;
  int n() const { return (int)P.size(); }
  int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    err = buf;
    g_thread_error = buf;
    return code;
  }
};

#define HIPCHK(s, call)                                                                       \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return (s)->fail(PDVM_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

namespace {

template <typename T>
std::vector<Geo<T>> &geos(pdvm_solver *s);
template <>
std::vector<Geo<double>> &geos<double>(pdvm_solver *s) { return s->gd; }
template <>
std::vector<Geo<float>> &geos<float>(pdvm_solver *s) { return s->gf; }
template <typename T>
Batch<T> &batch(pdvm_solver *s);
template <>
Batch<double> &batch<double>(pdvm_solver *s) { return s->bd; }
template <>
Batch<float> &batch<float>(pdvm_solver *s) { return s->bf; }

// Carve problem i's workspace, upload its tables and geometry, rest state.
template <typename T>
int setup_problem(pdvm_solver *s, int i) {
  const Problem &P = s->P[i];
  const Layout<T> L = make_layout<T>(P);
  Geo<T> g{};
  char *b = s->D[i].ws;
  g.dim = P.dim;
  for (int a = 0; a < 3; ++a) { g.n[a] = P.n[a]; g.tile[a] = P.tile[a]; g.ntile[a] = P.ntile[a]; }
  g.N = P.N;
  g.Ko = P.Ko; g.Ko_pad = P.Ko_pad; g.Kpad = P.Kpad; g.ngroups = P.ngroups;
  g.lateral_periodic = P.lateral_periodic;
  g.tau_fb = P.tau_fb;
  g.y2wall = P.stencil_rule == 0;
  g.dev = P.spec > 0 ? 0 : 1;
  g.jump = g.dev ? T(0) : T(P.jump);
  g.ramp = P.jump;
  {
    double w0 = 0, we = 0;
    for (int q = 0; q < P.Ko; ++q)
      if (P.vsqm[P.Ko_pad + q] != 0.0) {  // a slot of h (not psi)
        w0 += P.wq[q];
        we += P.wq[(1 + P.dim) * P.Ko_pad + q];
      }
    g.w0 = w0 * (double)(1 << P.dim);
    g.we = we * (double)(1 << P.dim);
  }
  g.nu = P.nu;
  for (int j = 0; j < 3; ++j) g.D[j] = P.D[j] > 0 ? P.D[j] : 1.0;
  g.ctl = (Ctl *)(b + L.ctl);
  g.flags = (const uint32_t *)(b + L.flags);
  g.absv = (const T *)(b + L.absv);
  g.av = (const T *)(b + L.av);
  g.vsqm = (const T *)(b + L.vsqm);
  g.phm = g.vsqm + P.Ko_pad;
  g.qsf = g.vsqm + 2 * P.Ko_pad;
  g.psi = P.psi;
  g.shakhov = P.prandtl > 0;
  g.sh_coef = P.prandtl > 0 ? 0.8 * (1.0 - P.prandtl) : 0.0;
  g.maxwell = P.spec > 0;
  g.spec = T(P.spec);
  g.alpha = T(1.0 - P.spec);
  g.rden = (const T *)(b + L.rden);
  g.wq = (const double *)(b + L.wq);
  for (int k = 0; k < 2; ++k) {
    g.h[k] = (T *)(b + L.h[k]);
    g.src[k] = (T *)(b + L.src[k]);
    g.srct[k] = (T *)(b + L.srct[k]);
    g.srcq[k] = P.prandtl > 0 ? (T *)(b + L.srcq[k]) : nullptr;
    g.wall[k] = (T *)(b + L.wall[k]);
    g.rho[k] = (double *)(b + L.rho[k]);
    g.u[k] = (double *)(b + L.u[k]);
  }
  g.part = (double *)(b + L.part);
  g.mom_blocks = P.mom_blocks;
  g.diag_tiles = (const int32_t *)(b + L.tiles);
  g.diag_off = (const int32_t *)(b + L.offs);
  g.fluid_idx = (const int32_t *)(b + L.fidx);
  g.nfluid = P.fluid;
  g.ndiag = P.ndiag;
  g.progress = (int32_t *)(b + L.progress);
  {
    int khz = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
        khz <= 0)
      khz = 100000;  // the 100 MHz of CDNA parts
    g.wait_ticks = (int64_t)khz * 2000;
  }
  s->D[i].scratch = (double *)(b + L.scratch);
  geos<T>(s)[i] = g;

  std::vector<T> absv(P.absv.size()), av(P.absv.size()), vsqm(P.vsqm.size()), rden(P.rden.size());
  for (size_t k = 0; k < absv.size(); ++k) { absv[k] = T(P.absv[k]); av[k] = T(P.absv[k] * P.n[0]); }
  for (size_t k = 0; k < vsqm.size(); ++k) vsqm[k] = T(P.vsqm[k]);
  for (size_t k = 0; k < rden.size(); ++k) rden[k] = T(P.rden[k]);
  hipStream_t st = s->stream;
  HIPCHK(s, hipMemsetAsync(b, 0, L.total, st));
  HIPCHK(s, hipMemcpyAsync((void *)g.flags, P.flags.data(), P.flags.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync((void *)g.absv, absv.data(), absv.size() * sizeof(T), hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync((void *)g.av, av.data(), av.size() * sizeof(T), hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync((void *)g.vsqm, vsqm.data(), vsqm.size() * sizeof(T), hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync((void *)g.rden, rden.data(), rden.size() * sizeof(T), hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync((void *)g.wq, P.wq.data(), P.wq.size() * 8, hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync((void *)g.diag_tiles, P.diag_tiles.data(), P.diag_tiles.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync((void *)g.fluid_idx, P.fluid_idx.data(), P.fluid_idx.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync((void *)g.diag_off, P.diag_off.data(), P.diag_off.size() * 4, hipMemcpyHostToDevice, st));
  Ctl c{};
  c.kn_coef = 2.0 / std::sqrt(M_PI) * (std::isinf(P.kn) ? 0.0 : P.kn);
  c.err = -1.0;
  c.stop = 1;
  HIPCHK(s, hipMemcpyAsync(g.ctl, &c, sizeof(Ctl), hipMemcpyHostToDevice, st));
  // the rest state: zeros, except where the offset form stores h - rho_r
  if (g.dev) HIPCHK(s, launch_init_state<T>(g, nullptr, nullptr, st));
  HIPCHK(s, hipStreamSynchronize(st));
  return PDVM_OK;
}

// Strip-pipeline shape (kStrip*): two velocity groups per wavefront halve the
// LDS reads of the voxel records per update; PDVM_STRIP_SHAPE (0..3)
// overrides the choice for tuning.
int strip_shape_for(const pdvm_solver *s) {
  if (const char *e = std::getenv("PDVM_STRIP_SHAPE")) {
    const int v = std::atoi(e);
    if (v >= 0 && v < kStripShapes) return v;
  }
  return s->P[0].ngroups >= 2 ? kStrip4x2 : kStrip4x1;
}

// Descriptor array and per-launch block offsets of the whole batch.
template <typename T>
int finalize_batch(pdvm_solver *s) {
  const int n = s->n();
  const Problem &P0 = s->P[0];
  int ndmax = 0;
  for (auto &P : s->P) ndmax = std::max(ndmax, P.ndiag);
  s->h_item_off.assign((size_t)ndmax * (n + 1), 0);
  for (int d = 0; d < ndmax; ++d) {
    int acc = 0;
    for (int p = 0; p < n; ++p) {
      s->h_item_off[(size_t)d * (n + 1) + p] = acc;
      const Problem &P = s->P[p];
      if (d < P.ndiag && P.dim == 2) acc += (P.diag_off[d + 1] - P.diag_off[d]) * (P.ngroups << 2);
      if (d < P.ndiag && P.dim == 3) acc += (P.diag_off[(d + 1) * 8] - P.diag_off[d * 8]) * P.ngroups;
    }
    s->h_item_off[(size_t)d * (n + 1) + n] = acc;
  }
  s->h_blk_off.assign(n + 1, 0);
  for (int p = 0; p < n; ++p) s->h_blk_off[p + 1] = s->h_blk_off[p] + s->P[p].mom_blocks;
  int tile_edge = kTileEdge[0];
  for (auto &P : s->P)
    if (std::max(P.tile[0], P.tile[1]) > kTileEdge[0]) tile_edge = kTileEdge[1];
  // row pipeline: per problem, bands of band_waves tile rows x (chains
  // rounded up to 8) blocks
  const int stride = ((P0.ngroups << P0.dim) + 7) / 8 * 8, nw = band_waves(tile_edge);
  s->h_row_off.assign(n + 1, 0);
  for (int p = 0; p < n; ++p) s->h_row_off[p + 1] = s->h_row_off[p] + (s->P[p].ntile[1] + nw - 1) / nw * stride;
  // strip pipeline (2D): bands of strip_nw strips of strip_th rows, per chain set
  const int sshape = strip_shape_for(s);
  const int sg = strip_g(sshape), sth = strip_th(sshape), snw = strip_nw(sshape);
  const int sstride = ((((P0.ngroups + sg - 1) / sg) << P0.dim) + 7) / 8 * 8;
  s->h_strip_off.assign(n + 1, 0);
  for (int p = 0; p < n; ++p)
    s->h_strip_off[p + 1] = s->h_strip_off[p] + ((s->P[p].n[1] + sth - 1) / sth + snw - 1) / snw * sstride;
  const size_t strip_b = align256(s->h_strip_off.size() * 4);
  const size_t geo_b = align256(n * sizeof(Geo<T>));
  const size_t item_b = align256(s->h_item_off.size() * 4);
  const size_t blk_b = align256(s->h_blk_off.size() * 4);
  const size_t row_b = align256(s->h_row_off.size() * 4);
  const size_t ctl_b = align256(n * sizeof(Ctl));
  const size_t xcc_b = align256((size_t)std::max(s->h_row_off[n], s->h_strip_off[n]));
  void *m = nullptr;
  if (hipMalloc(&m, geo_b + item_b + blk_b + row_b + ctl_b + xcc_b + strip_b) != hipSuccess)
    return s->fail(PDVM_E_NOMEM, "hipMalloc of the batch tables failed");
  s->meta = (char *)m;
  char *geo = s->meta, *item = geo + geo_b, *blk = item + item_b, *rowo = blk + blk_b;
  s->d_ctl_all = (Ctl *)(rowo + row_b);
  s->d_xcc = (uint8_t *)(rowo + row_b + ctl_b);
  char *stripo = rowo + row_b + ctl_b + xcc_b;
  HIPCHK(s, hipMemcpyAsync(stripo, s->h_strip_off.data(), s->h_strip_off.size() * 4, hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemcpyAsync(rowo, s->h_row_off.data(), s->h_row_off.size() * 4, hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemcpyAsync(geo, geos<T>(s).data(), n * sizeof(Geo<T>), hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemcpyAsync(item, s->h_item_off.data(), s->h_item_off.size() * 4, hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemcpyAsync(blk, s->h_blk_off.data(), s->h_blk_off.size() * 4, hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  Batch<T> &B = batch<T>(s);
  B.nprob = n;
  B.dim = P0.dim;
  B.Ko = P0.Ko;
  B.tile_edge = tile_edge;
  B.y2wall = P0.stencil_rule == 0;
  B.tau_fb = P0.tau_fb;
  B.psi = P0.psi;
  B.shakhov = P0.prandtl > 0;
  B.maxwell = P0.spec > 0;
  B.ndiag_max = ndmax;
  B.d_geo = (const Geo<T> *)geo;
  B.d_item_off = (const int *)item;
  B.d_blk_off = (const int *)blk;
  B.h_item_off = s->h_item_off.data();
  B.h_blk_off = s->h_blk_off.data();
  B.d_row_off = (const int *)rowo;
  B.h_row_off = s->h_row_off.data();
  B.row_stride = stride;
  B.d_strip_off = (const int *)stripo;
  B.h_strip_off = s->h_strip_off.data();
  B.strip_stride = sstride;
  B.strip_shape = sshape;
  if (hipHostMalloc((void **)&s->host_ctl, n * sizeof(Ctl), hipHostMallocDefault) != hipSuccess)
    return s->fail(PDVM_E_NOMEM, "pinned host allocation failed");
  return PDVM_OK;
}

template <typename T>
int enqueue_sweep(pdvm_solver *s, const Scratch &scr) {
  const Batch<T> &B = batch<T>(s);
  if (s->queue) {
    HIPCHK(s, launch_sweep_queue<T>(B, s->stream, scr));
  } else if (s->strips) {
    HIPCHK(s, launch_sweep_strips<T>(B, s->stream, scr));
  } else if (s->rows) {
    HIPCHK(s, launch_sweep_rows<T>(B, s->rows_local, s->stream, scr));
  } else {
    for (int d = 0; d < B.ndiag_max; ++d) HIPCHK(s, launch_sweep<T>(B, d, s->stream));
  }
  return PDVM_OK;
}

// One iteration: sweep, moments, reduction. `scr`: the kernels' scratch (the
// problems' own workspaces when empty).
template <typename T>
int enqueue_iteration(pdvm_solver *s, const Scratch &scr) {
  const Batch<T> &B = batch<T>(s);
  const int rc = enqueue_sweep<T>(s, scr);
  if (rc != PDVM_OK) return rc;
  HIPCHK(s, launch_moments<T>(B, s->stream, scr));
  HIPCHK(s, launch_reduce<T>(B, s->stream, scr));
  return PDVM_OK;
}

int enqueue_iteration_any(pdvm_solver *s, const Scratch &scr = Scratch{}) {
  return s->precision == PDVM_FP64 ? enqueue_iteration<double>(s, scr) : enqueue_iteration<float>(s, scr);
}

int build_graph(pdvm_solver *s) {
  if (s->graph) return PDVM_OK;
  // a few iterations per replay amortise the launch of the graph itself
  const int per = std::max(1, std::min(8, s->P[0].check_every));
  hipGraph_t gr;
  HIPCHK(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
  int rc = PDVM_OK;
  for (int i = 0; i < per && rc == PDVM_OK; ++i) rc = enqueue_iteration_any(s);
  hipError_t e = hipStreamEndCapture(s->stream, &gr);
  if (rc != PDVM_OK) return rc;
  if (e != hipSuccess) return s->fail(PDVM_E_HIP, "graph capture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&s->graph, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (e != hipSuccess) return s->fail(PDVM_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
  s->graph_iters = per;
  return PDVM_OK;
}

// All control blocks to the pinned host mirror (one gather, one copy).
int read_ctl(pdvm_solver *s) {
  if (s->precision == PDVM_FP64) HIPCHK(s, launch_ctl_gather<double>(s->bd, s->d_ctl_all, s->stream));
  else HIPCHK(s, launch_ctl_gather<float>(s->bf, s->d_ctl_all, s->stream));
  HIPCHK(s, hipMemcpyAsync(s->host_ctl, s->d_ctl_all, s->n() * sizeof(Ctl), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return PDVM_OK;
}

int arm(pdvm_solver *s, double tol, int mode, int64_t max_iters) {
  if (s->precision == PDVM_FP64) HIPCHK(s, launch_arm<double>(s->bd, tol, mode, max_iters, s->stream));
  else HIPCHK(s, launch_arm<float>(s->bf, tol, mode, max_iters, s->stream));
  return PDVM_OK;
}

Ctl *dev_ctl(pdvm_solver *s, int i) { return s->precision == PDVM_FP64 ? s->gd[i].ctl : s->gf[i].ctl; }

int check_index(pdvm_solver *s, int i) {
  if (!s) { set_thread_error("solver is NULL"); return PDVM_E_INVAL; }
  if (i < 0 || i >= s->n()) return s->fail(PDVM_E_INVAL, "problem index %d outside [0, %d)", i, s->n());
  return PDVM_OK;
}

bool same_velocity_grid(const Problem &a, const Problem &b) {
  return a.dim == b.dim && a.Ko == b.Ko && a.Ko_pad == b.Ko_pad && a.absv == b.absv && a.wq.size() == b.wq.size() &&
         std::equal(a.wq.begin(), a.wq.begin() + a.Ko_pad, b.wq.begin());
}

// Whether every chain of a one-launch pipeline (blocks off[p] + c, + stride,
// ...) runs on a single XCD: run the pipeline's grid (same blocks, same block
// size) once with a kernel that records each block's XCD. Needs at least two
// distinct XCDs in the record (so the register read is live) and one XCD per
// chain. sets: the real blocks per band.
int probe_xcd_locality(pdvm_solver *s, const std::vector<int> &off, int stride, int sets, int threads, bool *local_out) {
  const int n = s->n(), blocks = off[n];
  uint32_t *d = nullptr;
  if (hipMalloc(&d, sizeof(uint32_t) * blocks) != hipSuccess) return s->fail(PDVM_E_NOMEM, "probe allocation failed");
  std::vector<uint32_t> h(blocks);
  hipError_t e = launch_xcd_probe(d, blocks, threads, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, sizeof(uint32_t) * blocks, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return s->fail(PDVM_E_HIP, "XCD probe: %s", hipGetErrorString(e));
  bool local = true, several = false;
  for (int p = 0; p < n; ++p)
    for (int b = off[p]; b < off[p + 1]; ++b) {
      const int c = (b - off[p]) % stride;
      if (c < sets) local = local && h[b] == h[off[0] + c];
      several = several || h[b] != h[0];
    }
  *local_out = local && several;
  return PDVM_OK;
}

// Whether a grid of kQueueBlocks blocks reaches all 8 XCDs (the queue sweep
// serves the queue of an XCD only from blocks that run on it).
int probe_all_xcds(pdvm_solver *s, bool *ok) {
  uint32_t *d = nullptr;
  if (hipMalloc(&d, sizeof(uint32_t) * kQueueBlocks) != hipSuccess) return s->fail(PDVM_E_NOMEM, "probe allocation failed");
  std::vector<uint32_t> h(kQueueBlocks);
  hipError_t e = launch_xcd_probe(d, kQueueBlocks, kWave, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, sizeof(uint32_t) * kQueueBlocks, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return s->fail(PDVM_E_HIP, "XCD probe: %s", hipGetErrorString(e));
  bool seen[8] = {false, false, false, false, false, false, false, false};
  for (uint32_t x : h) seen[x & 7u] = true;
  *ok = true;
  for (bool b : seen) *ok = *ok && b;
  return PDVM_OK;
}

// The queue sweep's items (see sweep_queue_kernel): the velocity chains
// (problem, octant, group) are dealt to the 8 XCDs and their sub-queues,
// largest first to the least loaded; each queue lists its chains' tiles that hold fluid, by
// diagonal, then problem, octant, tile and group, with the waits each tile
// needs. With s->columns (3D) an item is a segment of kColumnTiles tiles of
// a column along x3 holding fluid, by the diagonal of its first tile, and
// each tile's waits go to the per-octant table Geo::qtinfo. Also the done
// flags (zero: below every stamp) and the counters.
template <typename T>
int build_queue(pdvm_solver *s) {
  const int n = s->n();
  std::vector<Geo<T>> &G = geos<T>(s);
  Batch<T> &B = batch<T>(s);
  std::vector<int64_t> chain_base(n + 1, 0), work(n, 0);
  int64_t flags = 0;
  int maxd = 0;
  for (int p = 0; p < n; ++p) {
    const Problem &P = s->P[p];
    const int64_t nt = (int64_t)P.ntile[0] * P.ntile[1] * P.ntile[2];
    if (nt >= (1 << 24) || n > 65535) return s->fail(PDVM_E_UNSUPPORTED, "queue sweep: at most 2^24 tiles per problem and 65535 problems");
    for (uint8_t l : P.live) work[p] += l;
    G[p].qflag_off = flags;
    G[p].ntiles_all = (int32_t)nt;
    const int chains = P.ngroups << P.dim;
    flags += chains * nt;
    chain_base[p + 1] = chain_base[p] + chains;
    maxd = std::max(maxd, P.ndiag);
  }
  // deal the chains: an octant of a problem (all its velocity groups, or a
  // share of them when there are fewer octants than XCDs) to one XCD, largest
  // work first to the least loaded, and its groups to that XCD's least loaded
  // sub-queues. The groups of an octant sweep the same tiles in the same
  // order, so the XCD's L2 serves each tile's records (flags, sources, wall
  // values) to all of them from one fetch.
  std::vector<int> owner(chain_base[n]);
  struct Unit {
    int p, o, g0, g1;
  };
  std::vector<Unit> units;
  int octants = 0;
  for (int p = 0; p < n; ++p) octants += 1 << s->P[p].dim;
  const int split = (8 + octants - 1) / octants;
  for (int p = 0; p < n; ++p)
    for (int o = 0; o < (1 << s->P[p].dim); ++o) {
      const int ng = s->P[p].ngroups, parts = std::min(split, ng);
      for (int k = 0; k < parts; ++k) units.push_back({p, o, ng * k / parts, ng * (k + 1) / parts});
    }
  std::stable_sort(units.begin(), units.end(), [&](const Unit &a, const Unit &b) {
    return work[a.p] * (a.g1 - a.g0) > work[b.p] * (b.g1 - b.g0);
  });
  // queue index x * kQueueSub + i: the XCD, then its sub-queue, both least
  // loaded (ties to the lowest index, so an XCD's used sub-queues come first)
  int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<int64_t> subload(8 * kQueueSub, 0);
  for (const Unit &u : units) {
    const int x = (int)(std::min_element(load, load + 8) - load);
    load[x] += work[u.p] * (u.g1 - u.g0);
    for (int g = u.g0; g < u.g1; ++g) {
      const auto b = subload.begin() + x * kQueueSub;
      const int i = (int)(std::min_element(b, b + kQueueSub) - b);
      owner[chain_base[u.p] + u.o * s->P[u.p].ngroups + g] = x * kQueueSub + i;
      subload[x * kQueueSub + i] += work[u.p];
    }
  }
  // per problem and diagonal: (octant, tile, waits) of the tiles holding
  // fluid, or (octant, column) of the columns holding fluid; tinfo: per
  // problem, octant and tile, 128 (fluid) + the waits along x1 and x2
  const bool col = s->columns;
  std::vector<std::vector<std::vector<uint64_t>>> diag(n);
  std::vector<int64_t> info_off(n + 1, 0);
  for (int p = 0; p < n; ++p) info_off[p + 1] = info_off[p] + (col ? 8 * (int64_t)G[p].ntiles_all : 0);
  std::vector<int32_t> tinfo((size_t)info_off[n], 0);
  for (int p = 0; p < n; ++p) {
    const Problem &P = s->P[p];
    const int nt[3] = {P.ntile[0], P.ntile[1], P.ntile[2]};
    const int64_t stride[3] = {1, nt[0], (int64_t)nt[0] * nt[1]};
    diag[p].assign(P.ndiag, {});
    const int S = std::min(kColumnTiles, nt[2]), nseg = (nt[2] + S - 1) / S;
    G[p].col_tiles = S;
    std::vector<uint8_t> col_live(col ? (size_t)8 * stride[2] * nseg : 0, 0);  // [octant][segment][column]
    for (int o = 0; o < (1 << P.dim); ++o)
      for (int c = 0; c < nt[2]; ++c)
        for (int b = 0; b < nt[1]; ++b)
          for (int a = 0; a < nt[0]; ++a) {
            const int ori[3] = {a, b, c};
            int ph[3];
            for (int j = 0; j < 3; ++j) ph[j] = ((o >> j) & 1) ? nt[j] - 1 - ori[j] : ori[j];
            const int64_t t = ph[0] + stride[1] * ph[1] + stride[2] * ph[2];
            if (!P.live[t]) continue;
            uint64_t waits = 0;
            for (int j = 0; j < P.dim; ++j) {
              const int sj = ((o >> j) & 1) ? -1 : 1;
              const int u1 = ph[j] - sj, u2 = ph[j] - 2 * sj;
              if (u1 >= 0 && u1 < nt[j] && P.live[t - sj * stride[j]]) waits |= 1ull << (2 * j);
              const bool thin = u1 >= 0 && u1 < nt[j] && std::min(P.tile[j], P.n[j] - u1 * P.tile[j]) == 1;
              if (thin && u2 >= 0 && u2 < nt[j] && P.live[t - 2 * sj * stride[j]]) waits |= 1ull << (2 * j + 1);
            }
            if (!col) {
              diag[p][a + b + c].push_back((uint64_t)t | ((uint64_t)o << 24) | (waits << 48));
            } else {
              tinfo[info_off[p] + o * G[p].ntiles_all + t] = 128 | (int32_t)waits;
              col_live[(o * nseg + c / S) * stride[2] + t % stride[2]] = 1;
            }
          }
    if (col)
      for (int o = 0; o < 8; ++o)
        for (int k = 0; k < nseg; ++k)
          for (int b = 0; b < nt[1]; ++b)
            for (int a = 0; a < nt[0]; ++a) {
              const int pa = (o & 1) ? nt[0] - 1 - a : a, pb = (o & 2) ? nt[1] - 1 - b : b;
              const int64_t cix = pa + stride[1] * pb;
              if (col_live[(o * nseg + k) * stride[2] + cix])
                diag[p][a + b + k * S].push_back((uint64_t)cix | ((uint64_t)o << 24) | ((uint64_t)k << 48));
            }
  }
  std::vector<std::vector<uint64_t>> q(8 * kQueueSub);
  for (int d = 0; d < maxd; ++d)
    for (int p = 0; p < n; ++p) {
      if (d >= (int)diag[p].size()) continue;
      const int ng = s->P[p].ngroups;
      for (uint64_t e : diag[p][d]) {
        const int o = (int)((e >> 24) & 7u);
        for (int g = 0; g < ng; ++g) {
          const int x = owner[chain_base[p] + o * ng + g];
          q[x].push_back(e | ((uint64_t)g << 27) | ((uint64_t)p << 32));
        }
      }
    }
  const int nq = 8 * kQueueSub;
  std::vector<int32_t> off(nq + 1, 0);
  std::vector<uint64_t> items;
  for (int x = 0; x < nq; ++x) {
    items.insert(items.end(), q[x].begin(), q[x].end());
    off[x + 1] = (int32_t)items.size();
  }
  if (items.size() >= ((size_t)1 << 31)) return s->fail(PDVM_E_UNSUPPORTED, "queue sweep: too many tiles");
  const size_t item_b = align256(std::max<size_t>(1, items.size()) * 8), off_b = align256((nq + 1) * 4),
               ctr_b = align256(kQueueCounterInts * 4);
  const size_t flag_b = align256((size_t)flags * 4), info_b = align256(tinfo.size() * 4);
  const size_t all_b = item_b + off_b + ctr_b + flag_b + info_b;
  if (hipMalloc(&s->qmem, all_b) != hipSuccess)
    return s->fail(PDVM_E_NOMEM, "queue sweep: device allocation of %zu bytes failed", all_b);
  char *m = s->qmem;
  HIPCHK(s, hipMemcpyAsync(m, items.data(), items.size() * 8, hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemcpyAsync(m + item_b, off.data(), (nq + 1) * 4, hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemsetAsync(m + item_b + off_b, 0, ctr_b + flag_b, s->stream));
  if (col) {
    const int32_t *dinfo = (const int32_t *)(m + item_b + off_b + ctr_b + flag_b);
    HIPCHK(s, hipMemcpyAsync((void *)dinfo, tinfo.data(), tinfo.size() * 4, hipMemcpyHostToDevice, s->stream));
    for (int p = 0; p < n; ++p) G[p].qtinfo = dinfo + info_off[p];
  }
  B.use_columns = col ? 1 : 0;
  B.use_queue = 1;
  B.q_total = (int)items.size();
  B.d_qitems = (const uint64_t *)m;
  B.d_q_off = (const int32_t *)(m + item_b);
  B.d_qctr = (int32_t *)(m + item_b + off_b);
  B.d_qflags = (int32_t *)(m + item_b + off_b + ctr_b);
  s->qflag_ints = (size_t)flags;
  HIPCHK(s, hipMemcpyAsync((void *)B.d_geo, G.data(), n * sizeof(Geo<T>), hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return PDVM_OK;
}

const char *sweep_name(const pdvm_solver *s) {
  return s->queue ? (s->columns ? "column-queue" : "queue")
                  : (s->strips ? "strip-pipeline" : (s->rows ? "row-pipeline" : "tile-diagonal"));
}

// Chain sets of the strip pipeline per band.
int strip_sets(const pdvm_solver *s, int shape) {
  const Problem &P = s->P[0];
  return ((P.ngroups + strip_g(shape) - 1) / strip_g(shape)) << P.dim;
}

// Point every problem's descriptor at its range of the per-block XCD records
// (block = row_off[p] + band * stride + chain) and upload the descriptors.
template <typename T>
int enable_xcc_check(pdvm_solver *s) {
  std::vector<Geo<T>> &G = geos<T>(s);
  Batch<T> &B = batch<T>(s);
  B.use_strips = s->strips ? 1 : 0;
  const std::vector<int> &off = s->strips ? s->h_strip_off : s->h_row_off;
  for (int p = 0; p < s->n(); ++p) {
    G[p].xcc_seen = s->d_xcc + off[p];
    G[p].row_blocks = off[p + 1] - off[p];
    G[p].row_stride = s->strips ? B.strip_stride : B.row_stride;
    G[p].row_sets = s->strips ? strip_sets(s, B.strip_shape) : (s->P[p].ngroups << s->P[p].dim);
  }
  HIPCHK(s, hipMemcpyAsync((void *)B.d_geo, G.data(), s->n() * sizeof(Geo<T>), hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return PDVM_OK;
}

// A problem whose sweep was abandoned stays stopped until its state is restored.
int check_not_poisoned(pdvm_solver *s) {
  int rc = read_ctl(s);
  if (rc != PDVM_OK) return rc;
  for (int i = 0; i < s->n(); ++i)
    if (s->host_ctl[i].fault)
      return s->fail(PDVM_E_STATE,
                     "problem %d: an earlier sweep was abandoned and its iterate discarded; restore a state "
                     "(set_initial or set_state) before iterating again", i);
  return PDVM_OK;
}

int create_common(const pdvm_config *cfgs, int n, void *dev_workspace, size_t ws_bytes, void *hip_stream,
                  pdvm_solver **out) {
  if (!out) { set_thread_error("out is NULL"); return PDVM_E_INVAL; }
  *out = nullptr;
  if (n < 1 || !cfgs) { set_thread_error("need at least one config"); return PDVM_E_INVAL; }
  pdvm_solver *s = new (std::nothrow) pdvm_solver();
  if (!s) { set_thread_error("host allocation failed"); return PDVM_E_NOMEM; }
  s->P.resize(n);
  s->D.resize(n);
  for (int i = 0; i < n; ++i) {
    std::string err;
    const int rc = validate_and_build(&cfgs[i], s->P[i], err);
    if (rc != PDVM_OK) {
      set_thread_error("config %d: %s", i, err.c_str());
      delete s;
      return rc;
    }
    const Problem &A = s->P[0], &B = s->P[i];
    if (B.precision != A.precision || !same_velocity_grid(A, B) || B.stencil_rule != A.stencil_rule ||
        B.tau_fb != A.tau_fb || (B.prandtl > 0) != (A.prandtl > 0) || (B.spec > 0) != (A.spec > 0)) {
      set_thread_error("config %d: a batch shares dimension, precision, velocity grid, stencil rule, tau feedback "
                       "and collision model", i);
      delete s;
      return PDVM_E_INVAL;
    }
  }
  s->precision = s->P[0].precision;
  if (s->precision == PDVM_FP64) s->gd.resize(n);
  else s->gf.resize(n);
  s->stream = (hipStream_t)hip_stream;
  if (!s->stream) {
    // the null stream cannot be captured into a graph: use a private one
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
      set_thread_error("hipStreamCreate failed");
      delete s;
      return PDVM_E_HIP;
    }
    s->own_stream = true;
  }
  for (int i = 0; i < n; ++i) {
    const size_t need = layout_bytes(s->P[i]);
    if (dev_workspace) {  // single problem only
      if (ws_bytes < need || ((uintptr_t)dev_workspace & 255)) {
        set_thread_error("workspace needs %zu bytes, 256-byte aligned (got %zu)", need, ws_bytes);
        pdvm_destroy(s);
        return PDVM_E_NOMEM;
      }
      s->D[i].ws = (char *)dev_workspace;
    } else {
      void *p = nullptr;
      if (hipMalloc(&p, need) != hipSuccess) {
        set_thread_error("hipMalloc of %zu bytes failed (problem %d)", need, i);
        pdvm_destroy(s);
        return PDVM_E_NOMEM;
      }
      s->D[i].ws = (char *)p;
      s->D[i].own_ws = true;
    }
    s->D[i].bytes = need;
    const int rc = s->precision == PDVM_FP64 ? setup_problem<double>(s, i) : setup_problem<float>(s, i);
    if (rc != PDVM_OK) {
      g_thread_error = s->err;
      pdvm_destroy(s);
      return rc;
    }
  }
  const int rc = s->precision == PDVM_FP64 ? finalize_batch<double>(s) : finalize_batch<float>(s);
  if (rc != PDVM_OK) {
    g_thread_error = s->err;
    pdvm_destroy(s);
    return rc;
  }
  const Problem &P0 = s->P[0];
  // the strip pipeline: 2D, the isothermal BGK source with diffuse walls, and
  // XCD-local placement (probed); the automatic choice when all three hold
  bool strip_model = P0.dim == 2 && !P0.tau_fb && !(P0.prandtl > 0) && !(P0.spec > 0);
  for (const Problem &P : s->P)  // a row of h addressed through one buffer resource, below 1 GiB
    strip_model = strip_model && (int64_t)P.n[0] * P.Kpad * (s->precision == PDVM_FP64 ? 8 : 4) < (int64_t(1) << 30);
  if (P0.schedule == PDVM_SCHEDULE_STRIPS && !strip_model) {
    set_thread_error("the strip pipeline serves 2D problems with the isothermal source and diffuse walls");
    pdvm_destroy(s);
    return PDVM_E_UNSUPPORTED;
  }
  // (measured slower than the row pipeline and the tile diagonals, so only on request)
  if (strip_model && P0.schedule == PDVM_SCHEDULE_STRIPS) {
    const int shape = s->precision == PDVM_FP64 ? s->bd.strip_shape : s->bf.strip_shape;
    bool local = false;
    const int rc2 = probe_xcd_locality(s, s->h_strip_off, s->precision == PDVM_FP64 ? s->bd.strip_stride
                                                                                      : s->bf.strip_stride,
                                       strip_sets(s, shape), kWave * strip_nw(shape), &local);
    if (rc2 != PDVM_OK) {
      g_thread_error = s->err;
      pdvm_destroy(s);
      return rc2;
    }
    if (!local && P0.schedule == PDVM_SCHEDULE_STRIPS) {
      set_thread_error("the strip pipeline needs every chain set on one XCD; the placement probe found otherwise");
      pdvm_destroy(s);
      return PDVM_E_UNSUPPORTED;
    }
    s->strips = local;
  }
  // automatic otherwise: the row pipeline for a single 2D problem; a batch
  // fills the machine better with per-diagonal launches (measured)
  s->rows = !s->strips && P0.dim == 2 &&
            (P0.schedule == PDVM_SCHEDULE_ROWS || P0.schedule == PDVM_SCHEDULE_ROWS_AGENT ||
             (P0.schedule == PDVM_SCHEDULE_AUTO && n == 1));
  if (s->rows) {
    // the row pipeline stores a tile through 32-bit byte offsets from its
    // lowest-addressed voxel
    const int edge = s->precision == PDVM_FP64 ? s->bd.tile_edge : s->bf.tile_edge;
    const int64_t elem = s->precision == PDVM_FP64 ? 8 : 4;
    bool fits = true;
    for (const Problem &P : s->P) fits = fits && (int64_t)edge * (P.n[0] + 1) * P.Kpad * elem < (int64_t(1) << 32);
    if (!fits) {
      if (P0.schedule != PDVM_SCHEDULE_AUTO) {
        set_thread_error("the row pipeline needs a tile's span of h below 4 GiB (use the diagonal schedule)");
        pdvm_destroy(s);
        return PDVM_E_UNSUPPORTED;
      }
      s->rows = false;
    }
  }
  if (s->rows && P0.schedule != PDVM_SCHEDULE_ROWS_AGENT) {
    const int rc2 = probe_xcd_locality(s, s->h_row_off, s->precision == PDVM_FP64 ? s->bd.row_stride
                                                                                  : s->bf.row_stride,
                                       P0.ngroups << P0.dim,
                                       kWave * band_waves(s->precision == PDVM_FP64 ? s->bd.tile_edge
                                                                                    : s->bf.tile_edge),
                                       &s->rows_local);
    if (rc2 != PDVM_OK) {
      g_thread_error = s->err;
      pdvm_destroy(s);
      return rc2;
    }
    // automatic choice: the row pipeline only with the cheap XCD-local protocol
    if (!s->rows_local && P0.schedule == PDVM_SCHEDULE_AUTO) s->rows = false;
  }
  if (s->strips || (s->rows && s->rows_local)) {
    // the XCD-local protocol is checked on every sweep: each block records its
    // XCD and the reduction discards an iterate whose chains were split
    const int rc3 = s->precision == PDVM_FP64 ? enable_xcc_check<double>(s) : enable_xcc_check<float>(s);
    if (rc3 != PDVM_OK) {
      g_thread_error = s->err;
      pdvm_destroy(s);
      return rc3;
    }
  }
  // the queue sweep: on request, and the automatic choice for 3D problems and
  // 2D batches (measured, FP32: 64 mixed 2D problems 2.5 ms per sweep against
  // 3.9 ms of per-diagonal launches with 8x8 tiles, 2.9 against 5.0 with 4x4;
  // the 96^3 pack 4.3 against 4.4 ms), when blocks reach all 8 XCDs
  if (!s->strips && !s->rows &&
      (P0.schedule == PDVM_SCHEDULE_QUEUE || P0.schedule == PDVM_SCHEDULE_COLUMNS ||
       (P0.schedule == PDVM_SCHEDULE_AUTO && (P0.dim == 3 || n > 1)))) {
    bool all = false;
    int rc4 = probe_all_xcds(s, &all);
    if (rc4 == PDVM_OK && !all && P0.schedule != PDVM_SCHEDULE_AUTO)
      rc4 = s->fail(PDVM_E_UNSUPPORTED, "the queue sweep needs blocks on all 8 XCDs; the placement probe found fewer");
    if (rc4 == PDVM_OK && all) {
      s->queue = true;
      s->columns = P0.schedule == PDVM_SCHEDULE_COLUMNS;
      rc4 = s->precision == PDVM_FP64 ? build_queue<double>(s) : build_queue<float>(s);
    }
    if (rc4 != PDVM_OK) {
      g_thread_error = s->err;
      pdvm_destroy(s);
      return rc4;
    }
  }
  // pdvm_iterate_noalloc: this GPU's static scratch (its address is taken
  // here, once per device) and the regions of it this batch would use
  {
    int dev = 0;
    void *ptr = nullptr;
    s->scratch_err = hipGetDevice(&dev);
    if (s->scratch_err == hipSuccess) s->scratch_err = scratch_address(dev, &ptr);
    s->scratch_dev = (char *)ptr;
    s->scr_part = 0;
    s->scr_prog = align256((size_t)s->h_blk_off[n] * 4 * sizeof(double));
    const size_t pipe = (size_t)std::max(s->h_row_off[n], s->h_strip_off[n]);
    s->scr_xcc = s->scr_prog + align256(pipe * sizeof(int32_t));
    s->scr_qctr = s->scr_xcc + align256(pipe);
    s->scr_qflags = s->scr_qctr + (s->queue ? align256(kQueueCounterInts * 4) : 0);
    s->scr_need = s->scr_qflags + (s->queue ? align256(s->qflag_ints * 4) : 0);
    s->start_iters.assign(n, 0);
  }
  *out = s;
  return PDVM_OK;
}

int set_initial_one(pdvm_solver *s, int i, const double *rho, const double *u) {
  const Problem &P = s->P[i];
  const int64_t N = P.N;
  double *drho = nullptr, *du = nullptr;
  if (rho) {
    drho = s->D[i].scratch + 4 * N;
    HIPCHK(s, hipMemcpyAsync(drho, rho, N * 8, hipMemcpyHostToDevice, s->stream));
  }
  if (u) {
    du = s->D[i].scratch + 5 * N;
    HIPCHK(s, hipMemcpyAsync(du, u, (size_t)P.dim * N * 8, hipMemcpyHostToDevice, s->stream));
  }
  int rc = read_ctl(s);
  if (rc != PDVM_OK) return rc;
  Ctl c = s->host_ctl[i];
  c.iter = 0;
  c.stop = 1;
  c.status = 0;
  c.fault = 0;
  c.err = -1.0;
  c.r = c.k = c.gp = 0;
  for (double &v : c.kring) v = 0;
  s->host_ctl[i] = c;
  HIPCHK(s, hipMemcpyAsync(dev_ctl(s, i), &s->host_ctl[i], sizeof(Ctl), hipMemcpyHostToDevice, s->stream));
  if (s->precision == PDVM_FP64) HIPCHK(s, launch_init_state<double>(s->gd[i], drho, du, s->stream));
  else HIPCHK(s, launch_init_state<float>(s->gf[i], drho, du, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return PDVM_OK;
}

// Iterate the whole batch until every problem stopped or max_iters ran.
int iterate_batch(pdvm_solver *s, int64_t max_iters, double tol, int32_t stop_mode, pdvm_stats *out) {
  if (max_iters < 0 || (stop_mode != PDVM_STOP_FIELD && stop_mode != PDVM_STOP_PAPER_ERR) || std::isnan(tol))
    return s->fail(PDVM_E_INVAL, "max_iters >= 0, a valid stop mode and a non-NaN tol are required");
  const auto t0 = std::chrono::steady_clock::now();
  int rc = check_not_poisoned(s);
  if (rc != PDVM_OK) return rc;
  rc = build_graph(s);
  if (rc != PDVM_OK) return rc;
  const int n = s->n();
  std::vector<int64_t> start(n);
  for (int i = 0; i < n; ++i) start[i] = s->host_ctl[i].iter;
  rc = arm(s, tol, stop_mode, max_iters);
  if (rc != PDVM_OK) return rc;
  int64_t launched = 0;
  const int per = s->graph_iters;
  const int poll = std::max(per, s->P[0].check_every / per * per);
  while (launched < max_iters) {
    int64_t b = 0;
    while (b < poll && launched < max_iters) {
      HIPCHK(s, hipGraphLaunch(s->graph, s->stream));
      b += per;
      launched += per;
    }
    rc = read_ctl(s);
    if (rc != PDVM_OK) return rc;
    bool all = true;
    for (int i = 0; i < n; ++i) all = all && s->host_ctl[i].stop;
    if (all) break;
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = PDVM_OK;
  for (int i = 0; i < n; ++i) {
    const Ctl &c = s->host_ctl[i];
    if (out) {
      out[i].iters = c.iter - start[i];
      out[i].total_iters = c.iter;
      out[i].r = c.r;
      out[i].err = c.err;
      out[i].k = c.k;
      out[i].gp = c.gp;
      out[i].seconds = secs;
      out[i].converged = c.status == 1;
    }
    if (c.fault == 1)
      return s->fail(PDVM_E_HIP, "problem %d: a %s sweep gave up waiting for its upstream tiles; the iterate "
                                 "was discarded and the previous state kept", i, sweep_name(s));
    if (c.fault)
      return s->fail(PDVM_E_HIP, "problem %d: %s; the iterate was discarded and the previous state kept", i,
                     s->queue ? "a queue sweep left tiles unswept (a queue had no block on its XCD)"
                              : "the blocks of a pipelined velocity chain ran on different XCDs");
    if (c.status == -4) worst = PDVM_E_NONFINITE;
    else if (c.status != 1 && worst == PDVM_OK) worst = PDVM_NOT_CONVERGED;
  }
  if (worst == PDVM_E_NONFINITE)
    return s->fail(PDVM_E_NONFINITE, "residual or permeability became non-finite; the previous state is kept");
  return worst;
}

// pdvm_iterate without allocating: no graph (its instantiation allocates);
// the kernels are enqueued directly, with their scratch in this GPU's static
// array; host work uses only what the solver allocated at creation.
int iterate_noalloc(pdvm_solver *s, int64_t max_iters, double tol, int32_t stop_mode, pdvm_stats *out) {
  if (max_iters < 0 || (stop_mode != PDVM_STOP_FIELD && stop_mode != PDVM_STOP_PAPER_ERR) || std::isnan(tol))
    return s->fail(PDVM_E_INVAL, "max_iters >= 0, a valid stop mode and a non-NaN tol are required");
  if (!s->scratch_dev)
    return s->fail(PDVM_E_HIP, "no device address for the library's static scratch on this GPU: %s",
                   hipGetErrorString(s->scratch_err));
  if (s->scr_need > kNoAllocScratchBytes)
    return s->fail(PDVM_E_NOMEM, "this solve needs %zu bytes of the library's static scratch; it holds %zu (use "
                                 "pdvm_iterate)", s->scr_need, kNoAllocScratchBytes);
  const auto t0 = std::chrono::steady_clock::now();
  int rc = check_not_poisoned(s);
  if (rc != PDVM_OK) return rc;
  const int n = s->n();
  for (int i = 0; i < n; ++i) s->start_iters[i] = s->host_ctl[i].iter;
  Scratch scr;
  scr.part = (double *)(s->scratch_dev + s->scr_part);
  scr.progress = (int32_t *)(s->scratch_dev + s->scr_prog);
  scr.xcc = (uint8_t *)(s->scratch_dev + s->scr_xcc);
  if (s->queue) {
    scr.qctr = (int32_t *)(s->scratch_dev + s->scr_qctr);
    scr.qflags = (int32_t *)(s->scratch_dev + s->scr_qflags);
  }
  rc = arm(s, tol, stop_mode, max_iters);
  if (rc != PDVM_OK) return rc;
  // the counters hold whatever an earlier solve on this GPU left: set them
  // below every stamp of this call
  if (s->queue) HIPCHK(s, launch_fill_i32(scr.qflags, (int64_t)s->qflag_ints, 0, s->stream));
  if (s->rows || s->strips) {
    if (s->precision == PDVM_FP64)
      HIPCHK(s, launch_progress_reset<double>(s->bd, s->strips ? s->bd.d_strip_off : s->bd.d_row_off, s->strips,
                                              scr.progress, s->stream));
    else
      HIPCHK(s, launch_progress_reset<float>(s->bf, s->strips ? s->bf.d_strip_off : s->bf.d_row_off, s->strips,
                                             scr.progress, s->stream));
  }
  const int64_t poll = std::max(1, s->P[0].check_every);
  int64_t launched = 0;
  while (launched < max_iters) {
    for (int64_t b = 0; b < poll && launched < max_iters; ++b, ++launched) {
      rc = enqueue_iteration_any(s, scr);
      if (rc != PDVM_OK) return rc;
    }
    rc = read_ctl(s);
    if (rc != PDVM_OK) return rc;
    bool all = true;
    for (int i = 0; i < n; ++i) all = all && s->host_ctl[i].stop;
    if (all) break;
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = PDVM_OK;
  for (int i = 0; i < n; ++i) {
    const Ctl &c = s->host_ctl[i];
    if (out) {
      out[i].iters = c.iter - s->start_iters[i];
      out[i].total_iters = c.iter;
      out[i].r = c.r;
      out[i].err = c.err;
      out[i].k = c.k;
      out[i].gp = c.gp;
      out[i].seconds = secs;
      out[i].converged = c.status == 1;
    }
    if (c.fault)
      return s->fail(PDVM_E_HIP, "problem %d: a %s sweep was abandoned; the iterate was discarded and the "
                                 "previous state kept", i, sweep_name(s));
    if (c.status == -4) worst = PDVM_E_NONFINITE;
    else if (c.status != 1 && worst == PDVM_OK) worst = PDVM_NOT_CONVERGED;
  }
  if (worst == PDVM_E_NONFINITE)
    return s->fail(PDVM_E_NONFINITE, "residual or permeability became non-finite; the previous state is kept");
  return worst;
}

int get_moments_one(pdvm_solver *s, int i, double *rho, double *u, double *tau, double *q) {
  int rc = read_ctl(s);
  if (rc != PDVM_OK) return rc;
  const int par = s->host_ctl[i].par;
  const Problem &P = s->P[i];
  const int64_t N = P.N;
  const double *drho = s->precision == PDVM_FP64 ? s->gd[i].rho[par] : s->gf[i].rho[par];
  const double *du = s->precision == PDVM_FP64 ? s->gd[i].u[par] : s->gf[i].u[par];
  if (rho) HIPCHK(s, hipMemcpyAsync(rho, drho, N * 8, hipMemcpyDeviceToHost, s->stream));
  if (u) HIPCHK(s, hipMemcpyAsync(u, du, (size_t)P.dim * N * 8, hipMemcpyDeviceToHost, s->stream));
  if (tau || q) {
    double *dt = s->D[i].scratch, *dq = s->D[i].scratch + N;
    if (s->precision == PDVM_FP64) HIPCHK(s, launch_diagnostics<double>(s->gd[i], dt, dq, s->stream));
    else HIPCHK(s, launch_diagnostics<float>(s->gf[i], dt, dq, s->stream));
    if (tau) HIPCHK(s, hipMemcpyAsync(tau, dt, N * 8, hipMemcpyDeviceToHost, s->stream));
    if (q) HIPCHK(s, hipMemcpyAsync(q, dq, (size_t)P.dim * N * 8, hipMemcpyDeviceToHost, s->stream));
  }
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return PDVM_OK;
}

int get_flux_one(pdvm_solver *s, int i, double *gp, double *k, double *gp_section) {
  const Problem &P = s->P[i];
  const int64_t N = P.N;
  std::vector<double> u1(N);
  int rc = read_ctl(s);
  if (rc != PDVM_OK) return rc;
  const int par = s->host_ctl[i].par;
  const double *du = s->precision == PDVM_FP64 ? s->gd[i].u[par] : s->gf[i].u[par];
  HIPCHK(s, hipMemcpyAsync(u1.data(), du, N * 8, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  double tot = 0;
  for (int64_t c = 0; c < N; ++c) tot += (P.flags[c] & F_SOLID) ? 0.0 : u1[c];
  const double G = tot / (double)N;
  if (gp) *gp = G;
  if (k) *k = 2.0 / std::sqrt(M_PI) * (std::isinf(P.kn) ? 0.0 : P.kn) * G;
  if (gp_section) {
    const int n0 = P.n[0];
    const int64_t A = N / n0;
    for (int x = 0; x < n0; ++x) gp_section[x] = 0;
    for (int64_t c = 0; c < N; ++c)
      if (!(P.flags[c] & F_SOLID)) gp_section[c % n0] += u1[c];
    for (int x = 0; x < n0; ++x) gp_section[x] /= (double)A;
  }
  return PDVM_OK;
}

// checkpoint layout: header, Ctl, then the parity-current rho, u, src, srct,
// (Shakhov: srcq,) wall, then the boundary layers of h (Maxwell walls: all of
// h, as their specular part reads the previous iterate next to every wall).
struct StateHeader {
  uint64_t magic;
  int32_t dim, n0, n1, n2, Kpad, precision;
  int64_t fluid;
  uint64_t fingerprint;
};
constexpr uint64_t kMagic = 0x31504d56444d4150ull;

std::vector<int> face_layers(const Problem &P, int a) {
  std::vector<int> r;
  for (int v : {0, 1, P.n[a] - 2, P.n[a] - 1})
    if (v >= 0 && v < P.n[a] && std::find(r.begin(), r.end(), v) == r.end()) r.push_back(v);
  return r;
}

// Velocity slots per voxel at a precision: each octant's Ko slots padded to a
// 128-byte line.
int64_t kpad_of(const Problem &P, int precision) {
  const int line = precision == PDVM_FP64 ? 16 : 32;
  return (int64_t)((P.Ko + line - 1) / line * line) << P.dim;
}

size_t state_bytes(const Problem &P, int precision) {
  const size_t es = precision == PDVM_FP64 ? 8 : 4;
  const size_t N = (size_t)P.N;
  const size_t kp = (size_t)kpad_of(P, precision);
  const size_t nq = P.prandtl > 0 ? 4 * N : 0;  // srcq
  size_t b = sizeof(StateHeader) + sizeof(Ctl) + N * 8 + 3 * N * 8 + N * kSrcStride * es + N * es + nq * es + N * 6 * es;
  if (P.spec > 0) return b + N * kp * es;
  for (int a = 0; a < P.dim; ++a) b += face_layers(P, a).size() * (N / P.n[a]) * kp * es;
  return b;
}
size_t state_bytes(const Problem &P) { return state_bytes(P, P.precision); }

// A checkpoint written at the other sweep precision, converted value by value
// (FP32 -> FP64 is exact). Everything after the FP64 moments is stored in the
// sweep precision, and the face layers also in that precision's slot layout.
template <typename S, typename D>
void convert_sections(const Problem &P, const char *in, char *out, int64_t kin, int64_t kout) {
  const size_t N = (size_t)P.N;
  const S *a = reinterpret_cast<const S *>(in);
  D *b = reinterpret_cast<D *>(out);
  const size_t flat = N * kSrcStride + N + (P.prandtl > 0 ? 4 * N : 0) + N * 6;  // src, srct, srcq, wall
  for (size_t i = 0; i < flat; ++i) b[i] = (D)a[i];
  a += flat;
  b += flat;
  const int64_t kin_o = kin >> P.dim, kout_o = kout >> P.dim;
  size_t cells = 0;
  if (P.spec > 0) cells = N;
  else
    for (int ax = 0; ax < P.dim; ++ax) cells += face_layers(P, ax).size() * (N / P.n[ax]);
  for (size_t c = 0; c < cells; ++c, a += kin, b += kout) {
    for (int64_t k = 0; k < kout; ++k) b[k] = D(0);
    for (int o = 0; o < (1 << P.dim); ++o)
      for (int q = 0; q < P.Ko; ++q) b[o * kout_o + q] = (D)a[o * kin_o + q];
  }
}

std::vector<char> convert_state(const Problem &P, const char *buf, int from) {
  std::vector<char> out(state_bytes(P));
  const size_t head = sizeof(StateHeader) + sizeof(Ctl) + (size_t)P.N * 8 * 4;
  std::memcpy(out.data(), buf, head);
  StateHeader h;
  std::memcpy(&h, buf, sizeof(h));
  h.precision = P.precision;
  h.Kpad = (int32_t)P.Kpad;
  std::memcpy(out.data(), &h, sizeof(h));
  if (from == PDVM_FP64)
    convert_sections<double, float>(P, buf + head, out.data() + head, kpad_of(P, from), P.Kpad);
  else
    convert_sections<float, double>(P, buf + head, out.data() + head, kpad_of(P, from), P.Kpad);
  return out;
}

template <typename T>
int state_io(pdvm_solver *s, int i, char *buf, bool save) {
  const Problem &P = s->P[i];
  Geo<T> &g = geos<T>(s)[i];
  const size_t N = (size_t)P.N;
  int rc = read_ctl(s);
  if (rc != PDVM_OK) return rc;
  const int par = s->host_ctl[i].par;
  char *p = buf + sizeof(StateHeader) + sizeof(Ctl);
  auto xfer = [&](void *dev, size_t bytes) -> int {
    hipError_t e = save ? hipMemcpyAsync(p, dev, bytes, hipMemcpyDeviceToHost, s->stream)
                        : hipMemcpyAsync(dev, p, bytes, hipMemcpyHostToDevice, s->stream);
    p += bytes;
    return e == hipSuccess ? PDVM_OK : s->fail(PDVM_E_HIP, "state copy: %s", hipGetErrorString(e));
  };
  if ((rc = xfer(g.rho[par], N * 8))) return rc;
  if ((rc = xfer(g.u[par], 3 * N * 8))) return rc;
  if ((rc = xfer(g.src[par], N * kSrcStride * sizeof(T)))) return rc;
  if ((rc = xfer(g.srct[par], N * sizeof(T)))) return rc;
  if (P.prandtl > 0 && (rc = xfer(g.srcq[par], 4 * N * sizeof(T)))) return rc;
  if ((rc = xfer(g.wall[par], N * 6 * sizeof(T)))) return rc;
  if (P.spec > 0) {
    if ((rc = xfer(g.h[par], N * (size_t)P.Kpad * sizeof(T)))) return rc;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return PDVM_OK;
  }
  T *stage = g.h[par ^ 1];  // free between iterations
  for (int a = 0; a < P.dim; ++a)
    for (int r : face_layers(P, a)) {
      const size_t bytes = (N / P.n[a]) * (size_t)P.Kpad * sizeof(T);
      if (save) {
        HIPCHK(s, launch_face_copy<T>(g, a, r, stage, 1, s->stream));
        if ((rc = xfer(stage, bytes))) return rc;
      } else {
        if ((rc = xfer(stage, bytes))) return rc;
        HIPCHK(s, launch_face_copy<T>(g, a, r, stage, 0, s->stream));
      }
      HIPCHK(s, hipStreamSynchronize(s->stream));
    }
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return PDVM_OK;
}

int get_state_one(pdvm_solver *s, int i, void *buf, size_t *bytes) {
  const Problem &P = s->P[i];
  const size_t need = state_bytes(P);
  if (!buf) { *bytes = need; return PDVM_OK; }
  if (*bytes < need) return s->fail(PDVM_E_STATE, "state buffer needs %zu bytes", need);
  int rc = read_ctl(s);
  if (rc != PDVM_OK) return rc;
  StateHeader h{kMagic, P.dim, P.n[0], P.n[1], P.n[2], P.Kpad, P.precision, P.fluid, P.fingerprint};
  std::memcpy(buf, &h, sizeof(h));
  std::memcpy((char *)buf + sizeof(h), &s->host_ctl[i], sizeof(Ctl));
  rc = s->precision == PDVM_FP64 ? state_io<double>(s, i, (char *)buf, true) : state_io<float>(s, i, (char *)buf, true);
  *bytes = need;
  return rc;
}

int set_state_one(pdvm_solver *s, int i, const void *buf, size_t bytes) {
  const Problem &P = s->P[i];
  StateHeader h;
  if (bytes < sizeof(h)) return s->fail(PDVM_E_STATE, "state too short");
  std::memcpy(&h, buf, sizeof(h));
  const int from = h.precision == PDVM_FP32 ? PDVM_FP32 : PDVM_FP64;
  const size_t need = state_bytes(P, from);
  if (bytes != need) return s->fail(PDVM_E_STATE, "state has %zu bytes, this problem needs %zu", bytes, need);
  if (h.magic != kMagic || h.dim != P.dim || h.n0 != P.n[0] || h.n1 != P.n[1] || h.n2 != P.n[2] ||
      h.Kpad != kpad_of(P, from) || (h.precision != PDVM_FP64 && h.precision != PDVM_FP32) || h.fluid != P.fluid ||
      h.fingerprint != P.fingerprint)
    return s->fail(PDVM_E_STATE, "state belongs to a different problem");
  std::vector<char> conv;
  if (from != P.precision) {
    conv = convert_state(P, (const char *)buf, from);
    buf = conv.data();
  }
  Ctl c;
  std::memcpy(&c, (const char *)buf + sizeof(h), sizeof(Ctl));
  int rc = read_ctl(s);
  if (rc != PDVM_OK) return rc;
  c.par = s->host_ctl[i].par;  // restore into this solver's current buffers
  c.stop = 1;
  c.fault = 0;
  if (c.status == -3) c.status = 0;
  s->host_ctl[i] = c;
  HIPCHK(s, hipMemcpyAsync(dev_ctl(s, i), &s->host_ctl[i], sizeof(Ctl), hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return s->precision == PDVM_FP64 ? state_io<double>(s, i, (char *)buf, false)
                                   : state_io<float>(s, i, (char *)buf, false);
}

int single(pdvm_solver *s) {
  if (!s) { set_thread_error("solver is NULL"); return PDVM_E_INVAL; }
  if (s->n() != 1) return s->fail(PDVM_E_INVAL, "this call needs a single-problem solver (use the pdvm_batch_* calls)");
  return PDVM_OK;
}

}  // namespace

extern "C" {

int pdvm_halfrange_gh(int32_t n_total, double *nodes, double *weights) { return halfrange_gh(n_total, nodes, weights); }

size_t pdvm_workspace_bytes(const pdvm_config *cfg) {
  Problem P;
  std::string err;
  if (validate_and_build(cfg, P, err) != PDVM_OK) {
    g_thread_error = err;
    return 0;
  }
  return layout_bytes(P);
}

int pdvm_create(const pdvm_config *cfg, void *dev_workspace, size_t ws_bytes, void *hip_stream, pdvm_solver **out) {
  return create_common(cfg, 1, dev_workspace, ws_bytes, hip_stream, out);
}

int pdvm_set_initial(pdvm_solver *s, const double *rho, const double *u) {
  int rc = single(s);
  return rc != PDVM_OK ? rc : set_initial_one(s, 0, rho, u);
}

int pdvm_iterate(pdvm_solver *s, int64_t max_iters, double tol, int32_t stop_mode, pdvm_stats *out) {
  int rc = single(s);
  return rc != PDVM_OK ? rc : iterate_batch(s, max_iters, tol, stop_mode, out);
}

int pdvm_iterate_noalloc(pdvm_solver *s, int64_t max_iters, double tol, int32_t stop_mode, pdvm_stats *out) {
  int rc = single(s);
  return rc != PDVM_OK ? rc : iterate_noalloc(s, max_iters, tol, stop_mode, out);
}

int pdvm_get_moments(pdvm_solver *s, double *rho, double *u, double *tau, double *q) {
  int rc = single(s);
  return rc != PDVM_OK ? rc : get_moments_one(s, 0, rho, u, tau, q);
}

int pdvm_get_flux(pdvm_solver *s, double *gp, double *k, double *gp_section) {
  int rc = single(s);
  return rc != PDVM_OK ? rc : get_flux_one(s, 0, gp, k, gp_section);
}

int pdvm_get_state(pdvm_solver *s, void *buf, size_t *bytes) {
  int rc = single(s);
  if (rc != PDVM_OK) return rc;
  if (!bytes) return s->fail(PDVM_E_INVAL, "bytes is NULL");
  return get_state_one(s, 0, buf, bytes);
}

int pdvm_set_state(pdvm_solver *s, const void *buf, size_t bytes) {
  int rc = single(s);
  if (rc != PDVM_OK) return rc;
  if (!buf) return s->fail(PDVM_E_INVAL, "buf is NULL");
  return set_state_one(s, 0, buf, bytes);
}

int pdvm_batch_create(int32_t n, const pdvm_config *cfgs, void *hip_stream, pdvm_solver **out) {
  return create_common(cfgs, n, nullptr, 0, hip_stream, out);
}

int32_t pdvm_batch_size(const pdvm_solver *s) { return s ? (int32_t)s->P.size() : 0; }

int pdvm_batch_set_initial(pdvm_solver *s, int32_t i, const double *rho, const double *u) {
  int rc = check_index(s, i);
  return rc != PDVM_OK ? rc : set_initial_one(s, i, rho, u);
}

int pdvm_batch_iterate(pdvm_solver *s, int64_t max_iters, double tol, int32_t stop_mode, pdvm_stats *out) {
  if (!s) { set_thread_error("solver is NULL"); return PDVM_E_INVAL; }
  return iterate_batch(s, max_iters, tol, stop_mode, out);
}

int pdvm_batch_get_moments(pdvm_solver *s, int32_t i, double *rho, double *u, double *tau, double *q) {
  int rc = check_index(s, i);
  return rc != PDVM_OK ? rc : get_moments_one(s, i, rho, u, tau, q);
}

int pdvm_batch_get_flux(pdvm_solver *s, int32_t i, double *gp, double *k, double *gp_section) {
  int rc = check_index(s, i);
  return rc != PDVM_OK ? rc : get_flux_one(s, i, gp, k, gp_section);
}

int pdvm_time_kernels(pdvm_solver *s, int32_t iters, pdvm_timing *out) {
  if (!s || !out || iters <= 0) { set_thread_error("bad arguments"); return PDVM_E_INVAL; }
  int rc = check_not_poisoned(s);
  if (rc != PDVM_OK) return rc;
  rc = arm(s, 0.0, 0, 2 * (int64_t)iters + 1);
  if (rc != PDVM_OK) return rc;
  const bool f64 = s->precision == PDVM_FP64;
  const int nd = (s->rows || s->strips || s->queue) ? 1 : (f64 ? s->bd.ndiag_max : s->bf.ndiag_max);
  auto sweep_launch = [&](int d) {
    if (s->queue) return f64 ? launch_sweep_queue<double>(s->bd, s->stream) : launch_sweep_queue<float>(s->bf, s->stream);
    if (s->strips) return f64 ? launch_sweep_strips<double>(s->bd, s->stream) : launch_sweep_strips<float>(s->bf, s->stream);
    if (s->rows)
      return f64 ? launch_sweep_rows<double>(s->bd, s->rows_local, s->stream)
                 : launch_sweep_rows<float>(s->bf, s->rows_local, s->stream);
    return f64 ? launch_sweep<double>(s->bd, d, s->stream) : launch_sweep<float>(s->bf, d, s->stream);
  };
  auto mom_launch = [&]() { return f64 ? launch_moments<double>(s->bd, s->stream) : launch_moments<float>(s->bf, s->stream); };
  auto red_launch = [&]() { return f64 ? launch_reduce<double>(s->bd, s->stream) : launch_reduce<float>(s->bf, s->stream); };
  std::vector<hipEvent_t> ev(2 * (size_t)nd + 4, nullptr);
  for (auto &e : ev) HIPCHK(s, hipEventCreate(&e));
  auto cleanup = [&]() { for (auto &e : ev) if (e) (void)hipEventDestroy(e); };
  double sweep_seq = 0, sweep_kern = 0, mom = 0, red = 0, tot = 0;
  int launches = 0;
  if (s->rows || s->strips || s->queue) launches = 1;
  else
    for (int d = 0; d < nd; ++d) launches += s->h_item_off[(size_t)d * (s->n() + 1) + s->n()] > 0;
  hipError_t e = hipSuccess;
  // pass 1: an event pair around every launch (kernel durations)
  for (int it = 0; it < iters && e == hipSuccess; ++it) {
    for (int d = 0; d < nd && e == hipSuccess; ++d) {
      e = hipEventRecord(ev[2 * d], s->stream);
      if (e == hipSuccess) e = sweep_launch(d);
      if (e == hipSuccess) e = hipEventRecord(ev[2 * d + 1], s->stream);
    }
    if (e == hipSuccess) e = hipEventRecord(ev[2 * nd], s->stream);
    if (e == hipSuccess) e = mom_launch();
    if (e == hipSuccess) e = hipEventRecord(ev[2 * nd + 1], s->stream);
    if (e == hipSuccess) e = red_launch();
    if (e == hipSuccess) e = hipEventRecord(ev[2 * nd + 2], s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev[2 * nd + 2]);
    for (int d = 0; d < nd && e == hipSuccess; ++d) {
      float a = 0;
      e = hipEventElapsedTime(&a, ev[2 * d], ev[2 * d + 1]);
      sweep_kern += a;
    }
    float b = 0, c = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[2 * nd], ev[2 * nd + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&c, ev[2 * nd + 1], ev[2 * nd + 2]);
    mom += b;
    red += c;
  }
  // pass 2: the whole sweep sequence and the whole iteration, as replayed
  for (int it = 0; it < iters && e == hipSuccess; ++it) {
    e = hipEventRecord(ev[0], s->stream);
    for (int d = 0; d < nd && e == hipSuccess; ++d) e = sweep_launch(d);
    if (e == hipSuccess) e = hipEventRecord(ev[1], s->stream);
    if (e == hipSuccess) e = mom_launch();
    if (e == hipSuccess) e = red_launch();
    if (e == hipSuccess) e = hipEventRecord(ev[2], s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev[2]);
    float a = 0, b = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&a, ev[0], ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[0], ev[2]);
    sweep_seq += a;
    tot += b;
  }
  cleanup();
  if (e != hipSuccess) return s->fail(PDVM_E_HIP, "kernel timing: %s", hipGetErrorString(e));
  rc = read_ctl(s);
  if (rc != PDVM_OK) return rc;
  for (int i = 0; i < s->n(); ++i)
    if (s->host_ctl[i].fault)
      return s->fail(PDVM_E_HIP, "problem %d: a %s sweep was abandoned during timing; the previous state is kept", i,
                     sweep_name(s));
  const double es = f64 ? 8.0 : 4.0;
  double fluid = 0, vel = 0;
  for (auto &P : s->P) {
    fluid += (double)P.fluid;
    vel = (double)(P.Ko << P.dim);
  }
  out->sweep_ms_per_iter = sweep_seq / iters;
  out->moments_ms_per_iter = mom / iters;
  out->iter_ms = tot / iters;
  out->sweep_launches_per_iter = launches;
  out->sweep_ms_per_launch = sweep_kern / iters / std::max(1, launches);
  out->moments_ms_per_launch = mom / iters;
  out->reduce_ms_per_launch = red / iters;
  out->fluid_cells = fluid;
  out->velocities = vel;
  out->sweep_bytes_per_iter = es * fluid * vel;
  out->moments_bytes_per_iter = es * fluid * vel;
  return PDVM_OK;
}

int32_t pdvm_sweep_schedule(const pdvm_solver *s) {
  if (!s) return -1;
  return s->queue ? (s->columns ? 5 : 4) : (s->strips ? 3 : (s->rows ? (s->rows_local ? 2 : 1) : 0));
}

int pdvm_set_wait_limit(pdvm_solver *s, double seconds) {
  if (!s) { set_thread_error("solver is NULL"); return PDVM_E_INVAL; }
  if (!(seconds >= 0 && seconds <= 3600)) return s->fail(PDVM_E_INVAL, "wait limit must be in [0, 3600] seconds");
  int khz = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      khz <= 0)
    khz = 100000;
  const int64_t ticks = (int64_t)(seconds * 1000.0 * khz);
  for (int i = 0; i < s->n(); ++i) {
    size_t off;
    int64_t *host;
    const void *dgeo;
    if (s->precision == PDVM_FP64) {
      s->gd[i].wait_ticks = ticks;
      host = &s->gd[i].wait_ticks;
      dgeo = s->bd.d_geo + i;
      off = offsetof(Geo<double>, wait_ticks);
    } else {
      s->gf[i].wait_ticks = ticks;
      host = &s->gf[i].wait_ticks;
      dgeo = s->bf.d_geo + i;
      off = offsetof(Geo<float>, wait_ticks);
    }
    HIPCHK(s, hipMemcpyAsync((char *)dgeo + off, host, sizeof(int64_t), hipMemcpyHostToDevice, s->stream));
  }
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return PDVM_OK;
}

void pdvm_destroy(pdvm_solver *s) {
  if (!s) return;
  if (s->graph) (void)hipGraphExecDestroy(s->graph);
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (auto &d : s->D)
    if (d.own_ws && d.ws) (void)hipFree(d.ws);
  if (s->meta) (void)hipFree(s->meta);
  if (s->qmem) (void)hipFree(s->qmem);
  if (s->host_ctl) (void)hipHostFree(s->host_ctl);
  if (s->own_stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

const char *pdvm_last_error(const pdvm_solver *s) {
  if (s) return s->err.c_str();
  return g_thread_error.c_str();
}

}  // extern "C"
