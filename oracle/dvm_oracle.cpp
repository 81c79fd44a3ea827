// Plain FP64 CPU oracle for the discrete-velocity solve of the steady linearised
// BGK equation on a voxelised porous geometry.
//
// TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark load this file's library. It shares no code,
// header, table or helper with the GPU path; it is written from the paper's
// definitions alone, in the paper's order and notation, with no blocking,
// fusion or reordering beyond what the definitions state.
//
// What it computes (paper section in brackets):
//   * model: v . grad h = nu [ rho + 2 u.v (+ tau(|v|^2 - 3/2)) - h ],
//     nu = sqrt(pi) / (2 Kn)                       [Sec. 2.1, Eq. linearised_Boltzmann_equation]
//   * moments rho, u, tau by quadrature             [Sec. 2.1, Eq. perturbed_quantities]
//   * diffuse wall (alpha = 1) with the wall density from zero mass flux
//                                                   [Sec. 2.1, Eqs. diffusive-specular_BC, wall_density]
//   * periodic pressure-jump inlet/outlet along x1 [Sec. 2.1, Eq. periodic_BC]
//   * specular ("symmetric") lateral faces          [Sec. 2.1, Eq. symmetric_BC]
//   * upwind finite differences, 2nd order, 1st order when the first upstream
//     point is a boundary (solid) point             [Sec. 2.3, Eq. numerical stencil]
//   * iteration: (i) sweep each discrete velocity by forward substitution in
//     the raster order set by the velocity's sign octant, with fluid upstream
//     values from the current sweep and boundary values from the previous
//     iteration; (ii) boundary data; (iii) moments and wall densities
//                                                   [Sec. 3.1, steps (i)-(iii), Algorithm 1]
//   * permeability k = (2/sqrt(pi)) Kn G_p and the 100-iteration convergence
//     criterion Err(l)                              [Sec. 2.1, Eq. k_Gp; Sec. 3.1 steps (iv)-(v),
//                                                    Eq. convergence_criterion]
//
// Readings taken where the paper is silent (each listed in the design notes):
//   voxel-centred nodes x_a = (i_a + 1/2)/N1, period N1 along x1, jump J = 1;
//   the specular plane is the outer voxel face (mirror node -c-1 / 2N-1-c);
//   first order when the immediate upstream image is solid (stencil_rule 0) or
//   when either upstream image is solid (stencil_rule 1);
//   wall density of the solid met by a stencil along axis j with upwind sign s
//   is taken from the fluid node next to it in the +s direction, with the
//   quadrature sum D_j = sum_{v_j>0} W v_j as denominator;
//   isothermal source (the tau term is dropped unless tau_feedback);
//   in 2D with tau_feedback the v3-integrated equation needs a second reduced
//   function psi = int (v3^2 - 1/2) h exp(-v3^2)/sqrt(pi) dv3, with source
//   tau/2, wall value 0 (a diffuse wall emits a v3-Maxwellian) and no jump
//   at the x1 wrap (the jump is v3-independent); phi (the reduced h) then
//   has the source tau (v1^2 + v2^2 - 1), and tau takes int W psi;
//   optional Shakhov model (a kinetic model the method extends to, Sec. 1
//   and Sec. 2.1): the source gains (4/5)(1 - Pr) q.v (|v|^2 - 5/2), with
//   the heat flux q = int v (|v|^2 - 5/2) h lagged like rho, u and tau, so
//   that the collision relaxes q at the rate Pr nu instead of nu; reduced
//   over v3 in 2D this is (4/5)(1 - Pr) q.v (v1^2 + v2^2 - 2) for phi and
//   (2/5)(1 - Pr) q.v for psi;
//   optional Maxwell walls with accommodation alpha < 1 (Eq.
//   diffusive-specular_BC): the wall value becomes alpha times the diffuse
//   value plus (1 - alpha) times the previous iteration's value at the fluid
//   node next to the wall (the node itself, as walls enter only through the
//   first-order stencil of stencil_rule 1) for the velocity mirrored in the
//   wall normal e_j; the wall density keeps its zero-mass-flux value;
//   residual r = max|u^l - u^(l-1)| / max|u^l| over fluid cells and components.
//
// Velocity order inside this file: k = a + n1 (b + n2 c) over the tensor grid
// of the given 1D node lists (ascending). Nothing outside depends on it.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdlib>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

struct Oracle {
  int dim = 2;
  int n[3] = {1, 1, 1};
  long N = 0;
  std::vector<uint8_t> solid;
  int nv[3] = {1, 1, 1};
  std::vector<double> xi[3], om[3];
  int K = 0;
  std::vector<double> v[3];  // v[j][k]
  std::vector<double> W;     // W[k]
  std::vector<int> mirror[3];
  double D[3] = {0, 0, 0};   // D_j = sum_{v_j > 0} W v_j
  double kn = 1.0, nu = 0.0, J = 1.0;
  int lateral_periodic = 0, tau_fb = 0, nthreads = 1;
  double prandtl = 0.0;  // > 0: Shakhov model with this Prandtl number (needs tau_fb)
  double alpha = 1.0;    // wall accommodation; < 1 keeps the previous iteration's h (and psi)
  std::vector<double> hold, psiold;  // [k * N + c] when alpha < 1
  double shakhov_coef() const { return prandtl > 0 ? 0.8 * (1.0 - prandtl) : 0.0; }
  // 0: first order iff the first upstream image is solid (a solid second
  //    upstream image enters the second-order stencil with its wall value);
  // 1: first order iff either upstream image is solid.
  int stencil_rule = 1;

  // lagged state (per cell; solid entries stay 0)
  std::vector<double> rho, tau;
  std::vector<double> u[3], q[3];
  std::vector<double> phi[3][2];  // [j][0]: v_j > 0 half-flux, [j][1]: v_j < 0
  // boundary store: per axis, 4 layers {0, 1, N-2, N-1} of the previous
  // iteration's h, all velocities: hbc[a][slot][facecell * K + k]
  std::vector<double> hbc[3][4];
  std::vector<double> psibc[3][4];  // the same layers of psi (2D with tau_fb)
  bool has_psi() const { return dim == 2 && tau_fb; }

  long iters_done = 0;
  double last_r = 0.0, last_err = -1.0, last_k = 0.0, last_gp = 0.0;
  std::vector<double> kring;  // k at multiples of 100 (index l/100)

  long idx(int i, int j, int l) const { return i + (long)n[0] * (j + (long)n[1] * l); }
  long face_count(int a) const { return N / n[a]; }
  long face_index(int a, const int c[3]) const {
    if (a == 0) return c[1] + (long)n[1] * c[2];
    if (a == 1) return c[0] + (long)n[0] * c[2];
    return c[0] + (long)n[0] * c[1];
  }
  static int slot_of(int r, int na) { return r <= 1 ? r : r - na + 4; }
};

struct Image {
  int r;        // real coordinate along the axis
  int mirrored; // 1 if reached through a specular face
  int jump;     // +1 / -1 / 0 multiples of J added to every value there
};

// Image of coordinate c (outside [0, N_a)) along axis a. [Eqs. periodic_BC, symmetric_BC]
Image image_of(const Oracle &o, int a, int c) {
  Image im{c, 0, 0};
  const int na = o.n[a];
  if (a == 0) {
    if (c < 0) { im.r = c + na; im.jump = +1; }
    else       { im.r = c - na; im.jump = -1; }
  } else if (o.lateral_periodic) {
    im.r = ((c % na) + na) % na;
  } else {
    im.r = c < 0 ? -c - 1 : 2 * na - 1 - c;
    im.mirrored = 1;
  }
  return im;
}

// Value of upstream node m (1 or 2) of fluid node x along axis j for velocity k.
// Returns via *is_solid whether the image is solid. hk holds the current sweep.
double upstream_value(const Oracle &o, const int x[3], int j, int m, int k,
                      const double *hk, int *is_solid, bool psi = false) {
  const int s = o.v[j][k] > 0 ? 1 : -1;
  int y[3] = {x[0], x[1], x[2]};
  y[j] -= m * s;
  int yr[3] = {y[0], y[1], y[2]};
  Image im{y[j], 0, 0};
  const bool ghost = (y[j] < 0 || y[j] >= o.n[j]);
  if (ghost) { im = image_of(o, j, y[j]); yr[j] = im.r; }
  const long cy = o.idx(yr[0], yr[1], yr[2]);
  if (o.solid[cy]) {
    *is_solid = 1;
    // specular part (alpha < 1): the previous iteration's value at the fluid
    // node x_f = y + s e_j (= x, m = 1) for the velocity mirrored in e_j
    // [Eq. diffusive-specular_BC]
    double spec = 0.0;
    if (o.alpha < 1.0) {
      const int km = o.mirror[j][k];
      spec = (1.0 - o.alpha) * (psi ? o.psiold : o.hold)[(size_t)km * o.N + o.idx(x[0], x[1], x[2])];
    }
    if (psi) return spec;  // the diffuse wall emits a Maxwellian in v3: psi = 0
    // wall value: wall density of the solid seen along s e_j, from the fluid
    // node x_f = y + s e_j next to it. [Eq. wall_density]
    int f[3] = {y[0], y[1], y[2]};
    f[j] += s;
    int fr[3] = {f[0], f[1], f[2]};
    Image fi{f[j], 0, 0};
    if (f[j] < 0 || f[j] >= o.n[j]) { fi = image_of(o, j, f[j]); fr[j] = fi.r; }
    const long cf = o.idx(fr[0], fr[1], fr[2]);
    // incoming molecules at that wall have s v_j < 0; a mirror flips v_j
    int incoming_pos = (s < 0);            // v_j > 0 is incoming when s = -1
    if (fi.mirrored) incoming_pos = !incoming_pos;
    const double flux = o.phi[j][incoming_pos ? 0 : 1][cf];
    return o.alpha * (flux / o.D[j] + fi.jump * o.J) + spec;
  }
  *is_solid = 0;
  if (!ghost) return hk[cy];
  // lagged boundary data from the previous iteration [Sec. 3.1 step (ii)]
  const int kk = im.mirrored ? o.mirror[j][k] : k;
  const int sl = Oracle::slot_of(im.r, o.n[j]);
  if (psi) return o.psibc[j][sl][o.face_index(j, yr) * o.K + kk];  // no jump for psi
  return o.hbc[j][sl][o.face_index(j, yr) * o.K + kk] + im.jump * o.J;
}

// Source term S_k(x) = rho + 2 u.v_k (+ tau(|v_k|^2 - 3/2)). [Eq. linearised_Boltzmann_equation]
// In 2D |v|^2 - 3/2 integrates over v3 to v1^2 + v2^2 - 1.
// Shakhov: + (4/5)(1 - Pr) q.v_k (|v_k|^2 - 5/2), in 2D (v1^2 + v2^2 - 2).
double source(const Oracle &o, long c, int k) {
  double S = o.rho[c];
  for (int j = 0; j < o.dim; ++j) S += 2.0 * o.u[j][c] * o.v[j][k];
  if (o.tau_fb) {
    double v2 = 0;
    for (int j = 0; j < o.dim; ++j) v2 += o.v[j][k] * o.v[j][k];
    S += o.tau[c] * (o.dim == 2 ? v2 - 1.0 : v2 - 1.5);
    if (o.prandtl > 0) {
      double qv = 0;
      for (int j = 0; j < o.dim; ++j) qv += o.q[j][c] * o.v[j][k];
      S += o.shakhov_coef() * qv * (o.dim == 2 ? v2 - 2.0 : v2 - 2.5);
    }
  }
  return S;
}

// Source of psi (2D with tau_fb): int (v3^2 - 1/2) S exp(-v3^2)/sqrt(pi) dv3
// = tau / 2 (+ (1/2)(4/5)(1 - Pr) q.v_k for Shakhov).
double psi_source(const Oracle &o, long c, int k) {
  double S = 0.5 * o.tau[c];
  if (o.prandtl > 0) {
    double qv = 0;
    for (int j = 0; j < o.dim; ++j) qv += o.q[j][c] * o.v[j][k];
    S += 0.5 * o.shakhov_coef() * qv;
  }
  return S;
}

// Step (i) for one velocity: forward substitution over all fluid nodes in the
// raster order of the velocity's sign octant. [Sec. 3.1 step (i), Eq. Discretised_...]
void sweep_velocity(const Oracle &o, int k, double *hk, bool psi = false) {
  const double inv_dx = (double)o.n[0];
  int sgn[3] = {1, 1, 1};
  for (int j = 0; j < o.dim; ++j) sgn[j] = o.v[j][k] > 0 ? 1 : -1;
  for (int lp = 0; lp < o.n[2]; ++lp) {
    const int l = sgn[2] > 0 ? lp : o.n[2] - 1 - lp;
    for (int jp = 0; jp < o.n[1]; ++jp) {
      const int jj = sgn[1] > 0 ? jp : o.n[1] - 1 - jp;
      for (int ip = 0; ip < o.n[0]; ++ip) {
        const int i = sgn[0] > 0 ? ip : o.n[0] - 1 - ip;
        const long c = o.idx(i, jj, l);
        if (o.solid[c]) continue;
        const int x[3] = {i, jj, l};
        double num = o.nu * (psi ? psi_source(o, c, k) : source(o, c, k));
        double den = o.nu;
        for (int j = 0; j < o.dim; ++j) {
          const double a = std::fabs(o.v[j][k]) * inv_dx;
          int s1 = 0, s2 = 0;
          const double y1 = upstream_value(o, x, j, 1, k, hk, &s1, psi);
          double y2 = 0.0;
          if (!s1) y2 = upstream_value(o, x, j, 2, k, hk, &s2, psi);
          if (s1 || (o.stencil_rule == 1 && s2)) {  // first order: C = (1, -1, 0)/dx
            den += a;
            num += a * y1;
          } else {                                   // second order: C = (1.5, -2, 0.5)/dx
            den += 1.5 * a;
            num += a * (2.0 * y1 - 0.5 * y2);
          }
        }
        hk[c] = num / den;
      }
    }
  }
}

// Cell index of the node whose coordinate along axis a is r and whose other
// coordinates are given by the face index f (the inverse of face_index).
long face_cell(const Oracle &o, int a, int r, long f) {
  int x[3];
  if (a == 0) { x[0] = r; x[1] = (int)(f % o.n[1]); x[2] = (int)(f / o.n[1]); }
  else if (a == 1) { x[1] = r; x[0] = (int)(f % o.n[0]); x[2] = (int)(f / o.n[0]); }
  else { x[2] = r; x[0] = (int)(f % o.n[0]); x[1] = (int)(f / o.n[0]); }
  return o.idx(x[0], x[1], x[2]);
}

}  // namespace

extern "C" {

// Create an oracle problem. nodes/weights: the 1D lists of axis 0, then 1, then
// 2, concatenated (nv[a] entries each; weights normalised to sum 1 per axis).
void *orc_create(int dim, const int *n, const uint8_t *solid, const int *nv,
                 const double *nodes, const double *weights, double kn,
                 double jump, int lateral_periodic, int tau_feedback,
                 int nthreads, int stencil_rule) {
  Oracle *o = new Oracle();
  o->stencil_rule = stencil_rule;
  o->dim = dim;
  for (int a = 0; a < 3; ++a) { o->n[a] = a < dim ? n[a] : 1; o->nv[a] = a < dim ? nv[a] : 1; }
  o->N = (long)o->n[0] * o->n[1] * o->n[2];
  o->solid.assign(solid, solid + o->N);
  int off = 0;
  for (int a = 0; a < dim; ++a) {
    o->xi[a].assign(nodes + off, nodes + off + nv[a]);
    o->om[a].assign(weights + off, weights + off + nv[a]);
    off += nv[a];
  }
  for (int a = dim; a < 3; ++a) { o->xi[a] = {0.0}; o->om[a] = {1.0}; }
  o->K = o->nv[0] * o->nv[1] * o->nv[2];
  for (int a = 0; a < 3; ++a) { o->v[a].resize(o->K); o->mirror[a].resize(o->K); }
  o->W.resize(o->K);
  for (int c3 = 0; c3 < o->nv[2]; ++c3)
    for (int b = 0; b < o->nv[1]; ++b)
      for (int a = 0; a < o->nv[0]; ++a) {
        const int k = a + o->nv[0] * (b + o->nv[1] * c3);
        o->v[0][k] = o->xi[0][a];
        o->v[1][k] = o->xi[1][b];
        o->v[2][k] = o->xi[2][c3];
        o->W[k] = o->om[0][a] * o->om[1][b] * o->om[2][c3];
        o->mirror[0][k] = (o->nv[0] - 1 - a) + o->nv[0] * (b + o->nv[1] * c3);
        o->mirror[1][k] = a + o->nv[0] * ((o->nv[1] - 1 - b) + o->nv[1] * c3);
        o->mirror[2][k] = a + o->nv[0] * (b + o->nv[1] * (o->nv[2] - 1 - c3));
      }
  for (int j = 0; j < dim; ++j) {
    double d = 0;
    for (int k = 0; k < o->K; ++k)
      if (o->v[j][k] > 0) d += o->W[k] * o->v[j][k];
    o->D[j] = d;
  }
  o->kn = kn;
  o->nu = std::isinf(kn) ? 0.0 : std::sqrt(M_PI) / (2.0 * kn);
  o->J = jump;
  o->lateral_periodic = lateral_periodic;
  o->tau_fb = tau_feedback;
  o->nthreads = nthreads > 0 ? nthreads : 1;
  o->rho.assign(o->N, 0.0);
  o->tau.assign(o->N, 0.0);
  for (int j = 0; j < 3; ++j) {
    o->u[j].assign(o->N, 0.0);
    o->q[j].assign(o->N, 0.0);
    o->phi[j][0].assign(o->N, 0.0);
    o->phi[j][1].assign(o->N, 0.0);
  }
  for (int a = 0; a < dim; ++a)
    for (int s = 0; s < 4; ++s) {
      o->hbc[a][s].assign(o->face_count(a) * o->K, 0.0);
      if (o->has_psi()) o->psibc[a][s].assign(o->face_count(a) * o->K, 0.0);
    }
  return o;
}

void orc_destroy(void *h) { delete static_cast<Oracle *>(h); }

// Maxwell walls with accommodation alpha in (0, 1] (1 = diffuse); needs
// stencil_rule 1. Call before orc_set_initial. Returns 0, or -1.
int orc_set_accommodation(void *hh, double alpha) {
  Oracle &o = *static_cast<Oracle *>(hh);
  if (!(alpha > 0 && alpha <= 1) || (alpha < 1 && o.stencil_rule != 1)) return -1;
  o.alpha = alpha;
  if (alpha < 1) {
    o.hold.assign((size_t)o.N * o.K, 0.0);
    if (o.has_psi()) o.psiold.assign((size_t)o.N * o.K, 0.0);
  }
  return 0;
}

// Switch to the Shakhov model with Prandtl number pr (0 < pr; pr = 1 is
// BGK); needs tau_feedback. Call before orc_set_initial. Returns 0, or -1.
int orc_set_shakhov(void *hh, double pr) {
  Oracle &o = *static_cast<Oracle *>(hh);
  if (!o.tau_fb || !(pr > 0)) return -1;
  o.prandtl = pr;
  return 0;
}

int orc_num_velocities(void *h) { return static_cast<Oracle *>(h)->K; }

// Initial state as a local linearised equilibrium of the given fields:
// h = rho + 2 u.v (+ tau(|v|^2-3/2)) everywhere on the boundary layers, and the
// moments / half-fluxes of that h. NULL fields are zero.
void orc_set_initial(void *hh, const double *rho, const double *u, const double *tau) {
  Oracle &o = *static_cast<Oracle *>(hh);
  for (long c = 0; c < o.N; ++c) {
    const bool f = !o.solid[c];
    o.rho[c] = (f && rho) ? rho[c] : 0.0;
    o.tau[c] = (f && tau && o.tau_fb) ? tau[c] : 0.0;
    for (int j = 0; j < o.dim; ++j) o.u[j][c] = (f && u) ? u[j * o.N + c] : 0.0;
    for (int j = 0; j < o.dim; ++j) o.q[j][c] = 0.0;  // the equilibrium carries no heat flux
  }
  // half-fluxes of h = S_k: sum_{+-v_j>0} W |v_j| S_k
  for (long c = 0; c < o.N; ++c)
    for (int j = 0; j < o.dim; ++j) {
      double p = 0, m = 0;
      if (!o.solid[c])
        for (int k = 0; k < o.K; ++k) {
          const double hk = source(o, c, k);
          if (o.v[j][k] > 0) p += o.W[k] * o.v[j][k] * hk;
          else m += o.W[k] * (-o.v[j][k]) * hk;
        }
      o.phi[j][0][c] = p;
      o.phi[j][1][c] = m;
    }
  for (int a = 0; a < o.dim; ++a)
    for (int s = 0; s < 4; ++s) {
      const int r = s <= 1 ? s : o.n[a] - 4 + s;
      if (r < 0 || r >= o.n[a]) continue;
      for (long f = 0; f < o.face_count(a); ++f) {
        const long c = face_cell(o, a, r, f);
        for (int k = 0; k < o.K; ++k) {
          o.hbc[a][s][f * o.K + k] = o.solid[c] ? 0.0 : source(o, c, k);
          // the local equilibrium's psi: tau int (v3^2 - 1/2) v3^2 = tau / 2
          if (o.has_psi()) o.psibc[a][s][f * o.K + k] = o.solid[c] ? 0.0 : psi_source(o, c, k);
        }
      }
    }
  if (o.alpha < 1.0)
    for (int k = 0; k < o.K; ++k)
      for (long c = 0; c < o.N; ++c) {
        o.hold[(size_t)k * o.N + c] = o.solid[c] ? 0.0 : source(o, c, k);
        if (o.has_psi()) o.psiold[(size_t)k * o.N + c] = o.solid[c] ? 0.0 : psi_source(o, c, k);
      }
  o.iters_done = 0;
  o.kring.clear();
}

// Run up to `iters` iterations. stop_mode 0: stop when r <= tol; 1: stop when
// Err(l) < tol at a multiple of 100 iterations; tol <= 0 never stops early.
// stats: [0] iterations done in this call, [1] r, [2] Err (-1 if not yet
// defined), [3] k, [4] G_p. Returns 0 if stopped on tolerance, 1 otherwise.
int orc_iterate(void *hh, long iters, double tol, int stop_mode, double *stats) {
  Oracle &o = *static_cast<Oracle *>(hh);
  const int T = o.nthreads;
  const long N = o.N;
  // rho, phi(+-), sum W|v|^2 h, q, then (2D with tau_fb) sum W psi
  const int nm = 1 + 2 * o.dim + 1 + o.dim + (o.has_psi() ? 1 : 0);
  const int PSI = 2 + 3 * o.dim;  // index of the psi sum
  std::vector<std::vector<double>> acc(T, std::vector<double>((size_t)nm * N));
  std::vector<std::vector<double>> hk(T, std::vector<double>(N));
  std::vector<std::vector<double>> pk(T, std::vector<double>(o.has_psi() ? N : 0));
  std::vector<double> hbc_new[3][4], psibc_new[3][4];
  std::vector<double> hold_new(o.hold.size()), psiold_new(o.psiold.size());
  for (int a = 0; a < o.dim; ++a)
    for (int s = 0; s < 4; ++s) {
      hbc_new[a][s].assign(o.hbc[a][s].size(), 0.0);
      if (o.has_psi()) psibc_new[a][s].assign(o.psibc[a][s].size(), 0.0);
    }
  long done = 0;
  int converged = 0;
  for (long it = 0; it < iters; ++it) {
    for (int t = 0; t < T; ++t) std::fill(acc[t].begin(), acc[t].end(), 0.0);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(T)
#endif
    for (int k = 0; k < o.K; ++k) {
#ifdef _OPENMP
      const int t = omp_get_thread_num();
#else
      const int t = 0;
#endif
      double *h = hk[t].data();
      sweep_velocity(o, k, h);
      double *ps = o.has_psi() ? pk[t].data() : nullptr;
      if (ps) sweep_velocity(o, k, ps, true);
      if (o.alpha < 1.0) {  // the whole iterate, for the next iteration's specular wall values
        std::copy(h, h + N, hold_new.begin() + (size_t)k * N);
        if (ps) std::copy(ps, ps + N, psiold_new.begin() + (size_t)k * N);
      }
      // step (iii): quadrature moments and half-fluxes [Eq. perturbed_quantities]
      double *A = acc[t].data();
      double v2 = 0;
      for (int j = 0; j < o.dim; ++j) v2 += o.v[j][k] * o.v[j][k];
      // reduced 2D distribution: v3 integrated out, which adds 1/2 to |v|^2
      const double vsq = o.dim == 2 ? v2 + 0.5 : v2;
      for (long c = 0; c < N; ++c) {
        if (o.solid[c]) continue;
        const double wh = o.W[k] * h[c];
        A[c] += wh;
        for (int j = 0; j < o.dim; ++j) {
          const double vj = o.v[j][k];
          if (vj > 0) A[(1 + 2 * j) * N + c] += wh * vj;
          else A[(2 + 2 * j) * N + c] += wh * (-vj);
          A[(2 + 2 * o.dim + j) * N + c] += wh * vj * (vsq - 2.5);
        }
        A[(1 + 2 * o.dim) * N + c] += wh * vsq;
        if (ps) {
          const double wp = o.W[k] * ps[c];
          A[PSI * N + c] += wp;
          // q_j gains int v_j v3^2 h = v_j (psi + phi/2); the phi/2 is in vsq
          for (int j = 0; j < o.dim; ++j) A[(2 + 2 * o.dim + j) * N + c] += wp * o.v[j][k];
        }
      }
      // step (ii): keep the boundary layers of h for the next iteration
      for (int a = 0; a < o.dim; ++a)
        for (int s = 0; s < 4; ++s) {
          const int r = s <= 1 ? s : o.n[a] - 4 + s;
          if (r < 0 || r >= o.n[a]) continue;
          for (long f = 0; f < o.face_count(a); ++f) {
            const long c = face_cell(o, a, r, f);
            hbc_new[a][s][f * o.K + k] = o.solid[c] ? 0.0 : h[c];
            if (ps) psibc_new[a][s][f * o.K + k] = o.solid[c] ? 0.0 : ps[c];
          }
        }
    }
    // combine thread partials in thread order
    std::vector<double> M((size_t)nm * N, 0.0);
    for (int t = 0; t < T; ++t)
      for (size_t i = 0; i < M.size(); ++i) M[i] += acc[t][i];
    double max_du = 0, max_u = 0, sum_u1 = 0;
    for (long c = 0; c < N; ++c) {
      if (o.solid[c]) continue;
      o.rho[c] = M[c];
      for (int j = 0; j < o.dim; ++j) {
        const double p = M[(1 + 2 * j) * N + c], m = M[(2 + 2 * j) * N + c];
        const double unew = p - m;
        max_du = std::max(max_du, std::fabs(unew - o.u[j][c]));
        max_u = std::max(max_u, std::fabs(unew));
        o.u[j][c] = unew;
        o.phi[j][0][c] = p;
        o.phi[j][1][c] = m;
        o.q[j][c] = M[(2 + 2 * o.dim + j) * N + c];
      }
      o.tau[c] = (2.0 / 3.0) * M[(1 + 2 * o.dim) * N + c] - (2.0 / 3.0) * 1.5 * M[c];
      if (o.has_psi()) o.tau[c] += (2.0 / 3.0) * M[PSI * N + c];
      sum_u1 += o.u[0][c];
    }
    for (int a = 0; a < o.dim; ++a)
      for (int s = 0; s < 4; ++s) {
        o.hbc[a][s].swap(hbc_new[a][s]);
        if (o.has_psi()) o.psibc[a][s].swap(psibc_new[a][s]);
      }
    o.hold.swap(hold_new);
    o.psiold.swap(psiold_new);
    ++o.iters_done;
    ++done;
    // steps (iv)-(v): G_p as the mean of u1 over all cells (solid = 0), k, r, Err
    const double Gp = sum_u1 / (double)N;
    const double kp = 2.0 / std::sqrt(M_PI) * o.kn * Gp;
    o.last_gp = Gp;
    o.last_k = kp;
    o.last_r = max_u > 0 ? max_du / max_u : max_du;
    if (o.iters_done % 100 == 0) {
      o.kring.push_back(kp);
      const size_t m = o.kring.size();
      if (m >= 2 && kp != 0.0)
        o.last_err = std::fabs((o.kring[m - 1] - o.kring[m - 2]) / kp) / 100.0;
    }
    if (tol > 0) {
      if (stop_mode == 0 && o.last_r <= tol) { converged = 1; break; }
      if (stop_mode == 1 && o.iters_done % 100 == 0 && o.last_err >= 0 && o.last_err < tol) {
        converged = 1;
        break;
      }
    }
  }
  if (stats) {
    stats[0] = (double)done;
    stats[1] = o.last_r;
    stats[2] = o.last_err;
    stats[3] = o.last_k;
    stats[4] = o.last_gp;
  }
  return converged ? 0 : 1;
}

// Moments at every cell (solid cells read 0). tau is the temperature
// perturbation, q the heat flux; 2D uses the reduced forms with v3 integrated
// out. u and q are dim * N, component-major. NULL skips an output.
void orc_get_moments(void *hh, double *rho, double *u, double *tau, double *q) {
  Oracle &o = *static_cast<Oracle *>(hh);
  for (long c = 0; c < o.N; ++c) {
    if (rho) rho[c] = o.rho[c];
    if (tau) tau[c] = o.tau[c];
    for (int j = 0; j < o.dim; ++j) {
      if (u) u[j * o.N + c] = o.u[j][c];
      if (q) q[j * o.N + c] = o.q[j][c];
    }
  }
}

// Half-fluxes phi[(2 j + s) * N + c], s = 0 for v_j > 0, 1 for v_j < 0.
void orc_get_phi(void *hh, double *phi) {
  Oracle &o = *static_cast<Oracle *>(hh);
  for (int j = 0; j < o.dim; ++j)
    for (int s = 0; s < 2; ++s)
      for (long c = 0; c < o.N; ++c) phi[(2 * j + s) * o.N + c] = o.phi[j][s][c];
}

// G_p (mean of u1 over all cells), k = (2/sqrt(pi)) Kn G_p, and optionally the
// per-section G_p(i) = mean over the cross-section at x1 index i.
void orc_get_flux(void *hh, double *Gp, double *kperm, double *Gp_section) {
  Oracle &o = *static_cast<Oracle *>(hh);
  double s = 0;
  for (long c = 0; c < o.N; ++c) s += o.u[0][c];
  if (Gp) *Gp = s / (double)o.N;
  if (kperm) *kperm = 2.0 / std::sqrt(M_PI) * o.kn * (s / (double)o.N);
  if (Gp_section) {
    const long A = o.N / o.n[0];
    for (int i = 0; i < o.n[0]; ++i) {
      double t = 0;
      for (int l = 0; l < o.n[2]; ++l)
        for (int j = 0; j < o.n[1]; ++j) t += o.u[0][o.idx(i, j, l)];
      Gp_section[i] = t / (double)A;
    }
  }
}

// The sweep's own operator, for pinning: for velocity k and a given field f on
// all cells, out(x) = sum_j |v_j| (C0 f(x) + C1 y1 + C2 y2)/dx at fluid x with the
// same image and order rules as the sweep (ghost and wall values from the
// current lagged state). [Eq. numerical stencil]
void orc_apply_advection(void *hh, int k, const double *f, double *out) {
  Oracle &o = *static_cast<Oracle *>(hh);
  const double inv_dx = (double)o.n[0];
  for (long c = 0; c < o.N; ++c) {
    out[c] = 0.0;
    if (o.solid[c]) continue;
    const int x[3] = {(int)(c % o.n[0]), (int)((c / o.n[0]) % o.n[1]), (int)(c / ((long)o.n[0] * o.n[1]))};
    double acc = 0;
    for (int j = 0; j < o.dim; ++j) {
      const double a = std::fabs(o.v[j][k]) * inv_dx;
      int s1 = 0, s2 = 0;
      const double y1 = upstream_value(o, x, j, 1, k, f, &s1);
      double y2 = 0.0;
      if (!s1) y2 = upstream_value(o, x, j, 2, k, f, &s2);
      if (s1 || (o.stencil_rule == 1 && s2)) acc += a * (f[c] - y1);
      else acc += a * (1.5 * f[c] - 2.0 * y1 + 0.5 * y2);
    }
    out[c] = acc;
  }
}

// Collision term nu (S_k - h_k) of a distribution h (K values) at one node:
// the moments of h by quadrature, then the isothermal (or full, with
// tau_feedback, or Shakhov) source, in the full velocity space (3D; in 2D the
// tau and q terms would need psi). [Eqs. linearised_Boltzmann_equation, perturbed_quantities]
void orc_collision(void *hh, const double *h, double *out) {
  Oracle &o = *static_cast<Oracle *>(hh);
  double rho = 0, u[3] = {0, 0, 0}, e = 0;
  for (int k = 0; k < o.K; ++k) {
    rho += o.W[k] * h[k];
    double v2 = 0;
    for (int j = 0; j < o.dim; ++j) { u[j] += o.W[k] * o.v[j][k] * h[k]; v2 += o.v[j][k] * o.v[j][k]; }
    e += o.W[k] * v2 * h[k];
  }
  const double tau = (2.0 / 3.0) * e - rho;
  double q[3] = {0, 0, 0};  // heat flux int v (|v|^2 - 5/2) h
  for (int k = 0; k < o.K; ++k) {
    double v2 = 0;
    for (int j = 0; j < o.dim; ++j) v2 += o.v[j][k] * o.v[j][k];
    for (int j = 0; j < o.dim; ++j) q[j] += o.W[k] * o.v[j][k] * (v2 - 2.5) * h[k];
  }
  for (int k = 0; k < o.K; ++k) {
    double S = rho;
    double v2 = 0, qv = 0;
    for (int j = 0; j < o.dim; ++j) { S += 2.0 * u[j] * o.v[j][k]; v2 += o.v[j][k] * o.v[j][k]; qv += q[j] * o.v[j][k]; }
    if (o.tau_fb) S += tau * (v2 - 1.5);
    if (o.tau_fb && o.prandtl > 0) S += o.shakhov_coef() * qv * (v2 - 2.5);
    out[k] = o.nu * (S - h[k]);
  }
}

// Replace the lagged boundary store by a given full field f (N * K values,
// cell-major, this file's velocity order): used to pin the operator.
void orc_set_boundary_field(void *hh, const double *f) {
  Oracle &o = *static_cast<Oracle *>(hh);
  for (int a = 0; a < o.dim; ++a)
    for (int s = 0; s < 4; ++s) {
      const int r = s <= 1 ? s : o.n[a] - 4 + s;
      if (r < 0 || r >= o.n[a]) continue;
      for (long fi = 0; fi < o.face_count(a); ++fi) {
        const long c = face_cell(o, a, r, fi);
        for (int k = 0; k < o.K; ++k) o.hbc[a][s][fi * o.K + k] = f[c * o.K + k];
      }
    }
}

// Set the lagged half-fluxes directly (same layout as orc_get_phi).
void orc_set_phi(void *hh, const double *phi) {
  Oracle &o = *static_cast<Oracle *>(hh);
  for (int j = 0; j < o.dim; ++j)
    for (int s = 0; s < 2; ++s)
      for (long c = 0; c < o.N; ++c) o.phi[j][s][c] = phi[(2 * j + s) * o.N + c];
}

// Velocity table of this file's order: v (dim * K, component-major) and W (K).
void orc_get_velocities(void *hh, double *v, double *W) {
  Oracle &o = *static_cast<Oracle *>(hh);
  for (int k = 0; k < o.K; ++k) {
    if (W) W[k] = o.W[k];
    for (int j = 0; j < o.dim; ++j)
      if (v) v[j * o.K + k] = o.v[j][k];
  }
}

long orc_iterations(void *hh) { return static_cast<Oracle *>(hh)->iters_done; }

}  // extern "C"
