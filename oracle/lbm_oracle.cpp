// Plain FP64 CPU oracle of the Euler-Lagrange bubble-column method (LBGK + Lagrangian
// particle tracking with two-way coupling) of Agarwal, Ravindra & Prakash, arXiv 1710.07073.
//
// TEST INFRASTRUCTURE ONLY. This file is the slow, obviously-correct reference that the GPU
// path is checked against. Only the test suite, the smoke check and the CPU-baseline leg of the
// benchmark may load it. It shares no code, header, table or helper with the GPU library.
//
// Every function follows the paper step by step, in double precision, with plain loops:
//   * lattice and equilibrium ............. Sec. 2.2, eq. (5)-(9)
//   * macroscopic moments ................. Sec. 2.2, eq. (10), (13)
//   * BGK collision + Guo forcing ......... Sec. 2.2, eq. (11)-(15)
//   * streaming + boundary conditions ..... Sec. 2.2, eq. (16); Sec. 3.3 (boundary conditions)
//   * polynomial mapping kernel ........... Sec. 3.2, eq. (18)-(21)
//   * bubble force closures and ODE ....... Sec. 2.1, eq. (1)-(4), Table 1
//   * the coupled time loop ............... Algorithm 1
// Where the paper is silent or garbled the reading used is stated next to the code (R-numbers
// refer to the list of readings kept with the design notes of this repository).
//
// Storage convention: populations are stored shifted, g_q = f_q - w_q (so a fluid at rest with
// rho = 1 is g = 0). The arithmetic below is the paper's, rewritten in the shifted variables:
// feq_q - w_q = w_q * (drho + rho * [3 c.u + 4.5 (c.u)^2 - 1.5 u.u]) with drho = rho - 1.
// Fields are structure-of-arrays, x fastest: pop[q][z][y][x], vec[a][z][y][x].

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------------------------
// D3Q19 velocity set and weights, eq. (7)-(8), in the paper's order: j = 1..6 the axis
// directions, j = 7..18 the face diagonals, j = 19 the rest particle (0-based here: q = j - 1).
// Lattice speed e = dx/dt = 1 (lattice units).
// ---------------------------------------------------------------------------------------------
const int C[19][3] = {
    {+1, 0, 0}, {-1, 0, 0}, {0, +1, 0}, {0, -1, 0}, {0, 0, +1}, {0, 0, -1},
    {+1, +1, 0}, {-1, +1, 0}, {+1, -1, 0}, {-1, -1, 0},
    {+1, 0, +1}, {-1, 0, +1}, {+1, 0, -1}, {-1, 0, -1},
    {0, +1, +1}, {0, -1, +1}, {0, +1, -1}, {0, -1, -1},
    {0, 0, 0}};

const double W[19] = {1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                      1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                      1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                      1.0 / 3};

// index of the velocity equal to the given integer vector (searched, not tabulated)
int find_q(int cx, int cy, int cz) {
  for (int q = 0; q < 19; ++q)
    if (C[q][0] == cx && C[q][1] == cy && C[q][2] == cz) return q;
  return -1;
}

enum { BC_BOUNCE_BACK = 0, BC_FREE_SLIP = 1, BC_PERIODIC = 2 };

struct Grid {
  int n[3];    // nx, ny, nz
  int bc[6];   // -x, +x, -y, +y, -z, +z
  long cells() const { return (long)n[0] * n[1] * n[2]; }
  long idx(int x, int y, int z) const { return ((long)z * n[1] + y) * n[0] + x; }
  bool periodic(int a) const { return bc[2 * a] == BC_PERIODIC; }
};

bool grid_ok(const Grid& g) {
  for (int a = 0; a < 3; ++a) {
    if (g.n[a] < 1) return false;
    bool plo = g.bc[2 * a] == BC_PERIODIC, phi = g.bc[2 * a + 1] == BC_PERIODIC;
    if (plo != phi) return false;
    for (int s = 0; s < 2; ++s)
      if (g.bc[2 * a + s] < 0 || g.bc[2 * a + s] > 2) return false;
  }
  return true;
}

int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// ---------------------------------------------------------------------------------------------
// Equilibrium, eq. (6), shifted: returns feq_q - w_q for density rho = 1 + drho and velocity u.
// The density deviation drho is passed on its own: forming rho - 1 again would round it to
// the resolution of 1.0 and throw away the benefit of the shifted storage.
// ---------------------------------------------------------------------------------------------
void equilibrium_shifted(double drho, const double u[3], double geq[19]) {
  const double rho = 1.0 + drho;
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int q = 0; q < 19; ++q) {
    const double cu = C[q][0] * u[0] + C[q][1] * u[1] + C[q][2] * u[2];
    geq[q] = W[q] * (drho + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
  }
}

// Guo discrete force term, eq. (12): F_q = (1 - omega/2) w_q [3 (c_q - u) + 9 (c_q.u) c_q] . F
void guo_source(double omega, const double u[3], const double F[3], double S[19]) {
  const double pre = 1.0 - 0.5 * omega;
  for (int q = 0; q < 19; ++q) {
    const double cu = C[q][0] * u[0] + C[q][1] * u[1] + C[q][2] * u[2];
    double s = 0.0;
    for (int a = 0; a < 3; ++a) s += (3.0 * (C[q][a] - u[a]) + 9.0 * cu * C[q][a]) * F[a];
    S[q] = pre * W[q] * s;
  }
}

// One node: first forcing step (13), equilibrium (6), collision (14), second forcing (15).
// g: shifted pre-collision populations; F: body force; out: shifted post-collision populations.
void collide_node(double omega, const double g[19], const double F[3], double out[19],
                  double* rho_out, double u_out[3]) {
  double drho = 0.0, m[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < 19; ++q) {
    drho += g[q];
    for (int a = 0; a < 3; ++a) m[a] += C[q][a] * g[q];
  }
  const double rho = 1.0 + drho;
  double u[3];
  for (int a = 0; a < 3; ++a) u[a] = (m[a] + 0.5 * F[a]) / rho;  // eq. (13)
  double geq[19], S[19];
  equilibrium_shifted(drho, u, geq);
  guo_source(omega, u, F, S);
  for (int q = 0; q < 19; ++q) out[q] = g[q] - omega * (g[q] - geq[q]) + S[q];  // (14), (15)
  if (rho_out) *rho_out = rho;
  if (u_out)
    for (int a = 0; a < 3; ++a) u_out[a] = u[a];
}

// Streaming, eq. (16), written as a gather: the population q arriving at node x comes from
// x - c_q. Periodic axes wrap. A source outside a wall is replaced by the boundary rule:
//   * half-way bounce-back (no-slip wall at the mid-link plane, Sec. 3.3): the population that
//     left x towards the wall returns reversed, f_q(x) = f*_{opp(q)}(x);
//   * free slip (specular reflection, Sec. 3.3, top face): the component normal to the wall is
//     mirrored, f_q(x) = f*_{q'}(x - c_q with the normal coordinate kept), q' = q with that
//     component of c negated; if that mirrored source is itself outside (an edge), bounce-back.
double pull_one(const Grid& G, const double* post, int x, int y, int z, int q) {
  const long N = G.cells();
  int s[3] = {x - C[q][0], y - C[q][1], z - C[q][2]};
  const int p[3] = {x, y, z};
  int out_axes = 0, out_axis = -1, out_side = 0;
  for (int a = 0; a < 3; ++a) {
    if (G.periodic(a)) {
      s[a] = wrap(s[a], G.n[a]);
    } else if (s[a] < 0 || s[a] >= G.n[a]) {
      ++out_axes;
      out_axis = a;
      out_side = s[a] < 0 ? 0 : 1;
    }
  }
  if (out_axes == 0) return post[q * N + G.idx(s[0], s[1], s[2])];
  if (out_axes == 1 && G.bc[2 * out_axis + out_side] == BC_FREE_SLIP) {
    int cm[3] = {C[q][0], C[q][1], C[q][2]};
    cm[out_axis] = -cm[out_axis];
    const int qm = find_q(cm[0], cm[1], cm[2]);
    s[out_axis] = p[out_axis];
    return post[qm * N + G.idx(s[0], s[1], s[2])];
  }
  const int qb = find_q(-C[q][0], -C[q][1], -C[q][2]);
  return post[qb * N + G.idx(x, y, z)];
}

// ---------------------------------------------------------------------------------------------
// Polynomial mapping kernel, eq. (18): Z(r) = 15/16 [r^4/n^5 - 2 r^2/n^3 + 1/n] on |r| <= n
// (the printed numerators lost their exponents; this is the form whose integral is one and
// which vanishes with zero slope at +-n). P is its antiderivative in s = r/n, P(-1)=0, P(1)=1.
// ---------------------------------------------------------------------------------------------
double kernel_Z(double r, double n) {
  if (r < -n || r > n) return 0.0;
  return 15.0 / 16.0 * (std::pow(r, 4) / std::pow(n, 5) - 2.0 * r * r / std::pow(n, 3) + 1.0 / n);
}

double kernel_P(double s) {
  if (s <= -1.0) return 0.0;
  if (s >= 1.0) return 1.0;
  return 0.5 + 15.0 / 16.0 * (s - 2.0 / 3.0 * s * s * s + 0.2 * std::pow(s, 5));
}

// Cell-integral weights along one axis, eq. (19) factorised: w(i) = integral of Z(x - xb) over
// the cell [i - 1/2, i + 1/2]. Cells outside a wall are dropped and the axis is renormalised to a
// sum of one ("clipped"); on a periodic axis the cell index wraps. Returns the count.
// point != 0 selects the point-sampled alternative of the coupling variants: w(i) = Z(i - xb) at
// the cell centre, renormalised to a sum of one on every axis (sampled values of Z do not sum to
// one even without a wall).
int axis_weights(double xb, double n, int N, bool periodic, int* idx, double* w, int cap,
                 bool point = false) {
  const int lo = (int)std::floor(xb - n - 0.5) + 1;
  const int hi = (int)std::ceil(xb + n + 0.5) - 1;
  int k = 0;
  double sum = 0.0;
  for (int i = lo; i <= hi; ++i) {
    const double wi = point ? kernel_Z(i - xb, n)
                            : kernel_P((i + 0.5 - xb) / n) - kernel_P((i - 0.5 - xb) / n);
    int j = i;
    if (periodic) {
      j = wrap(i, N);
    } else if (i < 0 || i >= N) {
      continue;
    }
    if (k >= cap) return -1;
    idx[k] = j;
    w[k] = wi;
    sum += wi;
    ++k;
  }
  if ((!periodic || point) && sum > 0.0)
    for (int m = 0; m < k; ++m) w[m] /= sum;
  if (point && !(sum > 0.0)) return -1;  // no cell centre inside the support
  return k;
}

// Velocity at an arbitrary integer position, with wall ghosts for positions one cell outside:
// bounce-back ghost = -U(mirror cell) (zero velocity on the mid-link wall plane), free-slip
// ghost = U(mirror cell) with the normal component negated, periodic = wrapped.
void velocity_at(const Grid& G, const double* U, int x, int y, int z, double out[3]) {
  const long N = G.cells();
  int p[3] = {x, y, z};
  double sign[3] = {1.0, 1.0, 1.0};
  for (int a = 0; a < 3; ++a) {
    if (G.periodic(a)) {
      p[a] = wrap(p[a], G.n[a]);
    } else if (p[a] < 0 || p[a] >= G.n[a]) {
      const int side = p[a] < 0 ? 0 : 1;
      const int mirror = side == 0 ? -1 - p[a] : 2 * G.n[a] - 1 - p[a];
      p[a] = mirror;
      if (G.bc[2 * a + side] == BC_FREE_SLIP) {
        sign[a] = -sign[a];
      } else {
        for (int b = 0; b < 3; ++b) sign[b] = -sign[b];
      }
    }
  }
  const long c = G.idx(p[0], p[1], p[2]);
  for (int a = 0; a < 3; ++a) out[a] = sign[a] * U[a * N + c];
}

// Curl of U at a cell by central differences (the paper does not state a discretisation).
void curl_at(const Grid& G, const double* U, int x, int y, int z, double w[3]) {
  double xp[3], xm[3], yp[3], ym[3], zp[3], zm[3];
  velocity_at(G, U, x + 1, y, z, xp);
  velocity_at(G, U, x - 1, y, z, xm);
  velocity_at(G, U, x, y + 1, z, yp);
  velocity_at(G, U, x, y - 1, z, ym);
  velocity_at(G, U, x, y, z + 1, zp);
  velocity_at(G, U, x, y, z - 1, zm);
  const double dUz_dy = 0.5 * (yp[2] - ym[2]), dUy_dz = 0.5 * (zp[1] - zm[1]);
  const double dUx_dz = 0.5 * (zp[0] - zm[0]), dUz_dx = 0.5 * (xp[2] - xm[2]);
  const double dUy_dx = 0.5 * (xp[1] - xm[1]), dUx_dy = 0.5 * (yp[0] - ym[0]);
  w[0] = dUz_dy - dUy_dz;
  w[1] = dUx_dz - dUz_dx;
  w[2] = dUy_dx - dUx_dy;
}

}  // namespace

// =============================================================================================
// C interface (ctypes). All arrays are caller-owned, host, double unless stated.
// Return 0 on success, a negative value on bad arguments.
// =============================================================================================
extern "C" {

typedef struct {
  double g;              // gravity magnitude (acts along -z)
  double rho_l;          // liquid density
  double rho_b;          // bubble density
  double sigma;          // surface tension
  double c_a;            // added-mass coefficient (Table 1: 0.5)
  double drag_scale;     // multiplier on F_D
  double lift_scale;     // multiplier on F_L
  double kernel_factor;  // half-width of the mapping window in diameters (Sec. 3.2: 1.5)
  double cd_k;           // constant in 24/Re (1 + k Re^0.687)
  double lift_f0;        // constant term of the lift polynomial f(Eo_d)
  int32_t n_sub;         // bubble sub-steps per liquid step (Table 2: dt_l / dt_b = 10)
  int32_t coupling;      // coupling variant bits, ORC_* below (0 = the default reading)
} orc_bubble_params;

// Coupling variants (readings R3, R13, R16 and their alternatives):
//   reaction (bits 0-1): 0 = -(F_D + F_L) at the updated velocity (Algorithm 1);
//     1 = the mean of -(F_D + F_L) over the sub-steps (the impulse those forces gave the bubble
//     during the liquid step, per unit time); 2 = -sum F, the net force of eq. (1) on the bubble,
//     averaged over the sub-steps (Sec. 3.2 states the reaction as minus the sum of the forces);
//   point-sampled kernel (bit 2): weights Z at cell centres instead of cell integrals;
//   exact time (bit 3): the forward coupling interpolates the velocity of the current state f^n
//     (eq. (10), no force term) instead of the velocity of the previous collision.
enum { ORC_REACTION_MASK = 3, ORC_REACTION_SUBSTEP_MEAN = 1, ORC_REACTION_NET_FORCE = 2,
       ORC_POINT_KERNEL = 4, ORC_EXACT_TIME = 8 };

int orc_lattice(int32_t* c /*19x3*/, double* w /*19*/, int32_t* opp /*19*/) {
  for (int q = 0; q < 19; ++q) {
    for (int a = 0; a < 3; ++a) c[3 * q + a] = C[q][a];
    w[q] = W[q];
    opp[q] = find_q(-C[q][0], -C[q][1], -C[q][2]);
  }
  return 0;
}

void orc_equilibrium(double rho, const double* u, double* feq) {
  double geq[19];
  equilibrium_shifted(rho - 1.0, u, geq);
  for (int q = 0; q < 19; ++q) feq[q] = geq[q] + W[q];
}

void orc_guo_source(double omega, const double* u, const double* F, double* S) {
  guo_source(omega, u, F, S);
}

void orc_collide_node(double omega, const double* g, const double* F, double* out, double* rho,
                      double* u) {
  collide_node(omega, g, F, out, rho, u);
}

double orc_kernel_Z(double r, double n) { return kernel_Z(r, n); }
double orc_kernel_P(double s) { return kernel_P(s); }

int orc_axis_weights(double xb, double n, int N, int periodic, int32_t* idx, double* w, int cap,
                     int point) {
  std::vector<int> tmp(cap > 0 ? cap : 1);
  int k = axis_weights(xb, n, N, periodic != 0, tmp.data(), w, cap, point != 0);
  for (int i = 0; i < k; ++i) idx[i] = tmp[i];
  return k;
}

// One liquid step (Sec. 2.2): collision with forcing at every node, then streaming with the
// boundary conditions. g: state f^n - w (pre-collision), overwritten with f^{n+1} - w.
// F: force density (3 x N, may be null = zero). U_out (3 x N, nullable): the velocity of
// eq. (13) used in the collision. tmp: 19 x N scratch. nthreads <= 0: library default.
int orc_lbm_step(int nx, int ny, int nz, const int32_t* bc, double omega, double* g, double* tmp,
                 const double* F, double* U_out, int nthreads) {
  Grid G{{nx, ny, nz}, {bc[0], bc[1], bc[2], bc[3], bc[4], bc[5]}};
  if (!grid_ok(G)) return -1;
  const long N = G.cells();
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(static)
  for (long c = 0; c < N; ++c) {
    double gi[19], go[19], Fc[3] = {0.0, 0.0, 0.0}, u[3];
    for (int q = 0; q < 19; ++q) gi[q] = g[q * N + c];
    if (F)
      for (int a = 0; a < 3; ++a) Fc[a] = F[a * N + c];
    collide_node(omega, gi, Fc, go, nullptr, u);
    for (int q = 0; q < 19; ++q) tmp[q * N + c] = go[q];
    if (U_out)
      for (int a = 0; a < 3; ++a) U_out[a * N + c] = u[a];
  }
#pragma omp parallel for schedule(static)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        for (int q = 0; q < 19; ++q) g[q * N + G.idx(x, y, z)] = pull_one(G, tmp, x, y, z, q);
  return 0;
}

// Streaming only, eq. (16) with the boundary rules (used by tests of the boundary conditions).
int orc_stream(int nx, int ny, int nz, const int32_t* bc, const double* post, double* pre) {
  Grid G{{nx, ny, nz}, {bc[0], bc[1], bc[2], bc[3], bc[4], bc[5]}};
  if (!grid_ok(G)) return -1;
  const long N = G.cells();
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        for (int q = 0; q < 19; ++q) pre[q * N + G.idx(x, y, z)] = pull_one(G, post, x, y, z, q);
  return 0;
}

// Macroscopic fields of the stored state, eq. (10): rho = sum f, rho u = sum c f (no force
// correction). rho, u nullable. sums (nullable) = (sum rho, sum rho ux, sum rho uy, sum rho uz),
// accumulated in the shifted variables: sum rho = N + sum g.
int orc_moments(int nx, int ny, int nz, const double* g, double* rho, double* u, double* sums) {
  const long N = (long)nx * ny * nz;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (long c = 0; c < N; ++c) {
    double drho = 0.0, m[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < 19; ++q) {
      drho += g[q * N + c];
      for (int a = 0; a < 3; ++a) m[a] += C[q][a] * g[q * N + c];
    }
    if (rho) rho[c] = 1.0 + drho;
    if (u)
      for (int a = 0; a < 3; ++a) u[a * N + c] = m[a] / (1.0 + drho);
    s[0] += drho;
    for (int a = 0; a < 3; ++a) s[a + 1] += m[a];
  }
  if (sums) {
    sums[0] = (double)N + s[0];
    for (int a = 0; a < 3; ++a) sums[a + 1] = s[a + 1];
  }
  return 0;
}

// Curl field of U (3 x N) with the wall ghosts of velocity_at.
int orc_curl(int nx, int ny, int nz, const int32_t* bc, const double* U, double* curl) {
  Grid G{{nx, ny, nz}, {bc[0], bc[1], bc[2], bc[3], bc[4], bc[5]}};
  if (!grid_ok(G)) return -1;
  const long N = G.cells();
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        double w[3];
        curl_at(G, U, x, y, z, w);
        for (int a = 0; a < 3; ++a) curl[a * N + G.idx(x, y, z)] = w[a];
      }
  return 0;
}

// Drag coefficient and lift coefficient of Table 1, with Re from eq. (3) read as
// Re = rho_l |u_r| d / mu_l and Eo as (rho_l - rho_b) g d^2 / sigma.
// Returns C_D * |u_r| (finite at u_r = 0) in *cdu and C_L in *cl.
void orc_closures(const orc_bubble_params* P, double nu, double d, double ur_mag, double* cdu,
                  double* cl, double* re_out) {
  const double Re = ur_mag * d / nu;
  const double Eo = (P->rho_l - P->rho_b) * P->g * d * d / P->sigma;
  // C_D = max[min{24/Re (1 + k Re^0.687), 48/Re}, 8/3 Eo/(Eo+4)], multiplied through by |u_r|
  // so that the 1/Re singularity cancels: 24/Re |u_r| = 24 nu / d.
  const double visc = std::min(24.0 * nu / d * (1.0 + P->cd_k * std::pow(Re, 0.687)), 48.0 * nu / d);
  const double shape = 8.0 / 3.0 * Eo / (Eo + 4.0) * ur_mag;
  *cdu = std::max(visc, shape);
  // Lift: Tomiyama-type three-branch coefficient.
  const double E = 1.0 / (1.0 + 0.163 * std::pow(Eo, 0.757));
  const double Eod = Eo / std::pow(E, 2.0 / 3.0);
  const double f = 0.00105 * Eod * Eod * Eod - 0.0159 * Eod * Eod - 0.0204 * Eod + P->lift_f0;
  double c;
  if (Eod < 4.0)
    c = std::min(0.288 * std::tanh(0.121 * Re), f);
  else if (Eod <= 10.0)
    c = f;
  else
    c = -0.29;
  *cl = c;
  if (re_out) *re_out = Re;
}

// Drag + lift on a bubble of diameter d moving at ub in liquid of velocity ul, vorticity wl.
void orc_drag_lift(const orc_bubble_params* P, double nu, double d, const double* ub,
                   const double* ul, const double* wl, double* FD, double* FL) {
  const double ur[3] = {ub[0] - ul[0], ub[1] - ul[1], ub[2] - ul[2]};
  const double mag = std::sqrt(ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2]);
  double cdu, cl;
  orc_closures(P, nu, d, mag, &cdu, &cl, nullptr);
  const double pi = 3.14159265358979323846;
  const double V = pi * d * d * d / 6.0;
  const double r = 0.5 * d;
  // F_D = -1/2 C_D rho_l pi r^2 |u_r| u_r
  for (int a = 0; a < 3; ++a) FD[a] = -0.5 * P->drag_scale * cdu * P->rho_l * pi * r * r * ur[a];
  // F_L = -C_L rho_l V u_r x (curl u_l)
  const double cr[3] = {ur[1] * wl[2] - ur[2] * wl[1], ur[2] * wl[0] - ur[0] * wl[2],
                        ur[0] * wl[1] - ur[1] * wl[0]};
  for (int a = 0; a < 3; ++a) FL[a] = -P->lift_scale * cl * P->rho_l * V * cr[a];
}

// Bubble ODE over one liquid step: n_sub explicit Euler sub-steps of eq. (4) with dt_b, the
// fluid quantities ul, wl and the fluid acceleration dul (= D_t u_l) frozen over the step.
// Newton's law eq. (1) with the forces of eq. (2) / Table 1; the virtual-mass term contains the
// bubble acceleration itself, so it is moved to the left-hand side (effective mass
// m_b + C_A rho_l V). Stress-gradient and the fluid part of virtual mass combine to
// (1 + C_A) rho_l V D_t u_l. Position S = dt_b * (new velocity).
// lo/hi (nullable): per axis position bounds [lo, hi] with clamp flags clamp_lo/hi[a] != 0 which
// clamp the position and zero that velocity component; periodic axes pass len[a] > 0 to wrap.
// psi (nullable): the reaction spread into the liquid: by default -(F_D + F_L) at the final
// velocity (Algorithm 1); the reaction bits of P->coupling select the sub-step mean of
// -(F_D + F_L) or minus the mean net force m_b du_b/dt.
void orc_bubble_ode(const orc_bubble_params* P, double nu, double dt_b, int n_sub, double d,
                    const double* ul, const double* wl, const double* dul, double* ub, double* xb,
                    const double* lo, const double* hi, const int32_t* clamp_lo,
                    const int32_t* clamp_hi, const double* len, double* psi) {
  const double pi = 3.14159265358979323846;
  const double V = pi * d * d * d / 6.0;
  const double m_b = P->rho_b * V;
  const double m_eff = m_b + P->c_a * P->rho_l * V;
  const double FB = (P->rho_l - P->rho_b) * V * P->g;  // buoyancy, +z
  const int reaction = P->coupling & ORC_REACTION_MASK;
  double sum_dl[3] = {0.0, 0.0, 0.0}, sum_net[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < n_sub; ++k) {
    double FD[3], FL[3];
    orc_drag_lift(P, nu, d, ub, ul, wl, FD, FL);
    for (int a = 0; a < 3; ++a) {
      double f = FD[a] + FL[a] + (1.0 + P->c_a) * P->rho_l * V * dul[a];
      if (a == 2) f += FB;
      sum_dl[a] += FD[a] + FL[a];
      sum_net[a] += m_b * (f / m_eff);  // eq. (1): the net force is m_b times the acceleration
      ub[a] += dt_b * f / m_eff;
    }
    for (int a = 0; a < 3; ++a) {
      xb[a] += dt_b * ub[a];
      if (len && len[a] > 0.0) {
        xb[a] = std::fmod(xb[a], len[a]);
        if (xb[a] < 0.0) xb[a] += len[a];
      } else if (lo && hi) {
        if (clamp_lo && clamp_lo[a] && xb[a] < lo[a]) { xb[a] = lo[a]; ub[a] = 0.0; }
        if (clamp_hi && clamp_hi[a] && xb[a] > hi[a]) { xb[a] = hi[a]; ub[a] = 0.0; }
      }
    }
  }
  if (psi) {
    if (reaction == ORC_REACTION_SUBSTEP_MEAN) {
      for (int a = 0; a < 3; ++a) psi[a] = -sum_dl[a] / n_sub;
    } else if (reaction == ORC_REACTION_NET_FORCE) {
      for (int a = 0; a < 3; ++a) psi[a] = -sum_net[a] / n_sub;
    } else {
      double FD[3], FL[3];
      orc_drag_lift(P, nu, d, ub, ul, wl, FD, FL);
      for (int a = 0; a < 3; ++a) psi[a] = -(FD[a] + FL[a]);
    }
  }
}

// Forward coupling, eq. (20): u_l = sum_j U(j) W_j and w_l = sum_j curl U(j) W_j over the
// separable cell weights of eq. (19) around position xb with half-width n.
int orc_interpolate(int nx, int ny, int nz, const int32_t* bc, const double* U, const double* xb,
                    double n, double* ul, double* wl, int point) {
  Grid G{{nx, ny, nz}, {bc[0], bc[1], bc[2], bc[3], bc[4], bc[5]}};
  if (!grid_ok(G)) return -1;
  const long N = G.cells();
  const int cap = 4 * (int)std::ceil(n) + 8;
  std::vector<int> ix(cap), iy(cap), iz(cap);
  std::vector<double> wx(cap), wy(cap), wz(cap);
  const int kx = axis_weights(xb[0], n, nx, G.periodic(0), ix.data(), wx.data(), cap, point != 0);
  const int ky = axis_weights(xb[1], n, ny, G.periodic(1), iy.data(), wy.data(), cap, point != 0);
  const int kz = axis_weights(xb[2], n, nz, G.periodic(2), iz.data(), wz.data(), cap, point != 0);
  if (kx < 0 || ky < 0 || kz < 0) return -2;
  for (int a = 0; a < 3; ++a) ul[a] = wl[a] = 0.0;
  for (int c = 0; c < kz; ++c)
    for (int b = 0; b < ky; ++b)
      for (int a = 0; a < kx; ++a) {
        const double Wj = wx[a] * wy[b] * wz[c];
        const long j = G.idx(ix[a], iy[b], iz[c]);
        double w[3];
        curl_at(G, U, ix[a], iy[b], iz[c], w);
        for (int m = 0; m < 3; ++m) {
          ul[m] += Wj * U[m * N + j];
          wl[m] += Wj * w[m];
        }
      }
  return 0;
}

// Backward coupling, eq. (21): F(j) += psi W_j with the same weights (added in place).
int orc_spread(int nx, int ny, int nz, const int32_t* bc, const double* xb, double n,
               const double* psi, double* F, int point) {
  Grid G{{nx, ny, nz}, {bc[0], bc[1], bc[2], bc[3], bc[4], bc[5]}};
  if (!grid_ok(G)) return -1;
  const long N = G.cells();
  const int cap = 4 * (int)std::ceil(n) + 8;
  std::vector<int> ix(cap), iy(cap), iz(cap);
  std::vector<double> wx(cap), wy(cap), wz(cap);
  const int kx = axis_weights(xb[0], n, nx, G.periodic(0), ix.data(), wx.data(), cap, point != 0);
  const int ky = axis_weights(xb[1], n, ny, G.periodic(1), iy.data(), wy.data(), cap, point != 0);
  const int kz = axis_weights(xb[2], n, nz, G.periodic(2), iz.data(), wz.data(), cap, point != 0);
  if (kx < 0 || ky < 0 || kz < 0) return -2;
  for (int c = 0; c < kz; ++c)
    for (int b = 0; b < ky; ++b)
      for (int a = 0; a < kx; ++a) {
        const double Wj = wx[a] * wy[b] * wz[c];
        const long j = G.idx(ix[a], iy[b], iz[c]);
        for (int m = 0; m < 3; ++m) F[m * N + j] += psi[m] * Wj;
      }
  return 0;
}

// One step of Algorithm 1 for nb bubbles (structure of arrays, doubles):
//   pos (3 x nb), vel (3 x nb), d (nb), ulp (3 x nb, previous interpolated liquid velocity),
//   state (nb): 0 inactive, 1 active without a previous liquid velocity, 2 active with one.
// g: liquid state f^n - w (in/out), U: velocity of the previous collision (in) and of this
// collision (out), F: force field work array (zeroed and rebuilt here), tmp: 19 x N scratch.
// psi_out (3 x nb, nullable) receives the reactions spread in this step.
int orc_method_step(int nx, int ny, int nz, const int32_t* bc, double omega,
                    const orc_bubble_params* P, int nb, double* pos, double* vel, const double* d,
                    double* ulp, int32_t* state, double* g, double* tmp, double* F, double* U,
                    double* psi_out, int nthreads) {
  Grid G{{nx, ny, nz}, {bc[0], bc[1], bc[2], bc[3], bc[4], bc[5]}};
  if (!grid_ok(G) || P->n_sub < 1) return -1;
  if ((P->coupling & ~(ORC_REACTION_MASK | ORC_POINT_KERNEL | ORC_EXACT_TIME)) ||
      (P->coupling & ORC_REACTION_MASK) > ORC_REACTION_NET_FORCE)
    return -1;
  const long N = G.cells();
  std::fill(F, F + 3 * N, 0.0);
  const double nu = (1.0 / omega - 0.5) / 3.0;  // eq. (9), dx = dt = 1
  const double dt_b = 1.0 / P->n_sub;
  double lo[3], hi[3], len[3];
  int32_t clo[3], chi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = 0.0;
    hi[a] = G.n[a] - 1.0;
    len[a] = G.periodic(a) ? (double)G.n[a] : 0.0;
    clo[a] = !G.periodic(a);
    chi[a] = !G.periodic(a) && a != 2;  // the top ends the bubble's life instead
  }
  // the velocity the forward coupling reads: that of the previous collision, or (exact time) that
  // of the current state f^n
  const double* Ui = U;
  std::vector<double> Un;
  if (P->coupling & ORC_EXACT_TIME) {
    Un.resize(3 * N);
    orc_moments(nx, ny, nz, g, nullptr, Un.data(), nullptr);
    Ui = Un.data();
  }
  const int point = (P->coupling & ORC_POINT_KERNEL) ? 1 : 0;
  // Forward coupling and ODE of every bubble: each reads only the velocity field Ui and its own
  // state, so the bubbles are independent here (threads over bubbles).
  std::vector<double> x0s(3 * (size_t)nb), xns(3 * (size_t)nb), ubs(3 * (size_t)nb),
      uls(3 * (size_t)nb), psis(3 * (size_t)nb);
  std::vector<int> rcs(nb, 0);
#pragma omp parallel for schedule(dynamic, 16)
  for (int b = 0; b < nb; ++b) {
    if (state[b] == 0) continue;
    double* x0 = &x0s[3 * (size_t)b];
    double* ub = &ubs[3 * (size_t)b];
    double* ul = &uls[3 * (size_t)b];
    double* xn = &xns[3 * (size_t)b];
    double* psi = &psis[3 * (size_t)b];
    for (int a = 0; a < 3; ++a) {
      x0[a] = pos[a * nb + b];
      ub[a] = vel[a * nb + b];
    }
    const double n = P->kernel_factor * d[b];
    double wl[3], dul[3] = {0.0, 0.0, 0.0};
    rcs[b] = orc_interpolate(nx, ny, nz, bc, Ui, x0, n, ul, wl, point);
    if (rcs[b]) continue;
    if (state[b] == 2)
      for (int a = 0; a < 3; ++a) dul[a] = ul[a] - ulp[a * nb + b];  // / dt_l, dt_l = 1
    for (int a = 0; a < 3; ++a) xn[a] = x0[a];
    orc_bubble_ode(P, nu, dt_b, P->n_sub, d[b], ul, wl, dul, ub, xn, lo, hi, clo, chi, len, psi);
  }
  for (int b = 0; b < nb; ++b)
    if (state[b] != 0 && rcs[b]) return rcs[b];
  // Backward coupling in bubble order (each cell sums its bubbles' forces in that order), then
  // the new bubble state.
  for (int b = 0; b < nb; ++b) {
    if (state[b] == 0) continue;
    const double* x0 = &x0s[3 * (size_t)b];
    const double* xn = &xns[3 * (size_t)b];
    const double* psi = &psis[3 * (size_t)b];
    const int rc = orc_spread(nx, ny, nz, bc, x0, P->kernel_factor * d[b], psi, F, point);
    if (rc) return rc;
    for (int a = 0; a < 3; ++a) {
      pos[a * nb + b] = xn[a];
      vel[a * nb + b] = ubs[3 * (size_t)b + a];
      ulp[a * nb + b] = uls[3 * (size_t)b + a];
      if (psi_out) psi_out[a * nb + b] = psi[a];
    }
    state[b] = 2;
    if (!G.periodic(2) && xn[2] >= G.n[2] - 1.0) state[b] = 0;  // reached the top layer
  }
  return orc_lbm_step(nx, ny, nz, bc, omega, g, tmp, F, U, nthreads);
}

}  // extern "C"
