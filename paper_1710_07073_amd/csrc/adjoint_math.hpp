// Host/device arithmetic of the method's adjoint: the transposed Jacobian of one cell's collision
// (BGK with Guo forcing, Sec. 2.2 eq. (6), (12)-(15)), the kernel weights with their derivative in
// the bubble position (eq. (18)-(19)), and the bubble ODE (eq. (1)-(4), Table 1) forward with
// recorded sub-steps and its reverse sweep. The kernels of adjoint.hip call these; the library
// also exports host wrappers so the same code can be checked against finite differences on a CPU.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "../../include/lbm.h"
#include "lattice.hpp"

namespace lbm {

#define LBM_HD __host__ __device__ inline

// ---------------------------------------------------------------------------------------------
// Collision of one cell, forward (generic arithmetic, any precision) and transposed Jacobian.
// p: pre-collision shifted populations, F: force density, out: post-collision populations,
// u: velocity of eq. (13).
// ---------------------------------------------------------------------------------------------
template <typename T>
LBM_HD void collide_cell(const T* p, const T* F, T omega, T* out, T* u) {
  T drho = 0, j[3] = {0, 0, 0};
  for (int q = 0; q < 19; ++q) {
    drho += p[q];
    j[0] += T(CX[q]) * p[q];
    j[1] += T(CY[q]) * p[q];
    j[2] += T(CZ[q]) * p[q];
  }
  const T rho = T(1) + drho;
  for (int a = 0; a < 3; ++a) u[a] = (j[a] + T(0.5) * F[a]) / rho;
  const T usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const T pre = T(1) - T(0.5) * omega;
  const T uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
  for (int q = 0; q < 19; ++q) {
    const T w = weight<T>(q);
    const T cu = T(CX[q]) * u[0] + T(CY[q]) * u[1] + T(CZ[q]) * u[2];
    const T cF = T(CX[q]) * F[0] + T(CY[q]) * F[1] + T(CZ[q]) * F[2];
    const T geq = w * (drho + rho * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq));
    const T X = T(3) * (cF - uF) + T(9) * cu * cF;
    out[q] = (T(1) - omega) * p[q] + omega * geq + pre * w * X;
  }
}

// c * v for a lattice weight c given in double. In FP32, c is carried as hi + lo floats: a single
// rounded weight is off by up to 3e-8 relative in one direction, and the transposed collision
// would multiply the adjoint's density and momentum modes by that factor on every step (as the
// forward collision does with its equilibrium, collide.hpp). FP64 keeps the plain product.
template <typename T>
LBM_HD T mul_weight_hd(double c, T v) {
  if constexpr (sizeof(T) == 4) {
    const float hi = (float)c, lo = (float)(c - (double)hi);
    return fmaf(hi, v, lo * v);
  } else {
    return T(c) * v;
  }
}

// s += c v for a lattice component c in {-1, 0, 1} (no arithmetic when c = 0).
template <typename T>
LBM_HD void add_c(T& s, int c, T v) {
  if (c > 0) s += v;
  else if (c < 0) s -= v;
}

// sum_a c_a v_a for a lattice velocity c.
template <typename T>
LBM_HD T dot_c(int cx, int cy, int cz, const T* v) {
  T s = T(0);
  bool first = true;
  const int c[3] = {cx, cy, cz};
  for (int a = 0; a < 3; ++a) {
    if (c[a] == 0) continue;
    s = first ? (c[a] > 0 ? v[a] : -v[a]) : (c[a] > 0 ? s + v[a] : s - v[a]);
    first = false;
  }
  return s;
}

// Given lam = dL/d(out) and lamU = dL/du of one cell, returns mu = dL/dp, lamF = dL/dF and the
// cell's share of dL/domega. With rho = 1 + sum p and u = (sum c p + F/2)/rho:
//   mu_k = (1 - omega) lam_k + A + sum_a B_a (c_ka - u_a) / rho,
//   A    = omega sum_q lam_q dgeq_q/drho,
//   B_a  = sum_q lam_q (omega dgeq_q/du_a + dS_q/du_a) + lamU_a,
//   lamF_a = sum_q lam_q dS_q/dF_a + B_a / (2 rho),
//   dL/domega = sum_q lam_q (geq_q - p_q - X_q w_q / 2), S_q = (1 - omega/2) w_q X_q.
// The sums over q are polynomials of degree at most two in c_q, so they reduce to the moments of
// m_q = w_q lam_q: M0 = sum m, M1_a = sum m c_a, M2_ab = sum m c_a c_b. With V = M2 u, G = M2 F:
//   A   = omega (M0 + 3 u.M1 + 4.5 u.V - 1.5 |u|^2 M0),
//   B_a = lamU_a + omega rho (3 M1_a + 9 V_a - 3 u_a M0) + (1 - omega/2)(9 G_a - 3 F_a M0),
//   sum_q lam_q dS_q/dF_a = (1 - omega/2)(3 M1_a - 3 u_a M0 + 9 V_a),
//   sum_q m_q X_q = 3 (F.M1 - (u.F) M0) + 9 u.G.
// The moments are summed per weight class (lam summed over the faces and over the edges, then
// multiplied by the class weight, as hi + lo in FP32). Only dL/domega keeps a term per direction:
// geq_q - p_q is the small non-equilibrium part, taken per direction before the sum.
template <typename T>
LBM_HD void collide_cell_adjoint(const T* p, const T* F, T omega, const T* lam, const T* lamU, T* mu,
                                 T* lamF, double* domega) {
  T drho = 0, j[3] = {0, 0, 0};
  for (int q = 0; q < 19; ++q) {
    drho += p[q];
    j[0] += T(CX[q]) * p[q];
    j[1] += T(CY[q]) * p[q];
    j[2] += T(CZ[q]) * p[q];
  }
  const T rho = T(1) + drho;
  const T inv = T(1) / rho;
  T u[3];
  for (int a = 0; a < 3; ++a) u[a] = (j[a] + T(0.5) * F[a]) * inv;
  const T usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const T pre = T(1) - T(0.5) * omega;
  const T uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
  // lam summed per class (0: faces, 1: edges): s0 = sum lam, s1_a = sum lam c_a, s2_a = sum lam
  // c_a^2, sx = sum lam c_a c_b over the edges (xy, xz, yz); dsum = sum lam (geq - p)
  T s0[2] = {0, 0}, s1[2][3] = {{0, 0, 0}, {0, 0, 0}}, s2[2][3] = {{0, 0, 0}, {0, 0, 0}};
  T sx[3] = {0, 0, 0}, dsum = 0;
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const int cx = CX[q], cy = CY[q], cz = CZ[q];
    const T l = lam[q];
    const T cu = dot_c<T>(cx, cy, cz, u);
    const T geq = weight<T>(q) * (drho + rho * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq));
    dsum += l * (geq - p[q]);
    if (q == 18) continue;
    const int k = q < 6 ? 0 : 1;
    s0[k] += l;
    add_c(s1[k][0], cx, l);
    add_c(s1[k][1], cy, l);
    add_c(s1[k][2], cz, l);
    if (cx) s2[k][0] += l;
    if (cy) s2[k][1] += l;
    if (cz) s2[k][2] += l;
    add_c(sx[0], cx * cy, l);
    add_c(sx[1], cx * cz, l);
    add_c(sx[2], cy * cz, l);
  }
  constexpr double wf = 1.0 / 18.0, we = 1.0 / 36.0;
  const T M0 = mul_weight_hd<T>(1.0 / 3.0, lam[18]) + mul_weight_hd<T>(wf, s0[0]) +
               mul_weight_hd<T>(we, s0[1]);
  T M1[3], M2[3][3];
  for (int a = 0; a < 3; ++a) {
    M1[a] = mul_weight_hd<T>(wf, s1[0][a]) + mul_weight_hd<T>(we, s1[1][a]);
    M2[a][a] = mul_weight_hd<T>(wf, s2[0][a]) + mul_weight_hd<T>(we, s2[1][a]);
  }
  M2[0][1] = M2[1][0] = mul_weight_hd<T>(we, sx[0]);
  M2[0][2] = M2[2][0] = mul_weight_hd<T>(we, sx[1]);
  M2[1][2] = M2[2][1] = mul_weight_hd<T>(we, sx[2]);
  T V[3], G[3];
  for (int a = 0; a < 3; ++a) {
    V[a] = M2[a][0] * u[0] + M2[a][1] * u[1] + M2[a][2] * u[2];
    G[a] = M2[a][0] * F[0] + M2[a][1] * F[1] + M2[a][2] * F[2];
  }
  const T uM1 = u[0] * M1[0] + u[1] * M1[1] + u[2] * M1[2];
  const T uV = u[0] * V[0] + u[1] * V[1] + u[2] * V[2];
  const T FM1 = F[0] * M1[0] + F[1] * M1[1] + F[2] * M1[2];
  const T uG = u[0] * G[0] + u[1] * G[1] + u[2] * G[2];
  const T A = omega * (M0 + T(3) * uM1 + T(4.5) * uV - T(1.5) * usq * M0);
  T b[3];
  for (int a = 0; a < 3; ++a) {
    const T B = lamU[a] + omega * rho * (T(3) * M1[a] + T(9) * V[a] - T(3) * u[a] * M0) +
                pre * (T(9) * G[a] - T(3) * F[a] * M0);
    lamF[a] = pre * (T(3) * M1[a] - T(3) * u[a] * M0 + T(9) * V[a]) + B * T(0.5) * inv;
    b[a] = B * inv;
  }
  const T K0 = A - (b[0] * u[0] + b[1] * u[1] + b[2] * u[2]);
  const T decay = T(1) - omega;
#pragma unroll
  for (int k = 0; k < 19; ++k) mu[k] = decay * lam[k] + (K0 + dot_c<T>(CX[k], CY[k], CZ[k], b));
  *domega = (double)dsum - 0.5 * (double)(T(3) * (FM1 - uF * M0) + T(9) * uG);
}

// ---------------------------------------------------------------------------------------------
// Kernel weights along one axis with their derivative in the bubble coordinate.
// ---------------------------------------------------------------------------------------------
constexpr int kAdjSpan = LBM_MAX_STENCIL + 2;

LBM_HD double kernel_P(double s) {
  if (s <= -1.0) return 0.0;
  if (s >= 1.0) return 1.0;
  const double s2 = s * s;
  return 0.5 + 15.0 / 16.0 * (s - 2.0 / 3.0 * s2 * s + 0.2 * s2 * s2 * s);
}
// dP/ds = Z in units of the half-width: 15/16 (1 - s^2)^2 inside the support
LBM_HD double kernel_dP(double s) {
  if (s <= -1.0 || s >= 1.0) return 0.0;
  const double t = 1.0 - s * s;
  return 15.0 / 16.0 * t * t;
}

struct AxisW {
  int lo, hi, clo, chi, dlo, dhi;
};

LBM_HD bool axis_window_hd(double x, double n, int ext, bool per, AxisW& w) {
  const double lo = floor(x - n - 0.5) + 1.0;
  const double hi = ceil(x + n + 0.5) - 1.0;
  if (!(hi - lo + 1.0 <= (double)LBM_MAX_STENCIL) || !(lo > -1e9) || !(hi < 1e9)) return false;
  w.lo = (int)lo;
  w.hi = (int)hi;
  w.clo = per ? w.lo : (w.lo > 0 ? w.lo : 0);
  w.chi = per ? w.hi : (w.hi < ext - 1 ? w.hi : ext - 1);
  if (w.clo > w.chi) return false;
  w.dlo = per ? w.clo - 1 : (w.clo - 1 > 0 ? w.clo - 1 : 0);
  w.dhi = per ? w.chi + 1 : (w.chi + 1 < ext - 1 ? w.chi + 1 : ext - 1);
  return true;
}

// Sequential evaluation of one axis: w, dw (curl weights with wall ghosts folded in) and their
// derivatives wx = dw/dx_b, dwx = d(dw)/dx_b, indexed by cell - lo + 1. s_lo, s_hi: ghost signs of
// the two faces (-1 bounce-back, +1 free slip); per: periodic axis.
LBM_HD bool axis_weights_dx(double x, double n, int ext, bool per, double s_lo, double s_hi,
                            AxisW& A, double* w, double* dw, double* wx, double* dwx) {
  if (!axis_window_hd(x, n, ext, per, A)) return false;
  double sum = 0.0, dsum = 0.0;
  for (int i = 0; i < kAdjSpan; ++i) {
    const int v = A.lo - 1 + i;
    double wi = 0.0, di = 0.0;
    if (v >= A.clo && v <= A.chi) {
      const double sp = (v + 0.5 - x) / n, sm = (v - 0.5 - x) / n;
      wi = kernel_P(sp) - kernel_P(sm);
      di = -(kernel_dP(sp) - kernel_dP(sm)) / n;
    }
    w[i] = wi;
    wx[i] = di;
    sum += wi;
    dsum += di;
  }
  if (!per && sum > 0.0) {  // clipped at a wall: renormalise, d(w/S) = (dw - (w/S) dS) / S
    for (int i = 0; i < kAdjSpan; ++i) {
      const double wn = w[i] / sum;
      wx[i] = (wx[i] - wn * dsum) / sum;
      w[i] = wn;
    }
  }
  for (int i = 0; i < kAdjSpan; ++i) {
    const int v = A.lo - 1 + i;
    const double wm = i > 0 ? w[i - 1] : 0.0, wp = i + 1 < kAdjSpan ? w[i + 1] : 0.0;
    const double xm = i > 0 ? wx[i - 1] : 0.0, xp = i + 1 < kAdjSpan ? wx[i + 1] : 0.0;
    double d = 0.5 * (wm - wp), dx = 0.5 * (xm - xp);
    if (!per) {
      if (v == 0) {
        d -= 0.5 * s_lo * w[i];
        dx -= 0.5 * s_lo * wx[i];
      }
      if (v == ext - 1) {
        d += 0.5 * s_hi * w[i];
        dx += 0.5 * s_hi * wx[i];
      }
    }
    dw[i] = d;
    dwx[i] = dx;
  }
  return true;
}

// ---------------------------------------------------------------------------------------------
// Bubble ODE with recorded sub-steps, and its reverse sweep.
// ---------------------------------------------------------------------------------------------
constexpr int kMaxSub = 32;

struct OdeBounds {
  double hi[3];   // upper bound of the clamp on the lateral axes (ext - 1)
  double len[3];  // period of a periodic axis, 0 otherwise
  int top;        // z has a top (non-periodic): no clamp there, the bubble stops instead
};

struct ForceJac {
  double F[3];      // F_D + F_L
  double FD1[3];    // F_D / drag_scale
  double FL1[3];    // F_L / lift_scale
  double J[3][3];   // d(F_D + F_L)/du_r
  double Jw[3][3];  // dF_L/d(curl u_l)
  double dnu[3];    // d(F_D + F_L)/dnu
};

// Per-bubble constants of the Table 1 closures (they depend on the diameter and nu only).
struct ForceConst {
  double KD, KL;     // 1/2 rho_l pi r^2 and rho_l V
  double shape;      // 8/3 Eo / (Eo + 4)
  double v24, v48;   // 24 nu / d and 48 nu / d
  double Eod, fl;    // modified Eotvos number and f(Eo_d) of the lift coefficient
};

LBM_HD ForceConst force_const(const bubble_params& P, double nu, double d) {
  const double pi = 3.14159265358979323846;
  const double V = pi * d * d * d / 6.0;
  const double r = 0.5 * d;
  ForceConst c;
  c.KD = 0.5 * P.rho_l * pi * r * r;
  c.KL = P.rho_l * V;
  const double Eo = (P.rho_l - P.rho_b) * P.g * d * d / P.sigma;
  c.shape = 8.0 / 3.0 * Eo / (Eo + 4.0);
  c.v24 = 24.0 * nu / d;
  c.v48 = 48.0 * nu / d;
  const double E = 1.0 / (1.0 + 0.163 * exp(0.757 * log(Eo)));
  c.Eod = Eo / exp(2.0 / 3.0 * log(E));
  c.fl = 0.00105 * c.Eod * c.Eod * c.Eod - 0.0159 * c.Eod * c.Eod - 0.0204 * c.Eod + P.lift_f0;
  return c;
}

// Drag and lift of Table 1 at relative velocity u_r = ub - ul; with J (nullable output f.J etc.)
// their derivatives. F alone (deriv false) takes the same operations as with the derivatives.
template <bool DERIV>
LBM_HD void force_eval(const bubble_params& P, const ForceConst& c, double nu, double d,
                       const double* ub, const double* ul, const double* wl, ForceJac& f) {
  const double ur[3] = {ub[0] - ul[0], ub[1] - ul[1], ub[2] - ul[2]};
  const double m = sqrt(ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2]);
  const double Re = m * d / nu;
  // viscous branch min{24/Re (1 + k Re^0.687), 48/Re} |u_r|, its m d/dm and d/dnu
  double visc = c.v48, visc_m = 0.0, visc_nu = 48.0 / d;
  if (Re > 0.0) {
    const double t = P.cd_k * exp(0.687 * log(Re));
    const double a = c.v24 * (1.0 + t);
    if (a < c.v48) {
      visc = a;
      visc_m = c.v24 * 0.687 * t;
      visc_nu = 24.0 / d * (1.0 + 0.313 * t);
    }
  } else if (c.v24 < c.v48) {
    visc = c.v24;
    visc_nu = 24.0 / d;
  }
  double cdu, cdu_m, cdu_nu;
  if (c.shape * m > visc) {
    cdu = c.shape * m;
    cdu_m = c.shape * m;
    cdu_nu = 0.0;
  } else {
    cdu = visc;
    cdu_m = visc_m;
    cdu_nu = visc_nu;
  }
  // lift coefficient and dC_L/dRe
  double cl, cl_re = 0.0;
  if (c.Eod < 4.0) {
    const double th = tanh(0.121 * Re);
    if (0.288 * th < c.fl) {
      cl = 0.288 * th;
      cl_re = 0.288 * 0.121 * (1.0 - th * th);
    } else {
      cl = c.fl;
    }
  } else if (c.Eod <= 10.0) {
    cl = c.fl;
  } else {
    cl = -0.29;
  }
  const double cr[3] = {ur[1] * wl[2] - ur[2] * wl[1], ur[2] * wl[0] - ur[0] * wl[2],
                        ur[0] * wl[1] - ur[1] * wl[0]};
  const double sD = P.drag_scale, sL = P.lift_scale;
  const double KD = c.KD, KL = c.KL;
  for (int a = 0; a < 3; ++a) {
    f.FD1[a] = -KD * cdu * ur[a];
    f.FL1[a] = -KL * cl * cr[a];
    f.F[a] = sD * f.FD1[a] + sL * f.FL1[a];
  }
  if constexpr (DERIV) {
    const double uh[3] = {m > 0.0 ? ur[0] / m : 0.0, m > 0.0 ? ur[1] / m : 0.0,
                          m > 0.0 ? ur[2] / m : 0.0};
    // d(u_r x w)/du_r and d(u_r x w)/dw
    const double dcr_du[3][3] = {{0.0, wl[2], -wl[1]}, {-wl[2], 0.0, wl[0]}, {wl[1], -wl[0], 0.0}};
    const double dcr_dw[3][3] = {{0.0, -ur[2], ur[1]}, {ur[2], 0.0, -ur[0]}, {-ur[1], ur[0], 0.0}};
    const double dcl_dm = cl_re * d / nu;  // dC_L/d|u_r|
    for (int a = 0; a < 3; ++a) {
      for (int b = 0; b < 3; ++b) {
        const double dd = -sD * KD * ((a == b ? cdu : 0.0) + cdu_m * uh[a] * uh[b]);
        const double dl = -sL * KL * (cl * dcr_du[a][b] + cr[a] * dcl_dm * uh[b]);
        f.J[a][b] = dd + dl;
        f.Jw[a][b] = -sL * KL * cl * dcr_dw[a][b];
      }
      f.dnu[a] = -sD * KD * cdu_nu * ur[a] - sL * KL * cr[a] * cl_re * (-Re / nu);
    }
  } else {
    (void)cdu_m;
    (void)cdu_nu;
    (void)cl_re;
  }
}

// Drag and lift of Table 1 at relative velocity u_r = ub - ul, with their derivatives.
LBM_HD void force_jac(const bubble_params& P, const ForceConst& c, double nu, double d,
                      const double* ub, const double* ul, const double* wl, ForceJac& f) {
  force_eval<true>(P, c, nu, d, ub, ul, wl, f);
}

struct OdeOut {
  double x[3], ub[3], psi[3];
};

// The ODE of one liquid step (n_sub explicit sub-steps with the added mass on the left), as the
// forward kernel computes it; ubs/clamped record the sub-step velocities and clamp events.
LBM_HD void ode_forward(const bubble_params& P, double nu, double d, const double* x0,
                        const double* ub0, const double* ul, const double* wl, const double* dul,
                        const OdeBounds& Bd, OdeOut& o, double (*ubs)[3], unsigned char (*clamped)[3]) {
  const double pi = 3.14159265358979323846;
  const double V = pi * d * d * d / 6.0;
  const double inv_meff = 1.0 / (P.rho_b * V + P.c_a * P.rho_l * V);
  const double va = (1.0 + P.c_a) * P.rho_l * V;
  const double fb = (P.rho_l - P.rho_b) * V * P.g;
  const double dt = 1.0 / P.n_sub;
  const ForceConst fc = force_const(P, nu, d);
  double ub[3] = {ub0[0], ub0[1], ub0[2]}, x[3] = {x0[0], x0[1], x0[2]};
  for (int k = 0; k < P.n_sub; ++k) {
    if (ubs)
      for (int a = 0; a < 3; ++a) ubs[k][a] = ub[a];
    ForceJac f;
    force_eval<false>(P, fc, nu, d, ub, ul, wl, f);
    for (int a = 0; a < 3; ++a) {
      double fa = f.F[a] + va * dul[a];
      if (a == 2) fa += fb;
      ub[a] += dt * fa * inv_meff;
    }
    for (int a = 0; a < 3; ++a) {
      unsigned char c = 0;
      x[a] += dt * ub[a];
      if (Bd.len[a] > 0.0) {
        x[a] = fmod(x[a], Bd.len[a]);
        if (x[a] < 0.0) x[a] += Bd.len[a];
      } else {
        if (x[a] < 0.0) {
          x[a] = 0.0;
          ub[a] = 0.0;
          c = 1;
        }
        if (!(a == 2 && Bd.top) && x[a] > Bd.hi[a]) {
          x[a] = Bd.hi[a];
          ub[a] = 0.0;
          c = 1;
        }
      }
      if (clamped) clamped[k][a] = c;
    }
  }
  if (ubs)
    for (int a = 0; a < 3; ++a) ubs[P.n_sub][a] = ub[a];
  ForceJac f;
  force_eval<false>(P, fc, nu, d, ub, ul, wl, f);
  for (int a = 0; a < 3; ++a) {
    o.x[a] = x[a];
    o.ub[a] = ub[a];
    o.psi[a] = -f.F[a];
  }
}

struct OdeAdj {
  double x[3], ub[3], ul[3], wl[3], dul[3];
  double dsD, dsL, dnu;
};

// Reverse sweep of ode_forward from its record (clamp events) and the force Jacobians at the
// sub-step velocities, jac[k] = force_jac at ubs[k] for k = 0..n_sub (jac[n_sub]: the final
// velocity, where the reaction is taken): given dL/dx_new, dL/dub_new, dL/dpsi, returns the
// derivatives in the step's inputs and in drag_scale, lift_scale and nu. The Jacobians do not
// depend on the adjoint state, so a caller may evaluate them in parallel.
LBM_HD void ode_adjoint_sweep(const bubble_params& P, double d, const unsigned char (*clamped)[3],
                              const ForceJac* jac, const double* lx_new, const double* lub_new,
                              const double* lpsi, OdeAdj& g) {
  const double pi = 3.14159265358979323846;
  const double V = pi * d * d * d / 6.0;
  const double inv_meff = 1.0 / (P.rho_b * V + P.c_a * P.rho_l * V);
  const double va = (1.0 + P.c_a) * P.rho_l * V;
  const double s = inv_meff / P.n_sub;
  double lx[3], lub[3];
  for (int a = 0; a < 3; ++a) {
    lx[a] = lx_new[a];
    lub[a] = lub_new[a];
    g.ul[a] = g.wl[a] = g.dul[a] = 0.0;
  }
  g.dsD = g.dsL = g.dnu = 0.0;
  {  // psi = -(F_D + F_L)(ub_n)
    const ForceJac& f = jac[P.n_sub];
    for (int b = 0; b < 3; ++b) {
      double t = 0.0, tw = 0.0;
      for (int a = 0; a < 3; ++a) {
        t += f.J[a][b] * lpsi[a];
        tw += f.Jw[a][b] * lpsi[a];
      }
      lub[b] -= t;
      g.ul[b] += t;
      g.wl[b] -= tw;
    }
    for (int a = 0; a < 3; ++a) {
      g.dsD -= f.FD1[a] * lpsi[a];
      g.dsL -= f.FL1[a] * lpsi[a];
      g.dnu -= f.dnu[a] * lpsi[a];
    }
  }
  for (int k = P.n_sub - 1; k >= 0; --k) {
    // x_{k+1} = x_k + dt ub'_{k+1} (then clamped), ub_{k+1} = ub' with clamped components zeroed
    double lup[3];
    for (int a = 0; a < 3; ++a) {
      if (clamped[k][a]) {
        lup[a] = 0.0;
        lx[a] = 0.0;
      } else {
        lup[a] = lub[a] + lx[a] / P.n_sub;
      }
    }
    // ub' = ub_k + dt/m_eff (F(ub_k) + va dul + fb e_z)
    const ForceJac& f = jac[k];
    for (int b = 0; b < 3; ++b) {
      double t = 0.0, tw = 0.0;
      for (int a = 0; a < 3; ++a) {
        t += f.J[a][b] * lup[a];
        tw += f.Jw[a][b] * lup[a];
      }
      lub[b] = lup[b] + s * t;
      g.ul[b] -= s * t;
      g.wl[b] += s * tw;
      g.dul[b] += s * va * lup[b];
    }
    for (int a = 0; a < 3; ++a) {
      g.dsD += s * f.FD1[a] * lup[a];
      g.dsL += s * f.FL1[a] * lup[a];
      g.dnu += s * f.dnu[a] * lup[a];
    }
  }
  for (int a = 0; a < 3; ++a) {
    g.x[a] = lx[a];
    g.ub[a] = lub[a];
  }
}

// The whole reverse step in one thread: forward recompute, Jacobians, sweep (host checks).
LBM_HD void ode_adjoint(const bubble_params& P, double nu, double d, const double* x0,
                        const double* ub0, const double* ul, const double* wl, const double* dul,
                        const OdeBounds& Bd, const double* lx_new, const double* lub_new,
                        const double* lpsi, OdeAdj& g) {
  double ubs[kMaxSub + 1][3];
  unsigned char clamped[kMaxSub][3];
  OdeOut o;
  ode_forward(P, nu, d, x0, ub0, ul, wl, dul, Bd, o, ubs, clamped);
  const ForceConst c = force_const(P, nu, d);
  ForceJac jac[kMaxSub + 1];
  for (int k = 0; k <= P.n_sub; ++k) force_jac(P, c, nu, d, ubs[k], ul, wl, jac[k]);
  ode_adjoint_sweep(P, d, clamped, jac, lx_new, lub_new, lpsi, g);
}

}  // namespace lbm
