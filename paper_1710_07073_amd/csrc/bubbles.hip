// Bubble half of one step of Algorithm 1, fused into one kernel with one workgroup per bubble:
//   1. cell-integral weights of the clipped fourth-order polynomial kernel along each axis
//      (eq. (18)-(19)), clipped at walls and renormalised, wrapped on periodic axes;
//   2. forward coupling (eq. (20)): the liquid velocity of the previous collision and its curl
//      (central differences, wall ghosts) are staged chunk by chunk in LDS and summed with the
//      weights, wavefront reductions in double precision;
//   3. the bubble ODE (eq. (1)-(4), Table 1) on one lane: n_sub explicit sub-steps with the
//      added-mass term on the left-hand side, in double precision;
//   4. backward coupling (eq. (21)): the reaction -(F_D + F_L) at the updated velocity is spread
//      into the force field with the same weights (atomic adds), and the 8^3 tiles the liquid step
//      must force, or must write the velocity in for the next interpolation, are flagged.
#include <math.h>

#include "internal.hpp"

namespace lbm {
namespace {

constexpr int kThreads = 256;
constexpr int kMax = LBM_MAX_STENCIL;
constexpr int kLdsBytes = 48 * 1024;

struct BubbleArgs {
  Geom G;
  bubble_params P;
  bubble_soa S;
  int nb;
  double nu;
  int32_t* status;
};

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// antiderivative of the kernel in s = r / n, P(-1) = 0, P(1) = 1
__device__ __forceinline__ double kernel_P(double s) {
  if (s <= -1.0) return 0.0;
  if (s >= 1.0) return 1.0;
  return 0.5 + 15.0 / 16.0 * (s - 2.0 / 3.0 * s * s * s + 0.2 * pow(s, 5.0));
}

// Velocity at an integer position at most one cell outside the domain, with the wall ghosts:
// bounce-back negates the mirror cell's velocity, free slip negates its normal component.
template <typename T>
__device__ __forceinline__ void ghost_velocity(const T* __restrict__ U, const Geom& G, int x, int y,
                                               int z, double out[3]) {
  int p[3] = {x, y, z};
  const int ext[3] = {G.nx, G.ny, G.nz};
  double sign[3] = {1.0, 1.0, 1.0};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (G.bc[2 * a] == BC_PER) {
      p[a] = wrapi(p[a], ext[a]);
    } else if (p[a] < 0 || p[a] >= ext[a]) {
      const int side = p[a] < 0 ? 0 : 1;
      p[a] = side == 0 ? -1 - p[a] : 2 * ext[a] - 1 - p[a];
      if (G.bc[2 * a + side] == BC_FS) {
        sign[a] = -sign[a];
      } else {
        sign[0] = -sign[0];
        sign[1] = -sign[1];
        sign[2] = -sign[2];
      }
    }
  }
  const uint32_t c = ((uint32_t)p[2] * G.ny + p[1]) * G.nx + p[0];
  out[0] = sign[0] * (double)U[c];
  out[1] = sign[1] * (double)U[G.N + c];
  out[2] = sign[2] * (double)U[2 * (size_t)G.N + c];
}

struct Closure {
  double cdu, cl;
};

// Table 1 drag and lift coefficients with Re = |u_r| d / nu; C_D is returned multiplied by |u_r|.
__device__ __forceinline__ Closure closures(const bubble_params& P, double nu, double d,
                                            double urm, double Eo, double Eod) {
  const double Re = urm * d / nu;
  const double visc = fmin(24.0 * nu / d * (1.0 + P.cd_k * pow(Re, 0.687)), 48.0 * nu / d);
  const double shape = 8.0 / 3.0 * Eo / (Eo + 4.0) * urm;
  const double f = 0.00105 * Eod * Eod * Eod - 0.0159 * Eod * Eod - 0.0204 * Eod + P.lift_f0;
  double cl;
  if (Eod < 4.0)
    cl = fmin(0.288 * tanh(0.121 * Re), f);
  else if (Eod <= 10.0)
    cl = f;
  else
    cl = -0.29;
  return {fmax(visc, shape), cl};
}

__device__ __forceinline__ void drag_lift(const bubble_params& P, double nu, double d, double Eo,
                                          double Eod, const double ub[3], const double ul[3],
                                          const double wl[3], double FD[3], double FL[3]) {
  const double pi = 3.14159265358979323846;
  const double ur[3] = {ub[0] - ul[0], ub[1] - ul[1], ub[2] - ul[2]};
  const double mag = sqrt(ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2]);
  const Closure c = closures(P, nu, d, mag, Eo, Eod);
  const double V = pi * d * d * d / 6.0;
  const double r = 0.5 * d;
  for (int a = 0; a < 3; ++a) FD[a] = -0.5 * P.drag_scale * c.cdu * P.rho_l * pi * r * r * ur[a];
  const double cr[3] = {ur[1] * wl[2] - ur[2] * wl[1], ur[2] * wl[0] - ur[0] * wl[2],
                        ur[0] * wl[1] - ur[1] * wl[0]};
  for (int a = 0; a < 3; ++a) FL[a] = -P.lift_scale * c.cl * P.rho_l * V * cr[a];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Tile ranges touched along one axis by the cell range [vlo, vhi] (virtual, may wrap when
// periodic): up to two ranges of 8-cell tiles.
struct TileRanges {
  int n;
  int lo[2], hi[2];
};

__device__ TileRanges tile_ranges(int vlo, int vhi, int ext, bool periodic) {
  TileRanges t;
  if (!periodic) {
    vlo = vlo < 0 ? 0 : vlo;
    vhi = vhi > ext - 1 ? ext - 1 : vhi;
    t.n = vlo <= vhi ? 1 : 0;
    t.lo[0] = vlo / (int)kTile;
    t.hi[0] = vhi / (int)kTile;
    return t;
  }
  if (vhi - vlo + 1 >= ext) {
    t.n = 1;
    t.lo[0] = 0;
    t.hi[0] = (ext - 1) / (int)kTile;
    return t;
  }
  const int a = wrapi(vlo, ext), b = wrapi(vhi, ext);
  if (a <= b) {
    t.n = 1;
    t.lo[0] = a / (int)kTile;
    t.hi[0] = b / (int)kTile;
  } else {
    t.n = 2;
    t.lo[0] = a / (int)kTile;
    t.hi[0] = (ext - 1) / (int)kTile;
    t.lo[1] = 0;
    t.hi[1] = b / (int)kTile;
  }
  return t;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_bubbles(const T* __restrict__ U, T* __restrict__ F,
                                                      uint8_t* __restrict__ tiles, BubbleArgs A) {
  constexpr int CAP = kLdsBytes / (3 * (int)sizeof(T));
  __shared__ T s_u[3][CAP];
  __shared__ double s_w[3][kMax];
  __shared__ int s_i[3][kMax];  // wrapped cell index, -1 outside a wall
  __shared__ double s_red[6][kThreads / 64];
  __shared__ double s_psi[3];
  __shared__ int s_box[3][2];   // clipped window, virtual coordinates
  __shared__ int s_lo[3];       // unclipped window start
  __shared__ int s_next[3][2];  // window at the new position
  __shared__ int s_ok;

  const Geom& G = A.G;
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int ext[3] = {G.nx, G.ny, G.nz};
  if (A.S.state[b] == 0) {
    if (tid == 0 && A.S.psix) {
      A.S.psix[b] = 0.0;
      A.S.psiy[b] = 0.0;
      A.S.psiz[b] = 0.0;
    }
    return;
  }
  const double xb[3] = {A.S.x[b], A.S.y[b], A.S.z[b]};
  const double d = A.S.d[b];
  const double n = A.P.kernel_factor * d;

  if (tid == 0) {
    int ok = isfinite(xb[0]) && isfinite(xb[1]) && isfinite(xb[2]) && d > 0.0 && isfinite(n);
    for (int a = 0; a < 3 && ok; ++a) {
      const double lo = floor(xb[a] - n - 0.5) + 1.0;
      const double hi = ceil(xb[a] + n + 0.5) - 1.0;
      if (!(hi - lo + 1.0 <= (double)kMax) || lo < -1e9 || hi > 1e9) {
        ok = 0;
        break;
      }
      s_lo[a] = (int)lo;
      const bool per = G.bc[2 * a] == BC_PER;
      int clo = (int)lo, chi = (int)hi;
      if (!per) {
        clo = clo < 0 ? 0 : clo;
        chi = chi > ext[a] - 1 ? ext[a] - 1 : chi;
      }
      if (clo > chi) ok = 0;  // window entirely outside the domain
      s_box[a][0] = clo;
      s_box[a][1] = chi;
    }
    if (!ok) atomicOr(A.status, (int32_t)STATUS_STENCIL_TOO_LARGE);
    s_ok = ok;
  }
  __syncthreads();
  if (!s_ok) return;

  // 1. axis weights
  for (int k = tid; k < 3 * kMax; k += kThreads) {
    const int a = k / kMax, i = k % kMax;
    const int v = s_lo[a] + i;
    const bool per = G.bc[2 * a] == BC_PER;
    double w = kernel_P((v + 0.5 - xb[a]) / n) - kernel_P((v - 0.5 - xb[a]) / n);
    int idx = per ? wrapi(v, ext[a]) : v;
    if (!per && (v < 0 || v >= ext[a])) {
      idx = -1;
      w = 0.0;
    }
    s_w[a][i] = w;
    s_i[a][i] = idx;
  }
  __syncthreads();
  if (tid < 3) {
    const int a = tid;
    if (G.bc[2 * a] != BC_PER) {
      double sum = 0.0;
      for (int v = s_box[a][0]; v <= s_box[a][1]; ++v) sum += s_w[a][v - s_lo[a]];
      if (sum > 0.0)
        for (int v = s_box[a][0]; v <= s_box[a][1]; ++v) s_w[a][v - s_lo[a]] /= sum;
    }
  }
  __syncthreads();

  // 2. forward coupling, staged in LDS chunk by chunk (whole x extent, chunks of y and z)
  const int kx = s_box[0][1] - s_box[0][0] + 1;
  const int ky = s_box[1][1] - s_box[1][0] + 1;
  const int kz = s_box[2][1] - s_box[2][0] + 1;
  const int ex = kx + 2;
  int sy = ky, sz = kz;
  // the window is at most kMax + 2 cells wide in x, so one 3 x 3 chunk column always fits
  static_assert((kMax + 2) * 9 <= CAP, "LDS staging buffer too small");
  while (ex * (sy + 2) * (sz + 2) > CAP) {
    if (sz >= sy && sz > 1)
      --sz;
    else if (sy > 1)
      --sy;
    else
      break;
  }
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int z0 = 0; z0 < kz; z0 += sz) {
    const int cz = kz - z0 < sz ? kz - z0 : sz;
    for (int y0 = 0; y0 < ky; y0 += sy) {
      const int cy = ky - y0 < sy ? ky - y0 : sy;
      const int ey = cy + 2, ez = cz + 2;
      const int tot = ex * ey * ez;
      for (int k = tid; k < tot; k += kThreads) {
        const int lx = k % ex, ly = (k / ex) % ey, lz = k / (ex * ey);
        double v[3];
        ghost_velocity(U, G, s_box[0][0] - 1 + lx, s_box[1][0] + y0 - 1 + ly,
                       s_box[2][0] + z0 - 1 + lz, v);
        s_u[0][k] = (T)v[0];
        s_u[1][k] = (T)v[1];
        s_u[2][k] = (T)v[2];
      }
      __syncthreads();
      const int cells = kx * cy * cz;
      for (int k = tid; k < cells; k += kThreads) {
        const int i = k % kx, j = (k / kx) % cy, l = k / (kx * cy);
        const double W = s_w[0][s_box[0][0] + i - s_lo[0]] * s_w[1][s_box[1][0] + y0 + j - s_lo[1]] *
                         s_w[2][s_box[2][0] + z0 + l - s_lo[2]];
        const int c0 = ((l + 1) * ey + (j + 1)) * ex + (i + 1);
        const int xp = c0 + 1, xm = c0 - 1, yp = c0 + ex, ym = c0 - ex, zp = c0 + ex * ey,
                  zm = c0 - ex * ey;
        const double dUz_dy = 0.5 * ((double)s_u[2][yp] - (double)s_u[2][ym]);
        const double dUy_dz = 0.5 * ((double)s_u[1][zp] - (double)s_u[1][zm]);
        const double dUx_dz = 0.5 * ((double)s_u[0][zp] - (double)s_u[0][zm]);
        const double dUz_dx = 0.5 * ((double)s_u[2][xp] - (double)s_u[2][xm]);
        const double dUy_dx = 0.5 * ((double)s_u[1][xp] - (double)s_u[1][xm]);
        const double dUx_dy = 0.5 * ((double)s_u[0][yp] - (double)s_u[0][ym]);
        acc[0] += W * (double)s_u[0][c0];
        acc[1] += W * (double)s_u[1][c0];
        acc[2] += W * (double)s_u[2][c0];
        acc[3] += W * (dUz_dy - dUy_dz);
        acc[4] += W * (dUx_dz - dUz_dx);
        acc[5] += W * (dUy_dx - dUx_dy);
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const double s = wave_sum(acc[m]);
    if ((tid & 63) == 0) s_red[m][tid >> 6] = s;
  }
  __syncthreads();

  // 3. the bubble ODE on one lane
  if (tid == 0) {
    double ul[3], wl[3];
    for (int m = 0; m < 3; ++m) {
      ul[m] = s_red[m][0] + s_red[m][1] + s_red[m][2] + s_red[m][3];
      wl[m] = s_red[3 + m][0] + s_red[3 + m][1] + s_red[3 + m][2] + s_red[3 + m][3];
    }
    const bubble_params& P = A.P;
    double dul[3] = {0.0, 0.0, 0.0};
    const int st = A.S.state[b];
    if (st == 2) {
      dul[0] = ul[0] - A.S.ulx[b];
      dul[1] = ul[1] - A.S.uly[b];
      dul[2] = ul[2] - A.S.ulz[b];
    }
    const double pi = 3.14159265358979323846;
    const double V = pi * d * d * d / 6.0;
    const double m_eff = P.rho_b * V + P.c_a * P.rho_l * V;
    const double FB = (P.rho_l - P.rho_b) * V * P.g;
    const double Eo = (P.rho_l - P.rho_b) * P.g * d * d / P.sigma;
    const double E = 1.0 / (1.0 + 0.163 * pow(Eo, 0.757));
    const double Eod = Eo / pow(E, 2.0 / 3.0);
    const double dt = 1.0 / P.n_sub;
    double ub[3] = {A.S.ux[b], A.S.uy[b], A.S.uz[b]};
    double xn[3] = {xb[0], xb[1], xb[2]};
    for (int k = 0; k < P.n_sub; ++k) {
      double FD[3], FL[3];
      drag_lift(P, A.nu, d, Eo, Eod, ub, ul, wl, FD, FL);
      for (int a = 0; a < 3; ++a) {
        double f = FD[a] + FL[a] + (1.0 + P.c_a) * P.rho_l * V * dul[a];
        if (a == 2) f += FB;
        ub[a] += dt * f / m_eff;
      }
      for (int a = 0; a < 3; ++a) {
        xn[a] += dt * ub[a];
        if (G.bc[2 * a] == BC_PER) {
          const double L = (double)ext[a];
          xn[a] = fmod(xn[a], L);
          if (xn[a] < 0.0) xn[a] += L;
        } else {
          if (xn[a] < 0.0) {
            xn[a] = 0.0;
            ub[a] = 0.0;
          }
          if (a != 2 && xn[a] > ext[a] - 1.0) {
            xn[a] = ext[a] - 1.0;
            ub[a] = 0.0;
          }
        }
      }
    }
    double FD[3], FL[3];
    drag_lift(P, A.nu, d, Eo, Eod, ub, ul, wl, FD, FL);
    for (int a = 0; a < 3; ++a) s_psi[a] = -(FD[a] + FL[a]);
    A.S.x[b] = xn[0];
    A.S.y[b] = xn[1];
    A.S.z[b] = xn[2];
    A.S.ux[b] = ub[0];
    A.S.uy[b] = ub[1];
    A.S.uz[b] = ub[2];
    A.S.ulx[b] = ul[0];
    A.S.uly[b] = ul[1];
    A.S.ulz[b] = ul[2];
    int nst = 2;
    if (G.bc[4] != BC_PER && xn[2] >= ext[2] - 1.0) nst = 0;  // reached the top layer
    A.S.state[b] = nst;
    if (A.S.psix) {
      A.S.psix[b] = s_psi[0];
      A.S.psiy[b] = s_psi[1];
      A.S.psiz[b] = s_psi[2];
    }
    for (int a = 0; a < 3; ++a) {
      // window at the new position, widened by the curl halo of the next interpolation
      const double nlo = floor(xn[a] - n - 0.5) + 1.0;
      const double nhi = ceil(xn[a] + n + 0.5) - 1.0;
      s_next[a][0] = (int)fmax(nlo, -1e9) - 1;
      s_next[a][1] = (int)fmin(nhi, 1e9) + 1;
    }
  }
  __syncthreads();

  // 4. backward coupling: spread psi W into the force field
  const double psi0 = s_psi[0], psi1 = s_psi[1], psi2 = s_psi[2];
  const int cells = kx * ky * kz;
  for (int k = tid; k < cells; k += kThreads) {
    const int i = k % kx, j = (k / kx) % ky, l = k / (kx * ky);
    const int vi = s_box[0][0] + i - s_lo[0], vj = s_box[1][0] + j - s_lo[1],
              vl = s_box[2][0] + l - s_lo[2];
    const double W = s_w[0][vi] * s_w[1][vj] * s_w[2][vl];
    const uint32_t c = ((uint32_t)s_i[2][vl] * G.ny + s_i[1][vj]) * G.nx + s_i[0][vi];
    atomicAdd(&F[c], (T)(psi0 * W));
    atomicAdd(&F[G.N + c], (T)(psi1 * W));
    atomicAdd(&F[2 * (size_t)G.N + c], (T)(psi2 * W));
  }
  // flag the tiles: the force window now, and the velocity window of the next step
  TileRanges tr[3];
  for (int a = 0; a < 3; ++a) {
    const bool per = G.bc[2 * a] == BC_PER;
    const int lo = min(s_box[a][0], s_next[a][0]);
    const int hi = max(s_box[a][1], s_next[a][1]);
    tr[a] = tile_ranges(lo, hi, ext[a], per);
  }
  for (int rz = 0; rz < tr[2].n; ++rz)
    for (int ry = 0; ry < tr[1].n; ++ry)
      for (int rx = 0; rx < tr[0].n; ++rx) {
        const int nx_ = tr[0].hi[rx] - tr[0].lo[rx] + 1;
        const int ny_ = tr[1].hi[ry] - tr[1].lo[ry] + 1;
        const int nz_ = tr[2].hi[rz] - tr[2].lo[rz] + 1;
        for (int k = tid; k < nx_ * ny_ * nz_; k += kThreads) {
          const int tx = tr[0].lo[rx] + k % nx_;
          const int ty = tr[1].lo[ry] + (k / nx_) % ny_;
          const int tz = tr[2].lo[rz] + k / (nx_ * ny_);
          tiles[((uint32_t)tz * G.tny + ty) * G.tnx + tx] = 1;
        }
      }
}

}  // namespace

hipError_t launch_bubbles(lbm_ctx* c, const bubble_params* p, const bubble_soa* s, int32_t nb) {
  BubbleArgs A;
  A.G = c->geom;
  A.P = *p;
  A.S = *s;
  A.nb = nb;
  A.nu = (1.0 / c->desc.omega - 0.5) / 3.0;  // eq. (9), dx = dt_l = 1
  A.status = c->status;
  hipError_t e = launch_fill(c->tiles, c->ntiles, c->stream);
  if (e != hipSuccess || nb == 0) return e;
  if (c->elem == 4)
    hipLaunchKernelGGL(k_bubbles<float>, dim3(nb), dim3(kThreads), 0, c->stream,
                       static_cast<const float*>(c->vel), static_cast<float*>(c->force), c->tiles, A);
  else
    hipLaunchKernelGGL(k_bubbles<double>, dim3(nb), dim3(kThreads), 0, c->stream,
                       static_cast<const double*>(c->vel), static_cast<double*>(c->force), c->tiles,
                       A);
  return hipGetLastError();
}

}  // namespace lbm
