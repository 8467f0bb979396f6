// Adjoint (reverse-mode derivative) of one method step of Algorithm 1, for gradients of a loss on
// bubble trajectories with respect to the drag scale, the lift scale and omega.
//
// Liquid step, k_adj_liquid: with lam = dL/d(post-collision buffer after the step), each cell
// rebuilds its pre-collision populations p = pull(h) and force, applies the transposed Jacobian
// of the collision (collide_cell_adjoint) and scatters the result to the sources of its pull.
// Streaming with the face rules is a permutation of (cell, population), so the scatter writes
// every element of the output exactly once.
//
// Bubble half, k_adj_bubble: one workgroup per bubble runs the transposes of the three forward
// bubble kernels in reverse order (spreading, sub-stepped ODE, interpolation).
#include <algorithm>
#include <utility>

#include "adjoint_math.hpp"
#include "collide.hpp"
#include "step_cell.hpp"

namespace lbm {
namespace {

constexpr int kB = 256;  // threads per bubble workgroup
constexpr int kBW = kB / 64;
static_assert(kRecordMaxSub == kMaxSub, "the record holds every sub-step the adjoint allows");
// adjoint bubble state (doubles)
constexpr int A_X = 0, A_UB = 3, A_ULP = 6, A_SIZE = LBM_BUBBLE_ADJ;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double bsum(double v, double* s_red) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < kBW; ++w) t += s_red[w];
  return t;
}

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

template <bool GENERAL, typename T, int... Qs>
__device__ __forceinline__ void push_all(T* __restrict__ dst, const T* mu, const Geom& G,
                                         uint32_t lc, const CellNbr& nb,
                                         std::integer_sequence<int, Qs...>) {
  ((dst[pull_index<Qs, GENERAL>(G, lc, nb)] = mu[Qs]), ...);
}

template <typename T, bool GENERAL>
__global__ __launch_bounds__(256) void k_adj_liquid(const T* __restrict__ h, const T* __restrict__ F,
                                                    const T* __restrict__ lam_next,
                                                    T* __restrict__ lam_prev, T* __restrict__ lam_u,
                                                    T* __restrict__ lam_f, Geom G, T omega,
                                                    double* __restrict__ grad) {
  __shared__ double s_red[4];
  const uint32_t cell = blockIdx.x * 256 + threadIdx.x;
  double dom = 0.0;
  if (cell < G.N) {
    const uint32_t x = cell % G.nx, y = (cell / G.nx) % G.ny, z = cell / G.plane;
    const CellNbr nb = cell_neighbours(G, (int)x, (int)y, (int)z);
    const uint32_t lc = layout_cell(G, cell, z);
    T p[19], lam[19], mu[19];
    pull_all<GENERAL>(p, h, G, lc, nb, std::make_integer_sequence<int, 19>{});
#pragma unroll
    for (int q = 0; q < 19; ++q) lam[q] = lam_next[(size_t)q * G.qs + lc];
    const T f[3] = {F[cell], F[G.N + cell], F[2 * (size_t)G.N + cell]};
    const T lu[3] = {lam_u[cell], lam_u[G.N + cell], lam_u[2 * (size_t)G.N + cell]};
    T lf[3];
    collide_cell_adjoint<T>(p, f, omega, lam, lu, mu, lf, &dom);
    push_all<GENERAL>(lam_prev, mu, G, lc, nb, std::make_integer_sequence<int, 19>{});
    lam_f[cell] = lf[0];
    lam_f[G.N + cell] = lf[1];
    lam_f[2 * (size_t)G.N + cell] = lf[2];
    // consumed: the next (earlier) step accumulates its own velocity adjoint here
    lam_u[cell] = T(0);
    lam_u[G.N + cell] = T(0);
    lam_u[2 * (size_t)G.N + cell] = T(0);
  }
  dom = wsum(dom);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = dom;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&grad[0], s_red[0] + s_red[1] + s_red[2] + s_red[3]);
}

template <typename T, int... Qs>
__device__ __forceinline__ void pull_push_bb(T* p, const T* __restrict__ h, const Geom& G, uint32_t lc4,
                                             uint32_t walls, std::integer_sequence<int, Qs...>) {
  ((p[Qs] = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(h) +
                                         pull_off_bb<Qs, T>(G, lc4, walls))),
   ...);
}

template <typename T, int... Qs>
__device__ __forceinline__ void push_bb(T* __restrict__ dst, const T* mu, const Geom& G, uint32_t lc4,
                                        uint32_t walls, std::integer_sequence<int, Qs...>) {
  ((*at_bytes(dst, pull_off_bb<Qs, T>(G, lc4, walls)) = mu[Qs]), ...);
}

// The same on the bounce-back fast path (every face bounce-back, byte offsets below 4 GiB): every
// access is a scalar base plus a 32-bit byte offset, and the push goes to the byte offsets the
// pull read from. The dL/domega partial of each workgroup goes to one of nbins bins (atomic adds
// spread over the bins instead of one address), summed by k_bins. In FP32 the compiler is held to
// four wavefronts per SIMD (116 VGPRs, no spills; a bound of five spills); in FP64 any such bound
// spills. tiles (or null: every tile): the step's tile mask; outside its flagged tiles F and lam_u
// are zero (the step neither forced nor wrote the velocity there), so a cell there takes them as
// zero without reading them and leaves lam_u and lam_f alone: 228 bytes per cell instead of 276.
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 4 : 1) void k_adj_liquid_bb(const T* __restrict__ h,
                                                       const T* __restrict__ F,
                                                       const T* __restrict__ lam_next,
                                                       T* __restrict__ lam_prev,
                                                       T* __restrict__ lam_u, T* __restrict__ lam_f,
                                                       const uint8_t* __restrict__ tiles,
                                                       Geom G, T omega, double* __restrict__ bins,
                                                       uint32_t nbins) {
  __shared__ double s_red[4];
  const uint32_t cell = blockIdx.x * 256 + threadIdx.x;
  double dom = 0.0;
  if (cell < G.N) {
    const uint32_t z = cell / G.plane, rem = cell - z * G.plane;
    const uint32_t y = rem / (uint32_t)G.nx, x = rem - y * (uint32_t)G.nx;
    constexpr uint32_t esz = sizeof(T);
    const uint32_t lc4 = layout_cell(G, cell, z) * esz;
    const uint32_t walls = wall_bits(G, (int)x, (int)y, z);
    const uint32_t c4 = cell * esz, n4 = G.N * esz, qs4 = G.qs * esz;
    T p[19], lam[19], mu[19];
    pull_push_bb<T>(p, h, G, lc4, walls, std::make_integer_sequence<int, 19>{});
#pragma unroll
    for (int q = 0; q < 19; ++q) lam[q] = *at_bytes(lam_next, lc4 + (uint32_t)q * qs4);
    const bool touched =
        !tiles || tiles[((z >> 3) * (uint32_t)G.tny + (y >> 3)) * (uint32_t)G.tnx + (x >> 3)] != 0;
    T f[3] = {T(0), T(0), T(0)}, lu[3] = {T(0), T(0), T(0)};
    if (touched) {
      f[0] = *at_bytes(F, c4);
      f[1] = *at_bytes(F, c4 + n4);
      f[2] = *at_bytes(F, c4 + 2 * n4);
      lu[0] = *at_bytes(lam_u, c4);
      lu[1] = *at_bytes(lam_u, c4 + n4);
      lu[2] = *at_bytes(lam_u, c4 + 2 * n4);
    }
    T lf[3];
    collide_cell_adjoint<T>(p, f, omega, lam, lu, mu, lf, &dom);
    push_bb<T>(lam_prev, mu, G, lc4, walls, std::make_integer_sequence<int, 19>{});
    if (touched) {
      *at_bytes(lam_f, c4) = lf[0];
      *at_bytes(lam_f, c4 + n4) = lf[1];
      *at_bytes(lam_f, c4 + 2 * n4) = lf[2];
      // consumed: the next (earlier) step accumulates its own velocity adjoint here
      *at_bytes(lam_u, c4) = T(0);
      *at_bytes(lam_u, c4 + n4) = T(0);
      *at_bytes(lam_u, c4 + 2 * n4) = T(0);
    }
  }
  dom = wsum(dom);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = dom;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicAdd(&bins[blockIdx.x % nbins], s_red[0] + s_red[1] + s_red[2] + s_red[3]);
}

// grad[0] += sum of the bins, in a fixed order; the bins are left at zero.
__global__ __launch_bounds__(64) void k_bins(double* __restrict__ bins, uint32_t nbins,
                                             double* __restrict__ grad) {
  double v = 0.0;
  if (threadIdx.x < nbins) {
    v = bins[threadIdx.x];
    bins[threadIdx.x] = 0.0;
  }
  v = wsum(v);
  if (threadIdx.x == 0) grad[0] += v;
}

// Weights of axis AX with their derivatives in the bubble coordinate, computed by one wavefront
// and stored in LDS, indexed by cell - lo + 1 (the forward's weights bit for bit: the same terms,
// the same butterfly sum, the same renormalisation). Lane l holds entries l and l + 64 (kAdjSpan
// = 66: lanes 0 and 1 hold a second one); the curl weights take their neighbours by shuffles,
// so the wavefront needs no barrier. Returns false (every lane) if the window is too large.
template <int AX>
__device__ bool wave_weights_dx(const Geom& G, const double* xb, double n, int lane,
                                double (*w)[kAdjSpan], double (*dw)[kAdjSpan],
                                double (*wx)[kAdjSpan], double (*dwx)[kAdjSpan], AxisW* win) {
  static_assert(kAdjSpan > 64 && kAdjSpan <= 128, "two entries per lane");
  const int ext = AX == 0 ? G.nx : (AX == 1 ? G.ny : G.nz);
  const bool per = G.bc[2 * AX] == BC_PER;
  const double s_lo = G.bc[2 * AX] == BC_FS ? 1.0 : -1.0;
  const double s_hi = G.bc[2 * AX + 1] == BC_FS ? 1.0 : -1.0;
  const double x = xb[AX];
  AxisW A;
  if (!axis_window_hd(x, n, ext, per, A)) return false;
  const int i0 = lane, i1 = lane + 64;
  auto entry = [&](int i, double& wi, double& di) {
    const int v = A.lo - 1 + i;
    wi = 0.0;
    di = 0.0;
    if (i < kAdjSpan && v >= A.clo && v <= A.chi) {
      const double sp = (v + 0.5 - x) / n, sm = (v - 0.5 - x) / n;
      wi = kernel_P(sp) - kernel_P(sm);
      di = -(kernel_dP(sp) - kernel_dP(sm)) / n;
    }
  };
  double w0, w1, d0, d1;
  entry(i0, w0, d0);
  entry(i1, w1, d1);
  if (!per) {  // clipped at a wall: renormalise, d(w/S) = (dw - (w/S) dS) / S
    const double sum = wsum(w0 + w1), dsum = wsum(d0 + d1);
    if (sum > 0.0) {
      w0 /= sum;
      w1 /= sum;
      d0 = (d0 - w0 * dsum) / sum;
      d1 = (d1 - w1 * dsum) / sum;
    }
  }
  // neighbours: entry l - 1 and l + 1 of entry l; entry 63, 64 and 65 for the second entries
  const int up = (lane + 63) & 63, dn = (lane + 1) & 63;
  const double wu = __shfl(w0, up, 64), wd = __shfl(w0, dn, 64);
  const double du = __shfl(d0, up, 64), dd = __shfl(d0, dn, 64);
  const double w64 = __shfl(w1, 0, 64), w65 = __shfl(w1, 1, 64);
  const double d64 = __shfl(d1, 0, 64), d65 = __shfl(d1, 1, 64);
  auto curl = [&](int i, double wi, double di, double wm, double wp, double xm, double xp) {
    const int v = A.lo - 1 + i;
    double c = 0.5 * (wm - wp), cx = 0.5 * (xm - xp);
    if (!per) {
      if (v == 0) {
        c -= 0.5 * s_lo * wi;
        cx -= 0.5 * s_lo * di;
      }
      if (v == ext - 1) {
        c += 0.5 * s_hi * wi;
        cx += 0.5 * s_hi * di;
      }
    }
    w[AX][i] = wi;
    wx[AX][i] = di;
    dw[AX][i] = c;
    dwx[AX][i] = cx;
  };
  curl(i0, w0, d0, lane > 0 ? wu : 0.0, lane < 63 ? wd : w64, lane > 0 ? du : 0.0,
       lane < 63 ? dd : d64);
  if (i1 < kAdjSpan) {
    const bool first = lane == 0;  // entry 64 (neighbours 63, 65), else entry 65 (64, none)
    curl(i1, w1, d1, first ? wu : w64, first ? w65 : 0.0, first ? du : d64, first ? d65 : 0.0);
  }
  if (lane == 0) win[AX] = A;
  return true;
}

// The six sums of the gather over the workgroup behind one barrier (the order of bsum).
__device__ __forceinline__ void bsum6(double v[6], double (*s_red6)[kBW]) {
#pragma unroll
  for (int m = 0; m < 6; ++m) v[m] = wsum(v[m]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int m = 0; m < 6; ++m) s_red6[m][threadIdx.x >> 6] = v[m];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    double t = 0.0;
    for (int w = 0; w < kBW; ++w) t += s_red6[m][w];
    v[m] = t;
  }
}

// Window entries f = tid, tid + kB, ... of a box Dx x Dy x Dz as f = i + Dx (j + Dy k), stepped
// by kB entries with carries.
struct WindowWalk {
  int Dx, Dy, i, j, k, di, dj, dk;
  __device__ WindowWalk(int Dx_, int Dy_, int f) : Dx(Dx_), Dy(Dy_) {
    i = f % Dx;
    j = (f / Dx) % Dy;
    k = f / Dx / Dy;
    di = kB % Dx;
    dj = (kB / Dx) % Dy;
    dk = kB / Dx / Dy;
  }
  __device__ void advance() {
    i += di;
    const int carry = i >= Dx;
    if (carry) i -= Dx;
    j += dj + carry;
    if (j >= Dy) {
      j -= Dy;
      ++k;
    }
    k += dk;
  }
};

// The bubble half of the adjoint for one bubble per workgroup:
//   wavefronts 0-2   the weights of axis 0, 1, 2 (with their derivatives), side by side with
//   wavefront 3      the sub-step velocities and clamp flags: from the record when the forward
//                    update wrote them, else the forward sub-steps again (one lane);
//   all              the gather dL/dpsi = sum_j W_j dL/dF(j) and the position term of the spreading
//                    weights, while lanes of wavefront 3 first evaluate the n_sub + 1 force
//                    Jacobians at the recorded velocities;
//   lane 0           the reverse sweep of the sub-steps (ode_adjoint_sweep), while every thread
//                    loads the velocities of its first scatter cells;
//   all              the scatter, transpose of the interpolation: dL/dU(j) += W_j dL/du_l + curl
//                    weights . dL/dw_l (atomic adds), and the position term of the interpolation.
template <typename T>
__global__ __launch_bounds__(kB) void k_adj_bubble(const T* __restrict__ lam_f,
                                                   const T* __restrict__ U, T* __restrict__ lam_u,
                                                   const double* __restrict__ rec,
                                                   double* __restrict__ lam,
                                                   const double* __restrict__ lam_x, bubble_params P,
                                                   Geom G, double nu, double dnu_domega, int nb,
                                                   double* __restrict__ grad) {
  __shared__ double w[3][kAdjSpan], dw[3][kAdjSpan], wx[3][kAdjSpan], dwx[3][kAdjSpan];
  __shared__ AxisW win[3];
  __shared__ int s_bad[3];
  __shared__ double s_red6[6][kBW];
  __shared__ double s_lul[3], s_lwl[3];
  __shared__ double s_ubs[kMaxSub + 1][3];
  __shared__ unsigned char s_clamped[kMaxSub][3];
  __shared__ ForceJac s_jac[kMaxSub + 1];
  const int b = (int)xcd_remap(blockIdx.x, nb);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const double* r = rec + (size_t)b * R_SIZE;
  double* l = lam + (size_t)b * A_SIZE;
  // the loss's own term in the positions after the step (lane 0 alone reads and writes l[A_X])
  if (lam_x && tid == 0)
    for (int a = 0; a < 3; ++a) l[A_X + a] += lam_x[(size_t)a * nb + b];
  const int st = (int)r[R_STATE];
  // a frozen bubble (inactive, or no valid window in the step): its adjoint state passes through
  if (st == 0 || r[R_VALID] == 0.0) return;
  const double xb[3] = {r[R_X], r[R_X + 1], r[R_X + 2]};
  const double* ul = r + R_UL;
  const double* ulp = r + R_ULP;
  double dul[3] = {0.0, 0.0, 0.0};
  if (st == 2)
    for (int a = 0; a < 3; ++a) dul[a] = ul[a] - ulp[a];

  // weights (wavefronts 0-2) beside the forward sub-steps (wavefront 3)
  if (wave < 3) {
    const double n = P.kernel_factor * r[R_D];
    bool ok;
    if (wave == 0)
      ok = wave_weights_dx<0>(G, xb, n, lane, w, dw, wx, dwx, win);
    else if (wave == 1)
      ok = wave_weights_dx<1>(G, xb, n, lane, w, dw, wx, dwx, win);
    else
      ok = wave_weights_dx<2>(G, xb, n, lane, w, dw, wx, dwx, win);
    if (lane == 0) s_bad[wave] = ok ? 0 : 1;
  } else if (r[R_SUB] != 0.0) {
    // sub-step velocities and clamp flags recorded by the forward update
    if (lane <= P.n_sub)
      for (int a = 0; a < 3; ++a) s_ubs[lane][a] = r[R_UBS + 3 * lane + a];
    if (lane < P.n_sub)
      for (int a = 0; a < 3; ++a) {
        const int bit = 3 * lane + a;
        s_clamped[lane][a] = (unsigned char)(((uint32_t)r[R_CLAMP + bit / 32] >> (bit % 32)) & 1u);
      }
  } else if (lane == 0) {
    OdeBounds Bd;
    const int ext[3] = {G.nx, G.ny, G.nz};
    for (int a = 0; a < 3; ++a) {
      Bd.hi[a] = ext[a] - 1.0;
      Bd.len[a] = G.bc[2 * a] == BC_PER ? (double)ext[a] : 0.0;
    }
    Bd.top = G.bc[4] != BC_PER;
    OdeOut o;
    ode_forward(P, nu, r[R_D], r + R_X, r + R_UB, ul, r + R_WL, dul, Bd, o, s_ubs, s_clamped);
  }
  __syncthreads();
  if (s_bad[0] | s_bad[1] | s_bad[2]) return;  // the forward step flagged this bubble's window
  const bool px = G.bc[0] == BC_PER, py = G.bc[2] == BC_PER, pz = G.bc[4] == BC_PER;
  auto cell = [&](int vx, int vy, int vz) {
    const int x = px ? wrapi(vx, G.nx) : vx, y = py ? wrapi(vy, G.ny) : vy,
              z = pz ? wrapi(vz, G.nz) : vz;
    return ((uint32_t)z * G.ny + y) * G.nx + x;
  };
  constexpr int kBatch = 8;  // cells per thread whose loads are in flight together

  // force Jacobians at the sub-step velocities (lanes of wavefront 3), then the gather
  if (wave == 3 && lane <= P.n_sub) {
    const ForceConst fc = force_const(P, nu, r[R_D]);
    force_jac(P, fc, nu, r[R_D], s_ubs[lane], ul, r + R_WL, s_jac[lane]);
  }
  double acc[6] = {0, 0, 0, 0, 0, 0};
  {
    const double psi[3] = {r[R_PSI], r[R_PSI + 1], r[R_PSI + 2]};
    const int Kx = win[0].chi - win[0].clo + 1, Ky = win[1].chi - win[1].clo + 1,
              Kz = win[2].chi - win[2].clo + 1;
    const int total = Kx * Ky * Kz;
    WindowWalk it(Kx, Ky, tid);
    for (int f0 = tid; f0 < total; f0 += kBatch * kB) {
      int ix[kBatch], iy[kBatch], iz[kBatch];
      T lf[kBatch][3];
#pragma clang loop unroll(full)
      for (int s = 0; s < kBatch; ++s) {
        if (f0 + s * kB < total) {
          const int vx = win[0].clo + it.i, vy = win[1].clo + it.j, vz = win[2].clo + it.k;
          ix[s] = vx - win[0].lo + 1;
          iy[s] = vy - win[1].lo + 1;
          iz[s] = vz - win[2].lo + 1;
          const uint32_t c = cell(vx, vy, vz);
          lf[s][0] = lam_f[c];
          lf[s][1] = lam_f[G.N + c];
          lf[s][2] = lam_f[2 * (size_t)G.N + c];
          it.advance();
        }
      }
#pragma clang loop unroll(full)
      for (int s = 0; s < kBatch; ++s) {
        if (f0 + s * kB < total) {
          const double l0 = (double)lf[s][0], l1 = (double)lf[s][1], l2 = (double)lf[s][2];
          const double a = w[0][ix[s]], bb = w[1][iy[s]], cc = w[2][iz[s]];
          const double W = a * bb * cc;
          const double pl = psi[0] * l0 + psi[1] * l1 + psi[2] * l2;
          acc[0] += W * l0;
          acc[1] += W * l1;
          acc[2] += W * l2;
          acc[3] += wx[0][ix[s]] * bb * cc * pl;
          acc[4] += a * wx[1][iy[s]] * cc * pl;
          acc[5] += a * bb * wx[2][iz[s]] * pl;
        }
      }
    }
  }
  bsum6(acc, s_red6);  // every thread now holds dL/dpsi (0-2) and the spreading position term

  // the reverse sweep (lane 0) while every thread loads its first scatter cells
  const int Dx = win[0].dhi - win[0].dlo + 1, Dy = win[1].dhi - win[1].dlo + 1,
            Dz = win[2].dhi - win[2].dlo + 1;
  const int dtotal = Dx * Dy * Dz;
  WindowWalk it(Dx, Dy, tid);
  int ix[kBatch], iy[kBatch], iz[kBatch];
  uint32_t cs[kBatch];
  T u[kBatch][3];
  auto load_batch = [&](int f0) {
#pragma clang loop unroll(full)
    for (int s = 0; s < kBatch; ++s) {
      if (f0 + s * kB < dtotal) {
        const int vx = win[0].dlo + it.i, vy = win[1].dlo + it.j, vz = win[2].dlo + it.k;
        ix[s] = vx - win[0].lo + 1;
        iy[s] = vy - win[1].lo + 1;
        iz[s] = vz - win[2].lo + 1;
        cs[s] = cell(vx, vy, vz);
        u[s][0] = U[cs[s]];
        u[s][1] = U[G.N + cs[s]];
        u[s][2] = U[2 * (size_t)G.N + cs[s]];
        it.advance();
      }
    }
  };
  load_batch(tid);
  double gxode[3] = {0.0, 0.0, 0.0};
  if (tid == 0) {
    const double lpsi[3] = {acc[0], acc[1], acc[2]};
    OdeAdj g;
    ode_adjoint_sweep(P, r[R_D], s_clamped, s_jac, l + A_X, l + A_UB, lpsi, g);
    for (int a = 0; a < 3; ++a) {
      // u_l enters the drag/lift, D_t u_l = u_l - u_l,prev (state 2) and u_l,prev of the next step
      s_lul[a] = g.ul[a] + (st == 2 ? g.dul[a] : 0.0) + l[A_ULP + a];
      s_lwl[a] = g.wl[a];
      gxode[a] = g.x[a];
      l[A_UB + a] = g.ub[a];
      l[A_ULP + a] = st == 2 ? -g.dul[a] : 0.0;
    }
    atomicAdd(&grad[1], g.dsD);
    atomicAdd(&grad[2], g.dsL);
    atomicAdd(&grad[3], g.dnu);
    // omega reaches the closures through nu = (1/omega - 1/2)/3 (eq. (9))
    atomicAdd(&grad[0], g.dnu * dnu_domega);
  }
  __syncthreads();

  // scatter
  const double lu[3] = {s_lul[0], s_lul[1], s_lul[2]};
  const double lw[3] = {s_lwl[0], s_lwl[1], s_lwl[2]};
  double gx[6] = {0, 0, 0, 0, 0, 0};  // 3-5 unused: the six-sum reduction
  for (int f0 = tid; f0 < dtotal; f0 += kBatch * kB) {
    if (f0 != tid) load_batch(f0);
#pragma clang loop unroll(full)
    for (int s = 0; s < kBatch; ++s) {
      if (f0 + s * kB >= dtotal) continue;
      const uint32_t c = cs[s];
      const double a = w[0][ix[s]], da = dw[0][ix[s]], bb = w[1][iy[s]], db = dw[1][iy[s]],
                   cc = w[2][iz[s]], dc = dw[2][iz[s]];
      // forward: ul += W U; wx += Uz a db c - Uy a b dc; wy += Ux a b dc - Uz da b c;
      //          wz += Uy da b c - Ux a db c
      const double W = a * bb * cc, adbc = a * db * cc, abdc = a * bb * dc, dabc = da * bb * cc;
      const double gUx = W * lu[0] + abdc * lw[1] - adbc * lw[2];
      const double gUy = W * lu[1] - abdc * lw[0] + dabc * lw[2];
      const double gUz = W * lu[2] + adbc * lw[0] - dabc * lw[1];
      if (gUx != 0.0) atomicAdd(&lam_u[c], (T)gUx);
      if (gUy != 0.0) atomicAdd(&lam_u[G.N + c], (T)gUy);
      if (gUz != 0.0) atomicAdd(&lam_u[2 * (size_t)G.N + c], (T)gUz);
      const double ux = (double)u[s][0], uy = (double)u[s][1], uz = (double)u[s][2];
      // derivative of the same sums in the bubble coordinate along each axis
      const double ax = wx[0][ix[s]], dax = dwx[0][ix[s]], by = wx[1][iy[s]], dby = dwx[1][iy[s]],
                   cz = wx[2][iz[s]], dcz = dwx[2][iz[s]];
      {  // x: a -> ax, da -> dax
        const double Wd = ax * bb * cc, adbc_d = ax * db * cc, abdc_d = ax * bb * dc, dabc_d = dax * bb * cc;
        gx[0] += lu[0] * Wd * ux + lu[1] * Wd * uy + lu[2] * Wd * uz +
                 lw[0] * (uz * adbc_d - uy * abdc_d) + lw[1] * (ux * abdc_d - uz * dabc_d) +
                 lw[2] * (uy * dabc_d - ux * adbc_d);
      }
      {  // y: b -> by, db -> dby
        const double Wd = a * by * cc, adbc_d = a * dby * cc, abdc_d = a * by * dc, dabc_d = da * by * cc;
        gx[1] += lu[0] * Wd * ux + lu[1] * Wd * uy + lu[2] * Wd * uz +
                 lw[0] * (uz * adbc_d - uy * abdc_d) + lw[1] * (ux * abdc_d - uz * dabc_d) +
                 lw[2] * (uy * dabc_d - ux * adbc_d);
      }
      {  // z: c -> cz, dc -> dcz
        const double Wd = a * bb * cz, adbc_d = a * db * cz, abdc_d = a * bb * dcz, dabc_d = da * bb * cz;
        gx[2] += lu[0] * Wd * ux + lu[1] * Wd * uy + lu[2] * Wd * uz +
                 lw[0] * (uz * adbc_d - uy * abdc_d) + lw[1] * (ux * abdc_d - uz * dabc_d) +
                 lw[2] * (uy * dabc_d - ux * adbc_d);
      }
    }
  }
  // s_red6 is free again: every thread read its gather sums before the sweep's barrier
  bsum6(gx, s_red6);
  if (tid == 0)
    for (int a = 0; a < 3; ++a) l[A_X + a] = gxode[a] + acc[3 + a] + gx[a];
}

// Step record of every bubble (one lane per bubble): stage 0, before the step's bubble half, takes
// x, u_b, u_l,prev, state and d from the bubble arrays; stage 1, after it, takes u_l, w_l, psi and
// the window flag from the bubble workspace. (An armed record is filled by the bubble update
// itself, sub-steps included.)
__global__ __launch_bounds__(64) void k_record(bubble_soa S, int nb, int stage, double* __restrict__ rec) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= nb) return;
  double* r = rec + (size_t)b * R_SIZE;
  if (stage == 0) {
    r[R_X] = S.x[b];
    r[R_X + 1] = S.y[b];
    r[R_X + 2] = S.z[b];
    r[R_UB] = S.ux[b];
    r[R_UB + 1] = S.uy[b];
    r[R_UB + 2] = S.uz[b];
    r[R_ULP] = S.ulx[b];
    r[R_ULP + 1] = S.uly[b];
    r[R_ULP + 2] = S.ulz[b];
    r[R_STATE] = (double)S.state[b];
    r[R_D] = S.d[b];
    r[R_SUB] = 0.0;  // the sub-steps are not recorded: the adjoint runs them again
  } else {
    const double* wk = S.work + (size_t)b * LBM_BUBBLE_WORK;
    for (int m = 0; m < 6; ++m) r[R_UL + m] = wk[W_UL + m];  // u_l then w_l
    for (int m = 0; m < 3; ++m) r[R_PSI + m] = wk[W_PSI + m];
    r[R_VALID] = wk[W_VALID];
  }
}

// Records the armed timing events (lbm_time_next_adjoint_liquid) around one launch, then disarms.
template <typename F>
hipError_t timed_adjoint(lbm_ctx* c, F&& launch) {
  hipEvent_t a = c->ta_start, b = c->ta_end;
  c->ta_start = c->ta_end = nullptr;
  hipError_t e = a ? hipEventRecord(a, c->stream) : hipSuccess;
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess && b) e = hipEventRecord(b, c->stream);
  return e;
}

template <typename T, bool GENERAL>
hipError_t liquid_typed(lbm_ctx* c, const void* state, const void* force, const void* lam_next,
                        void* lam_prev, void* lam_u, void* lam_f, const uint8_t* tiles,
                        double* grad) {
  if (!GENERAL && bb_fast_ok(c->geom, sizeof(T))) {
    // bins for the dL/domega partials: the moments reduction scratch (at least 64 doubles for
    // lattices of 4096 cells or more)
    const uint32_t nbins = std::min<uint32_t>(64, c->nred * 4);
    hipError_t e = hipSuccess;
    if (!c->bins_clean) e = launch_fill(c->partials, nbins * sizeof(double), c->stream);
    if (e != hipSuccess) return e;
    e = timed_adjoint(c, [&] {
      hipLaunchKernelGGL((k_adj_liquid_bb<T>), dim3(div_up(c->geom.N, 256)), dim3(256), 0,
                         c->stream, static_cast<const T*>(state), static_cast<const T*>(force),
                         static_cast<const T*>(lam_next), static_cast<T*>(lam_prev),
                         static_cast<T*>(lam_u), static_cast<T*>(lam_f), tiles, c->geom,
                         (T)c->desc.omega, c->partials, nbins);
      return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bins, dim3(1), dim3(64), 0, c->stream, c->partials, nbins, grad);
    e = hipGetLastError();
    c->bins_clean = e == hipSuccess;
    return e;
  }
  return timed_adjoint(c, [&] {
    hipLaunchKernelGGL((k_adj_liquid<T, GENERAL>), dim3(div_up(c->geom.N, 256)), dim3(256), 0,
                       c->stream, static_cast<const T*>(state), static_cast<const T*>(force),
                       static_cast<const T*>(lam_next), static_cast<T*>(lam_prev),
                       static_cast<T*>(lam_u), static_cast<T*>(lam_f), c->geom, (T)c->desc.omega,
                       grad);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t bubbles_typed(lbm_ctx* c, const bubble_params* p, const double* rec, const void* vel_prev,
                         const void* lam_f, void* lam_u, double* lam, const double* lam_x, int32_t nb,
                         double* grad) {
  const double nu = (1.0 / c->desc.omega - 0.5) / 3.0;
  const double dnu_domega = -1.0 / (3.0 * c->desc.omega * c->desc.omega);
  hipLaunchKernelGGL((k_adj_bubble<T>), dim3(nb), dim3(kB), 0, c->stream,
                     static_cast<const T*>(lam_f), static_cast<const T*>(vel_prev),
                     static_cast<T*>(lam_u), rec, lam, lam_x, *p, c->geom, nu, dnu_domega, nb, grad);
  return hipGetLastError();
}

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" {

lbm_status lbm_adjoint_liquid_tiles(lbm_ctx* ctx, const void* state, const void* force,
                                    const void* lam_next, void* lam_prev, void* lam_u, void* lam_f,
                                    const uint8_t* tiles, double* grad) {
  if (!ctx || !state || !force || !lam_next || !lam_prev || !lam_u || !lam_f || !grad)
    return LBM_EINVAL;
  if (lam_next == lam_prev) return LBM_EINVAL;
  // a static force field is read everywhere: the mask does not bound it
  if (ctx->desc.flags & LBM_FLAG_STATIC_FORCE) tiles = nullptr;
  hipError_t e;
  if (ctx->elem == 4)
    e = ctx->general
            ? liquid_typed<float, true>(ctx, state, force, lam_next, lam_prev, lam_u, lam_f, tiles, grad)
            : liquid_typed<float, false>(ctx, state, force, lam_next, lam_prev, lam_u, lam_f, tiles, grad);
  else
    e = ctx->general
            ? liquid_typed<double, true>(ctx, state, force, lam_next, lam_prev, lam_u, lam_f, tiles, grad)
            : liquid_typed<double, false>(ctx, state, force, lam_next, lam_prev, lam_u, lam_f, tiles, grad);
  return e == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_adjoint_liquid(lbm_ctx* ctx, const void* state, const void* force,
                              const void* lam_next, void* lam_prev, void* lam_u, void* lam_f,
                              double* grad) {
  return lbm_adjoint_liquid_tiles(ctx, state, force, lam_next, lam_prev, lam_u, lam_f, nullptr,
                                  grad);
}

lbm_status lbm_time_next_adjoint_liquid(lbm_ctx* ctx, void* start, void* end) {
  if (!ctx) return LBM_EINVAL;
  ctx->ta_start = static_cast<hipEvent_t>(start);
  ctx->ta_end = static_cast<hipEvent_t>(end);
  return LBM_OK;
}

lbm_status lbm_adjoint_bubbles(lbm_ctx* ctx, const bubble_params* p, const double* record,
                               const void* vel_prev, const void* lam_f, void* lam_u, double* lam,
                               const double* lam_x, int32_t nb, double* grad) {
  if (!ctx || !p || nb < 0 || !grad) return LBM_EINVAL;
  if (nb == 0) return LBM_OK;
  if (!record || !vel_prev || !lam_f || !lam_u || !lam) return LBM_EINVAL;
  if (p->n_sub < 1 || p->n_sub > kMaxSub) return LBM_EINVAL;
  if (p->coupling != 0) return LBM_EUNSUPPORTED;  // the adjoint of the default coupling only
  const hipError_t e =
      ctx->elem == 4 ? bubbles_typed<float>(ctx, p, record, vel_prev, lam_f, lam_u, lam, lam_x, nb, grad)
                     : bubbles_typed<double>(ctx, p, record, vel_prev, lam_f, lam_u, lam, lam_x, nb, grad);
  return e == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_bubble_record(lbm_ctx* ctx, const bubble_soa* soa, int32_t nb, int32_t stage,
                             double* record) {
  if (!ctx || !soa || nb < 0 || (stage != 0 && stage != 1)) return LBM_EINVAL;
  if (nb == 0) return LBM_OK;
  if (!record) return LBM_EINVAL;
  if (stage == 0 && (!soa->x || !soa->y || !soa->z || !soa->ux || !soa->uy || !soa->uz ||
                     !soa->ulx || !soa->uly || !soa->ulz || !soa->state || !soa->d))
    return LBM_EINVAL;
  if (stage == 1 && !soa->work) return LBM_EINVAL;
  hipLaunchKernelGGL(k_record, dim3(div_up((uint32_t)nb, 64)), dim3(64), 0, ctx->stream, *soa, nb,
                     stage, record);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

// ---- host evaluation of the same arithmetic (for checks on a CPU) ----

lbm_status lbm_host_collide(const double* p, const double* F, double omega, const double* lam,
                            const double* lam_u, double* out, double* u, double* mu, double* lam_f,
                            double* domega) {
  if (!p || !F) return LBM_EINVAL;
  double o[19], uu[3];
  collide_cell<double>(p, F, omega, o, uu);
  if (out)
    for (int q = 0; q < 19; ++q) out[q] = o[q];
  if (u)
    for (int a = 0; a < 3; ++a) u[a] = uu[a];
  if (lam && lam_u && mu && lam_f && domega)
    collide_cell_adjoint<double>(p, F, omega, lam, lam_u, mu, lam_f, domega);
  return LBM_OK;
}

lbm_status lbm_host_axis_weights(double x, double n, int32_t ext, int32_t periodic, double s_lo,
                                 double s_hi, int32_t* lo, double* w, double* dw, double* wx,
                                 double* dwx) {
  if (!lo || !w || !dw || !wx || !dwx || ext < 1 || !(n > 0.0)) return LBM_EINVAL;
  AxisW A;
  if (!axis_weights_dx(x, n, ext, periodic != 0, s_lo, s_hi, A, w, dw, wx, dwx)) return LBM_EINVAL;
  *lo = A.lo;
  return LBM_OK;
}

lbm_status lbm_host_bubble_ode(const bubble_params* p, double nu, double d, const double* x0,
                               const double* ub0, const double* ul, const double* wl,
                               const double* dul, const int32_t* ext, const int32_t* periodic,
                               double* x, double* ub, double* psi) {
  if (!p || !x0 || !ub0 || !ul || !wl || !dul || !ext || !periodic || !x || !ub || !psi)
    return LBM_EINVAL;
  if (p->n_sub < 1 || p->n_sub > kMaxSub) return LBM_EINVAL;
  OdeBounds Bd;
  for (int a = 0; a < 3; ++a) {
    Bd.hi[a] = ext[a] - 1.0;
    Bd.len[a] = periodic[a] ? (double)ext[a] : 0.0;
  }
  Bd.top = !periodic[2];
  OdeOut o;
  ode_forward(*p, nu, d, x0, ub0, ul, wl, dul, Bd, o, nullptr, nullptr);
  for (int a = 0; a < 3; ++a) {
    x[a] = o.x[a];
    ub[a] = o.ub[a];
    psi[a] = o.psi[a];
  }
  return LBM_OK;
}

lbm_status lbm_host_bubble_ode_adjoint(const bubble_params* p, double nu, double d,
                                       const double* x0, const double* ub0, const double* ul,
                                       const double* wl, const double* dul, const int32_t* ext,
                                       const int32_t* periodic, const double* lx,
                                       const double* lub, const double* lpsi, double* out) {
  if (!p || !x0 || !ub0 || !ul || !wl || !dul || !ext || !periodic || !lx || !lub || !lpsi || !out)
    return LBM_EINVAL;
  if (p->n_sub < 1 || p->n_sub > kMaxSub) return LBM_EINVAL;
  OdeBounds Bd;
  for (int a = 0; a < 3; ++a) {
    Bd.hi[a] = ext[a] - 1.0;
    Bd.len[a] = periodic[a] ? (double)ext[a] : 0.0;
  }
  Bd.top = !periodic[2];
  OdeAdj g;
  ode_adjoint(*p, nu, d, x0, ub0, ul, wl, dul, Bd, lx, lub, lpsi, g);
  for (int a = 0; a < 3; ++a) {
    out[a] = g.x[a];
    out[3 + a] = g.ub[a];
    out[6 + a] = g.ul[a];
    out[9 + a] = g.wl[a];
    out[12 + a] = g.dul[a];
  }
  out[15] = g.dsD;
  out[16] = g.dsL;
  out[17] = g.dnu;
  return LBM_OK;
}

}  // extern "C"
