// Bubble half of one step of Algorithm 1 as three kernels:
//   k_interp  (one workgroup per bubble) cell-integral weights of the clipped fourth-order
//             polynomial kernel (eq. (18)-(19)) and the forward coupling (eq. (20)) of the
//             liquid velocity and of its curl, reduced across the workgroup in double precision;
//             with several bubbles it also enters the bubble in the per-tile lists;
//   k_ode     (one lane per bubble) the force closures of Table 1 and n_sub explicit sub-steps
//             of eq. (4), in double precision; with several bubbles it flags the tiles the
//             liquid step must force, or must write the velocity in;
//   k_spread  (one bubble: one workgroup) the backward coupling (eq. (21)) of the reaction into
//             the force field with the same weights (atomic adds) and the tile flags, or
//   k_spread_gather (several bubbles: one wavefront per tile) the same sums per cell in bubble
//             order from the lists, so that the force field is bit-reproducible.
// Up to 256 bubbles on one lattice and 512 over many columns (not in the exact-time variant)
// k_interp's workgroup also runs k_ode's update of its bubble on one lane and flags the bubble's
// tiles, and k_ode is not launched.
// The coupling variants of bubble_params.coupling (reaction, point-sampled weights, exact-time
// forward coupling) are modes of these kernels. k_mark marks the region of an overlapped step.
//
// The curl is the central-difference curl of the velocity with wall ghosts (bounce-back ghost =
// -U of the mirror cell, free-slip ghost = mirror cell with the normal component negated). Its
// kernel-weighted sum is evaluated by summation by parts: since the weights are separable,
//   sum_j w(j) (U(j+1) - U(j-1)) / 2 = sum_j U(j) dw(j),  dw(j) = (w(j-1) - w(j+1)) / 2,
// plus the folded ghost terms at a wall, so every cell of the window widened by one is read once
// and no neighbour values are needed. A component is never differentiated along its own axis,
// so the ghost sign along an axis is -1 at a bounce-back face and +1 at a free-slip face.
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "batch_cell.hpp"
#include "collide.hpp"

namespace lbm {
namespace {

constexpr int kMax = LBM_MAX_STENCIL;  // window cells per axis
constexpr int kSpan = kMax + 2;        // window widened by one cell on each side
constexpr int kWork = LBM_BUBBLE_WORK; // doubles of per-bubble workspace
constexpr int kBlock = 256;            // threads per bubble in the stencil kernels
constexpr int kBlockWaves = kBlock / 64;

struct BubbleArgs {
  bubble_params P;
  bubble_soa S;
  int nb;
  int32_t* status;
  double* rec;  // armed step record (nb x R_SIZE), filled by the bubble update, or null
  // trajectory recording: the update writes each bubble's position after the step into row
  // *traj_row of traj (3 x nb doubles per row, [a * nb + b]) while the row is below traj_rows; the
  // kernel that ends the bubble half then advances the row
  double* traj;
  int traj_rows;
  uint32_t* traj_row;
};

// The bubble half's last kernel advances the trajectory row (every update of the step has run).
__device__ __forceinline__ void advance_traj_row(const BubbleArgs& A) {
  if (A.traj && blockIdx.x == 0 && threadIdx.x == 0) *A.traj_row += 1u;
}

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// antiderivative of the kernel in s = r / n, P(-1) = 0, P(1) = 1
__device__ __forceinline__ double kernel_P(double s) {
  if (s <= -1.0) return 0.0;
  if (s >= 1.0) return 1.0;
  const double s2 = s * s;
  return 0.5 + 15.0 / 16.0 * (s - 2.0 / 3.0 * s2 * s + 0.2 * s2 * s2 * s);
}

// the kernel itself, eq. (18): Z(r) = 15/16 (s^4 - 2 s^2 + 1) / n with s = r / n on |s| <= 1
__device__ __forceinline__ double kernel_Z(double r, double n) {
  const double s = r / n;
  if (s < -1.0 || s > 1.0) return 0.0;
  const double s2 = s * s;
  return 15.0 / 16.0 * (s2 * s2 - 2.0 * s2 + 1.0) / n;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// The window of one bubble along one axis: cells [lo, hi] overlap the kernel support
// [x - n, x + n]; [clo, chi] is the part inside the domain (all of it on a periodic axis, in
// unwrapped coordinates); [dlo, dhi] widens that by one cell, clipped to the domain unless
// periodic.
struct Axis {
  int lo, hi, clo, chi, dlo, dhi;
};

__device__ __forceinline__ bool axis_window(double x, double n, int ext, bool per, Axis& w) {
  const double lo = floor(x - n - 0.5) + 1.0;
  const double hi = ceil(x + n + 0.5) - 1.0;
  if (!(hi - lo + 1.0 <= (double)kMax) || !(lo > -1e9) || !(hi < 1e9)) return false;
  w.lo = (int)lo;
  w.hi = (int)hi;
  w.clo = per ? w.lo : max(w.lo, 0);
  w.chi = per ? w.hi : min(w.hi, ext - 1);
  if (w.clo > w.chi) return false;
  w.dlo = per ? w.clo - 1 : max(w.clo - 1, 0);
  w.dhi = per ? w.chi + 1 : min(w.chi + 1, ext - 1);
  return true;
}

// Weights of one axis (eq. (19)): cell integrals of the kernel over the clipped window [clo, chi],
// indexed by (cell - lo + 1), renormalised to a sum of one when a wall clips the window. One full
// wavefront (lane = 0..63) computes; the renormalising sum is taken in a fixed order. point: the
// point-sampled variant, Z at the cell centres renormalised on every axis. Returns false if a
// point-sampled window holds no cell centre inside the kernel's support.
__device__ bool wave_axis_weights(const Axis& A, double xa, double n, bool per, bool point, int lane,
                                  double* s_w_a) {
  double part = 0.0;
  for (int i = lane; i < kSpan; i += 64) {
    const int v = A.lo - 1 + i;
    double w = 0.0;
    if (v >= A.clo && v <= A.chi)
      w = point ? kernel_Z(v - xa, n) : kernel_P((v + 0.5 - xa) / n) - kernel_P((v - 0.5 - xa) / n);
    s_w_a[i] = w;
    part += w;
  }
  if (!per || point) {
    const double sum = wave_sum(part);
    if (sum > 0.0)
      for (int i = lane; i < kSpan; i += 64) s_w_a[i] /= sum;
    return sum > 0.0 || !point;
  }
  return true;
}

// The weights of axis AX into s_w[AX] (one wavefront), and their derivative weights into
// s_dw[AX] once every wavefront's weights are in LDS. AX is a constant, so the window and the
// face conditions of the axis are plain registers.
template <int AX>
__device__ __forceinline__ bool axis_weights_wave(const Geom& G, const double xb[3], double n,
                                                  bool point, int lane, const Axis win[3],
                                                  double (*s_w)[kSpan]) {
  return wave_axis_weights(win[AX], xb[AX], n, G.bc[2 * AX] == BC_PER, point, lane, s_w[AX]);
}

template <int AX>
__device__ __forceinline__ void axis_dweights_wave(const Geom& G, int lane, const Axis win[3],
                                                   const double (*s_w)[kSpan],
                                                   double (*s_dw)[kSpan]) {
  const int e = AX == 0 ? G.nx : (AX == 1 ? G.ny : G.nz);
  const bool per = G.bc[2 * AX] == BC_PER;
  const double s_lo = G.bc[2 * AX] == BC_FS ? 1.0 : -1.0;
  const double s_hi = G.bc[2 * AX + 1] == BC_FS ? 1.0 : -1.0;
  const Axis& A = win[AX];
  for (int i = lane; i < kSpan; i += 64) {
    const int v = A.lo - 1 + i;
    const double wm = i > 0 ? s_w[AX][i - 1] : 0.0;
    const double wp = i + 1 < kSpan ? s_w[AX][i + 1] : 0.0;
    double dw = 0.5 * (wm - wp);
    if (!per) {
      if (v == 0) dw -= 0.5 * s_lo * s_w[AX][i];       // ghost below cell 0
      if (v == e - 1) dw += 0.5 * s_hi * s_w[AX][i];  // ghost above the last cell
    }
    s_dw[AX][i] = dw;
  }
}

// Weights w and derivative weights dw of the bubble at xb along the three axes, into LDS,
// indexed by (cell - lo + 1). Called by the whole workgroup; wavefront a computes axis a, the
// three side by side. point: the point-sampled variant of the weights.
__device__ bool build_weights(const Geom& G, const double xb[3], double n, int tid,
                              double (*s_w)[kSpan], double (*s_dw)[kSpan], Axis win[3],
                              bool point) {
  static_assert(kBlock >= 192, "one wavefront per axis");
  __shared__ int s_bad[3];
  const int ext[3] = {G.nx, G.ny, G.nz};
  for (int a = 0; a < 3; ++a) {
    const bool per = G.bc[2 * a] == BC_PER;
    if (!axis_window(xb[a], n, ext[a], per, win[a])) return false;
  }
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: a scalar branch
  const int lane = tid & 63;
  if (wave < 3) {
    bool ok;
    if (wave == 0)
      ok = axis_weights_wave<0>(G, xb, n, point, lane, win, s_w);
    else if (wave == 1)
      ok = axis_weights_wave<1>(G, xb, n, point, lane, win, s_w);
    else
      ok = axis_weights_wave<2>(G, xb, n, point, lane, win, s_w);
    if (lane == 0) s_bad[wave] = ok ? 0 : 1;
  }
  __syncthreads();
  if (wave == 0)
    axis_dweights_wave<0>(G, lane, win, s_w, s_dw);
  else if (wave == 1)
    axis_dweights_wave<1>(G, lane, win, s_w, s_dw);
  else if (wave == 2)
    axis_dweights_wave<2>(G, lane, win, s_w, s_dw);
  __syncthreads();
  return (s_bad[0] | s_bad[1] | s_bad[2]) == 0;
}

// Bubble handled by a workgroup: consecutive workgroups on one XCD take consecutive bubbles, so
// a caller that orders its bubbles in space keeps each XCD's share of the force field in its L2.
__device__ __forceinline__ int bubble_of_block(int nb) { return (int)xcd_remap(blockIdx.x, nb); }

__device__ __forceinline__ double block_sum(double v, double* s_red, int tid) {
  v = wave_sum(v);
  __syncthreads();
  if ((tid & 63) == 0) s_red[tid >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < kBlockWaves; ++w) t += s_red[w];
  return t;
}

// block_sum of six values at once, behind one barrier: the same butterfly in each wavefront and
// the same order over the wavefronts, so each sum has the bits block_sum gives it.
__device__ __forceinline__ void block_sum6(double v[6], double (*s_red6)[kBlockWaves], int tid) {
#pragma unroll
  for (int m = 0; m < 6; ++m) v[m] = wave_sum(v[m]);
  if ((tid & 63) == 0)
#pragma unroll
    for (int m = 0; m < 6; ++m) s_red6[m][tid >> 6] = v[m];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    double t = 0.0;
    for (int w = 0; w < kBlockWaves; ++w) t += s_red6[m][w];
    v[m] = t;
  }
}

// ---------------------------------------------------------------------------------------------
// Tiles of stencil windows.
// ---------------------------------------------------------------------------------------------
// Tile ranges touched along one axis by the cell range [vlo, vhi] (unwrapped on a periodic axis):
// up to two ranges of tiles.
struct TileRanges {
  int n;
  int lo[2], hi[2];
};

__device__ TileRanges tile_ranges(int vlo, int vhi, int ext, int tile, bool periodic) {
  TileRanges t;
  if (!periodic) {
    vlo = vlo < 0 ? 0 : vlo;
    vhi = vhi > ext - 1 ? ext - 1 : vhi;
    t.n = vlo <= vhi ? 1 : 0;
    t.lo[0] = vlo / tile;
    t.hi[0] = vhi / tile;
    return t;
  }
  if (vhi - vlo + 1 >= ext) {
    t.n = 1;
    t.lo[0] = 0;
    t.hi[0] = (ext - 1) / tile;
    return t;
  }
  const int a = wrapi(vlo, ext), b = wrapi(vhi, ext);
  if (a <= b) {
    t.n = 1;
    t.lo[0] = a / tile;
    t.hi[0] = b / tile;
  } else if (b / tile >= a / tile) {  // the two wrapped pieces share a tile: every tile once
    t.n = 1;
    t.lo[0] = 0;
    t.hi[0] = (ext - 1) / tile;
  } else {
    t.n = 2;
    t.lo[0] = a / tile;
    t.hi[0] = (ext - 1) / tile;
    t.lo[1] = 0;
    t.hi[1] = b / tile;
  }
  return t;
}

// Force window of a bubble at x0 (the clipped stencil window [clo, chi] of each axis).
__device__ bool force_windows(const Geom& G, const double x0[3], double n, Axis win[3]) {
  const int ext[3] = {G.nx, G.ny, G.nz};
  for (int a = 0; a < 3; ++a)
    if (!axis_window(x0[a], n, ext[a], G.bc[2 * a] == BC_PER, win[a])) return false;
  return true;
}

// Calls f(tile) for every tile of the ranges tr, over the threads of the workgroup.
template <class Fn>
__device__ void for_tiles(const Geom& G, const TileRanges tr[3], int tid, int nthreads, Fn&& f) {
  for (int rz = 0; rz < tr[2].n; ++rz)
    for (int ry = 0; ry < tr[1].n; ++ry)
      for (int rx = 0; rx < tr[0].n; ++rx) {
        const int nx_ = tr[0].hi[rx] - tr[0].lo[rx] + 1;
        const int ny_ = tr[1].hi[ry] - tr[1].lo[ry] + 1;
        const int nz_ = tr[2].hi[rz] - tr[2].lo[rz] + 1;
        for (int k = tid; k < nx_ * ny_ * nz_; k += nthreads) {
          const int tx = tr[0].lo[rx] + k % nx_;
          const int ty = tr[1].lo[ry] + (k / nx_) % ny_;
          const int tz = tr[2].lo[rz] + k / (nx_ * ny_);
          f(((uint32_t)tz * G.tny + ty) * G.tnx + tx);
        }
      }
}

// Number of tiles of the ranges tr, and the k-th of them in the order for_tiles visits them
// (k below the number).
__device__ __forceinline__ int tile_count(const TileRanges tr[3]) {
  int n[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    n[a] = tr[a].hi[0] - tr[a].lo[0] + 1;
    if (tr[a].n == 2) n[a] += tr[a].hi[1] - tr[a].lo[1] + 1;
  }
  return tr[0].n && tr[1].n && tr[2].n ? n[0] * n[1] * n[2] : 0;
}

__device__ __forceinline__ uint32_t nth_tile(const Geom& G, const TileRanges tr[3], int k) {
  uint32_t t = 0;
#pragma unroll
  for (int rz = 0; rz < 2; ++rz)
#pragma unroll
    for (int ry = 0; ry < 2; ++ry)
#pragma unroll
      for (int rx = 0; rx < 2; ++rx) {
        if (rz >= tr[2].n || ry >= tr[1].n || rx >= tr[0].n || k < 0) continue;
        const int nx_ = tr[0].hi[rx] - tr[0].lo[rx] + 1;
        const int ny_ = tr[1].hi[ry] - tr[1].lo[ry] + 1;
        const int nz_ = tr[2].hi[rz] - tr[2].lo[rz] + 1;
        if (k < nx_ * ny_ * nz_) {
          const int tx = tr[0].lo[rx] + k % nx_;
          const int ty = tr[1].lo[ry] + (k / nx_) % ny_;
          const int tz = tr[2].lo[rz] + k / (nx_ * ny_);
          t = ((uint32_t)tz * G.tny + ty) * G.tnx + tx;
        }
        k -= nx_ * ny_ * nz_;
      }
  return t;
}

// Tiles of the force window.
__device__ void force_tiles(const Geom& G, const Axis win[3], TileRanges tr[3]) {
  const int ext[3] = {G.nx, G.ny, G.nz};
  for (int a = 0; a < 3; ++a)
    tr[a] = tile_ranges(win[a].clo, win[a].chi, ext[a], (int)kTile, G.bc[2 * a] == BC_PER);
}

// Flags the tiles the liquid step must force (the force window now) or write the velocity in (the
// velocity window, with the curl ring, that the next interpolation reads at the new position).
template <typename T>
__device__ void mark_tiles(const ColumnView<T>& col, const BubbleArgs& A, const Axis win[3],
                           const double xn[3], double n, int tid, int nthreads) {
  const Geom& G = col.G;
  uint8_t* __restrict__ tiles = col.tiles;
  const int ext[3] = {G.nx, G.ny, G.nz};
  TileRanges tr[3];
  // In an overlapped step k_mark marked the tile rows (y, z) of the window at x0 widened by the
  // curl ring and kRegionMargin cells. Cell ranges inside those on y and z lie in marked rows, so
  // their flags need no reading; otherwise each tile's row flag is read.
  bool inside = true;
  for (int a = 0; a < 3; ++a) {
    const bool per = G.bc[2 * a] == BC_PER;
    int lo = win[a].clo, hi = win[a].chi;
    Axis nw;
    if (axis_window(xn[a], n, ext[a], per, nw)) {
      lo = min(lo, nw.dlo);
      hi = max(hi, nw.dhi);
    }
    if (a > 0)
      inside = inside && lo >= win[a].lo - 1 - kRegionMargin && hi <= win[a].hi + 1 + kRegionMargin;
    tr[a] = tile_ranges(lo, hi, ext[a], (int)kTile, per);
  }
  const uint32_t* __restrict__ region = inside ? nullptr : col.region;
  for_tiles(G, tr, tid, nthreads, [&](uint32_t t) {
    tiles[t] = 1;
    // in an overlapped step the bulk launch has updated the rows outside the region
    // concurrently: a tile forced or needing the velocity there is an error
    if (region && !region[t / (uint32_t)G.tnx]) atomicOr(A.status, (int32_t)STATUS_REGION_MISS);
  });
}

// Velocity of the current state at a cell, eq. (10) without a force term: the populations are
// pulled from the post-collision buffer with the face conditions, as the moments kernel does.
template <typename T>
__device__ __forceinline__ void state_velocity(const T* __restrict__ src, const Geom& G, int x, int y,
                                               int z, uint32_t cell, double& ux, double& uy,
                                               double& uz) {
  const CellNbr nb = cell_neighbours(G, x, y, z);
  T g[19];
  pull_all<true>(g, src, G, layout_cell(G, cell, (uint32_t)z), nb,
                 std::make_integer_sequence<int, 19>{});
  double drho = 0, m[3] = {0, 0, 0};
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    drho += (double)g[q];
    if (CX[q]) m[0] += CX[q] * (double)g[q];
    if (CY[q]) m[1] += CY[q] * (double)g[q];
    if (CZ[q]) m[2] += CZ[q] * (double)g[q];
  }
  const double r = 1.0 + drho;
  ux = m[0] / r;
  uy = m[1] / r;
  uz = m[2] / r;
}

// ---------------------------------------------------------------------------------------------
// Forward coupling: u_l = sum W U and w_l = sum W curl U over the window.
// ---------------------------------------------------------------------------------------------
// EXACT: the exact-time coupling variant (single lattice), reading the current state's velocity.
// GATHER: cells of a thread's window column whose loads are in flight together. Few bubbles (all
// their workgroups on the chip at once): 8, so each thread waits for one round trip per 8 cells.
// Many bubbles: 4, at fewer VGPRs, so that more workgroups stay resident beside the bulk launch
// (20 000 bubbles with the earlier cell-by-cell loop: 394 us against 1289 us with 8 beside the
// bulk launch; with the column sums, alone on the chip, 154 us with 4 against 177 us with 1).
// FUSE (few bubbles on one lattice): the workgroup then also runs its bubble's update (k_ode's
// arithmetic, one lane) and flags its tiles, so the step has one launch less. The fourth wavefront,
// idle while the other three compute the weights, prepares the update's closure constants and
// loads, and the update takes the sums from registers instead of reading them back.
// Per-bubble constants of the Table 1 closures (they depend on the diameter only).
struct BubbleConst {
  double V, r2pi, fb, inv_meff, va;  // volume, pi r^2, buoyancy, 1/m_eff, (1 + C_A) rho_l V
  double visc24, visc48, re_sat;     // 24 nu/d, 48 nu/d, Re beyond which 48/Re wins
  double shape;                      // 8/3 Eo/(Eo + 4)
  double f_lift;                     // f(Eo_d)
  double Eod;
};

__device__ BubbleConst bubble_constants(const bubble_params& P, double nu, double d) {
  const double pi = 3.14159265358979323846;
  BubbleConst k;
  k.V = pi * d * d * d / 6.0;
  const double r = 0.5 * d;
  k.r2pi = pi * r * r;
  k.fb = (P.rho_l - P.rho_b) * k.V * P.g;
  k.inv_meff = 1.0 / (P.rho_b * k.V + P.c_a * P.rho_l * k.V);
  k.va = (1.0 + P.c_a) * P.rho_l * k.V;
  k.visc24 = 24.0 * nu / d;
  k.visc48 = 48.0 * nu / d;
  // 1 + k Re^0.687 >= 2 for Re >= (1/k)^(1/0.687): there the min{} of C_D is 48/Re
  k.re_sat = P.cd_k > 0.0 ? exp(log(1.0 / P.cd_k) / 0.687) : INFINITY;
  const double Eo = (P.rho_l - P.rho_b) * P.g * d * d / P.sigma;
  k.shape = 8.0 / 3.0 * Eo / (Eo + 4.0);
  const double E = 1.0 / (1.0 + 0.163 * exp(0.757 * log(Eo)));
  k.Eod = Eo / exp(2.0 / 3.0 * log(E));
  k.f_lift = 0.00105 * k.Eod * k.Eod * k.Eod - 0.0159 * k.Eod * k.Eod - 0.0204 * k.Eod + P.lift_f0;
  return k;
}

// The inputs of one bubble's update: its state before the step and the coupling sums of eq. (20).
struct OdeIn {
  int st;
  double valid, d;
  double ul[3], wl[3], ulp[3], ub[3], xn[3];
};

// What the fused update takes from the start of its workgroup: the closure constants and the
// bubble's velocity and liquid velocity of the last step.
struct FusePre {
  BubbleConst kc;
  double ub[3], ulp[3];
};

template <typename Geo>
__device__ bool ode_lane(const Geo& geo, const BubbleArgs& A, int b, double x0[3], double xn_out[3],
                         double& n_out);
template <typename Geo>
__device__ bool ode_update(const Geo& geo, const BubbleArgs& A, int b, const OdeIn& in,
                           const BubbleConst* kc_in, const double* x0_in, double x0[3],
                           double xn_out[3], double& n_out);

// What the first workgroup of a step's first bubble kernel clears for the step.
template <typename Geo>
__device__ __forceinline__ void clear_for_step(const Geo& geo) {
  if constexpr (std::is_same_v<Geo, OneColumn>) {
    // in an overlapped step, the other parity's region list (its region launch ran before)
    // starts empty
    if (geo.clear_count) *geo.clear_count = 0u;
  }
  geo.clear_other_jobs();  // many columns: the next step's tile jobs start empty
}

// Forward coupling of bubble b by the whole workgroup (and, FUSE, its update and tile flags).
template <typename T, typename Geo, bool EXACT, int GATHER, bool FUSE>
__device__ void interp_bubble(const Geo& geo, const BubbleArgs& A, const int b) {
  __shared__ double s_w[3][kSpan];
  __shared__ double s_dw[3][kSpan];
  __shared__ double s_red6[6][kBlockWaves];
  const int tid = threadIdx.x;
  const ColumnView<T> col = geo.template view<T>(b);
  const Geom& G = col.G;
  const T* __restrict__ U = col.U;
  double* work = A.S.work + (size_t)b * kWork;
  // the bubble update of a bubble without a valid window: nothing but its cleared reaction
  auto ode_skip = [&] {
    if constexpr (FUSE) {
      double x0[3], xn[3], m;
      ode_lane(geo, A, b, x0, xn, m);
    }
  };
  const int st = A.S.state[b];
  if (st == 0) {
    if (tid == 0) {
      work[W_VALID] = 0.0;
      ode_skip();
    }
    return;
  }
  const double xb[3] = {A.S.x[b], A.S.y[b], A.S.z[b]};
  const double d = A.S.d[b];
  const double n = A.P.kernel_factor * d;
  Axis win[3];
  const bool finite = isfinite(xb[0]) && isfinite(xb[1]) && isfinite(xb[2]) && d > 0.0;
  const bool point = A.P.coupling & LBM_COUPLING_POINT_KERNEL;
  __shared__ FusePre s_pre;
  if constexpr (FUSE) {
    // wavefront 3 has no axis to weigh: it prepares the update's constants and loads meanwhile
    static_assert(kBlock >= 256, "a fourth wavefront");
    if (tid == 192) {
      s_pre.kc = bubble_constants(geo.params(A.P, b), col.nu, d);
      s_pre.ub[0] = A.S.ux[b];
      s_pre.ub[1] = A.S.uy[b];
      s_pre.ub[2] = A.S.uz[b];
      s_pre.ulp[0] = A.S.ulx[b];
      s_pre.ulp[1] = A.S.uly[b];
      s_pre.ulp[2] = A.S.ulz[b];
    }
  }
  if (!finite || !build_weights(G, xb, n, tid, s_w, s_dw, win, point)) {
    if (tid == 0) {
      work[W_VALID] = 0.0;
      atomicOr(A.status, (int32_t)STATUS_STENCIL_TOO_LARGE);
      ode_skip();
    }
    return;
  }
  // the weights at x0 for the spreading of this step
  for (int i = tid; i < 3 * kSpan; i += kBlock) work[W_WGT + i] = s_w[i / kSpan][i % kSpan];
  // enter the bubble in the list of every tile of its force window: the slot of each thread's
  // first tile is taken now and written after the gather, so the atomic is in flight meanwhile
  uint32_t t0 = 0, slot0 = kTileCap;
  uint32_t* const tcount = geo.tcount_of(b);
  uint32_t* const tlist = geo.tlist_of(b);
  if (geo.use_lists()) {
    TileRanges tr[3];
    force_tiles(G, win, tr);
    const int nt = tile_count(tr);
    if (tid < nt) {
      t0 = nth_tile(G, tr, tid);
      slot0 = atomicAdd(&tcount[t0], 1u);
      if (slot0 == 0u) geo.note_tile(b, t0);
    }
    for (int k = tid + kBlock; k < nt; k += kBlock) {
      const uint32_t t = nth_tile(G, tr, k);
      const uint32_t slot = atomicAdd(&tcount[t], 1u);
      if (slot == 0u) geo.note_tile(b, t);
      if (slot < kTileCap) tlist[(size_t)t * kTileCap + slot] = (uint32_t)b;
    }
  }
  const int Dx = win[0].dhi - win[0].dlo + 1;
  const int Dy = win[1].dhi - win[1].dlo + 1;
  const int Dz = win[2].dhi - win[2].dlo + 1;
  const int total = Dx * Dy * Dz;
  const bool px = G.bc[0] == BC_PER, py = G.bc[2] == BC_PER, pz = G.bc[4] == BC_PER;
  const T* __restrict__ S = nullptr;  // exact-time coupling: the current state
  if constexpr (EXACT) S = static_cast<const T*>(geo.state);
  double acc[6] = {0, 0, 0, 0, 0, 0};
  if constexpr (EXACT) {
    // The thread's window entries f = tid, tid + kBlock, ... as f = i + Dx (j + Dy k), stepped by
    // kBlock entries with carries (one division per thread); each cell's velocity (from the
    // state) times its weight and curl weights into the six sums.
    int ci = tid % Dx, cj = (tid / Dx) % Dy, ck = tid / Dx / Dy;
    const int di = kBlock % Dx, dj = (kBlock / Dx) % Dy, dk = kBlock / Dx / Dy;
    for (int f = tid; f < total; f += kBlock) {
      const int vx = win[0].dlo + ci, vy = win[1].dlo + cj, vz = win[2].dlo + ck;
      const int ix = vx - win[0].lo + 1, iy = vy - win[1].lo + 1, iz = vz - win[2].lo + 1;
      const int x = px ? wrapi(vx, G.nx) : vx;
      const int y = py ? wrapi(vy, G.ny) : vy;
      const int z = pz ? wrapi(vz, G.nz) : vz;
      const uint32_t c = ((uint32_t)z * G.ny + y) * G.nx + x;
      double ux, uy, uz;
      state_velocity<T>(S, G, x, y, z, c, ux, uy, uz);
      const double wa = s_w[0][ix], da = s_dw[0][ix];
      const double wb = s_w[1][iy], db = s_dw[1][iy];
      const double wc = s_w[2][iz], dc = s_dw[2][iz];
      const double W = wa * wb * wc;
      const double a_dbc = wa * db * wc;  // weight of d/dy
      const double a_bdc = wa * wb * dc;  // weight of d/dz
      const double da_bc = da * wb * wc;  // weight of d/dx
      acc[0] += W * ux;
      acc[1] += W * uy;
      acc[2] += W * uz;
      acc[3] += uz * a_dbc - uy * a_bdc;  // dUz/dy - dUy/dz
      acc[4] += ux * a_bdc - uz * da_bc;  // dUx/dz - dUz/dx
      acc[5] += uy * da_bc - ux * a_dbc;  // dUy/dx - dUx/dy
      ci += di;
      const int carry = ci >= Dx;
      if (carry) ci -= Dx;
      cj += dj + carry;
      if (cj >= Dy) {
        cj -= Dy;
        ++ck;
      }
      ck += dk;
    }
  } else {
    // Separable sums by window column: a thread takes the column (i, j) of the window over a
    // slab of z (one slab unless the window has fewer columns than the workgroup has threads)
    // and sums along z the velocity times the z weight and times the z derivative weight; the
    // column's x and y weights then enter once:
    //   sum_k wa wb wc_k u = wa wb Sw,  curl terms from wa db Sw, wa wb Sd and da wb Sw,
    // with Sw = sum_k wc_k u_k and Sd = sum_k dc_k u_k. Consecutive lanes take consecutive x, and
    // the three components are read at one 32-bit offset from their planes' bases. The loads of
    // GATHER z cells are issued together, the sums then taken in z order.
    constexpr int kZ = GATHER;
    const int cols = Dx * Dy;
    const int slabs = min(max(1, kBlock / cols), Dz);
    const uint32_t plane = (uint32_t)G.nx * (uint32_t)G.ny;
    const uint32_t wrap_back = (uint32_t)G.nz * plane;
    const T* __restrict__ Ux = U;
    const T* __restrict__ Uy = U + G.N;
    const T* __restrict__ Uz = U + 2 * (size_t)G.N;
    const int iz_base = win[2].dlo - win[2].lo + 1;
    for (int t = tid; t < cols * slabs; t += kBlock) {
      const int colm = t % cols, slab = t / cols;
      const int ci = colm % Dx, cj = colm / Dx;
      const int k0 = slab * Dz / slabs, k1 = (slab + 1) * Dz / slabs;
      const int vx = win[0].dlo + ci, vy = win[1].dlo + cj, vz = win[2].dlo + k0;
      const int x = px ? wrapi(vx, G.nx) : vx;
      const int y = py ? wrapi(vy, G.ny) : vy;
      int z = pz ? wrapi(vz, G.nz) : vz;
      uint32_t c = ((uint32_t)z * G.ny + y) * G.nx + x;
      double sw[3] = {0.0, 0.0, 0.0}, sd[3] = {0.0, 0.0, 0.0};
      for (int k = k0; k < k1; k += kZ) {
        T u[kZ][3];
#pragma clang loop unroll(full)
        for (int s = 0; s < kZ; ++s) {
          if (k + s < k1) {
            u[s][0] = Ux[c];
            u[s][1] = Uy[c];
            u[s][2] = Uz[c];
            c += plane;
            if (++z == G.nz) {  // periodic z only: a clipped window ends inside the domain
              z = 0;
              c -= wrap_back;
            }
          }
        }
#pragma clang loop unroll(full)
        for (int s = 0; s < kZ; ++s) {
          if (k + s < k1) {
            const double wc = s_w[2][iz_base + k + s], dc = s_dw[2][iz_base + k + s];
            for (int m = 0; m < 3; ++m) {
              sw[m] += wc * (double)u[s][m];
              sd[m] += dc * (double)u[s][m];
            }
          }
        }
      }
      const int ix = vx - win[0].lo + 1, iy = vy - win[1].lo + 1;
      const double wa = s_w[0][ix], da = s_dw[0][ix];
      const double wb = s_w[1][iy], db = s_dw[1][iy];
      const double w_ab = wa * wb, w_adb = wa * db, w_dab = da * wb;
      acc[0] += w_ab * sw[0];
      acc[1] += w_ab * sw[1];
      acc[2] += w_ab * sw[2];
      acc[3] += w_adb * sw[2] - w_ab * sd[1];  // dUz/dy - dUy/dz
      acc[4] += w_ab * sd[0] - w_dab * sw[2];  // dUx/dz - dUz/dx
      acc[5] += w_dab * sw[1] - w_adb * sw[0];  // dUy/dx - dUx/dy
    }
  }
  if (slot0 < kTileCap) tlist[(size_t)t0 * kTileCap + slot0] = (uint32_t)b;
  block_sum6(acc, s_red6, tid);
  if (tid == 0) {
    for (int m = 0; m < 6; ++m) work[W_UL + m] = acc[m];
    work[W_X0 + 0] = xb[0];
    work[W_X0 + 1] = xb[1];
    work[W_X0 + 2] = xb[2];
    work[W_VALID] = 1.0;
  }
  if constexpr (FUSE) {
    // the update's inputs are at hand: the sums (in every thread), the position, a valid window
    // and what wavefront 3 prepared; the force window at x0 is win
    __shared__ double s_xn[3];
    __shared__ int s_flag;
    if (tid == 0) {
      OdeIn in;
      in.st = st;
      in.valid = 1.0;
      in.d = d;
      for (int a = 0; a < 3; ++a) {
        in.ul[a] = acc[a];
        in.wl[a] = acc[3 + a];
        in.ulp[a] = s_pre.ulp[a];
        in.ub[a] = s_pre.ub[a];
        in.xn[a] = xb[a];
      }
      double x0[3], xn[3], m = 0.0;
      s_flag = ode_update(geo, A, b, in, &s_pre.kc, xb, x0, xn, m) ? 1 : 0;
      for (int a = 0; a < 3; ++a) s_xn[a] = xn[a];
    }
    __syncthreads();
    if (s_flag) {
      const double xn[3] = {s_xn[0], s_xn[1], s_xn[2]};
      mark_tiles<T>(col, A, win, xn, n, tid, kBlock);
    }
  }
}

template <typename T, typename Geo, bool EXACT = false, int GATHER = 1, bool FUSE = false>
__global__ __launch_bounds__(kBlock) void k_interp(Geo geo, BubbleArgs A) {
  if (blockIdx.x == 0 && threadIdx.x == 0) clear_for_step(geo);
  interp_bubble<T, Geo, EXACT, GATHER, FUSE>(geo, A, bubble_of_block(A.nb));
}

// ---------------------------------------------------------------------------------------------
// Bubble dynamics, one lane per bubble.
// ---------------------------------------------------------------------------------------------

// Drag and lift of Table 1 on a bubble moving at ub in liquid of velocity ul and vorticity wl,
// with Re = |u_r| d / nu (eq. (3)). C_D is used multiplied by |u_r| so that the viscous
// branches stay finite at u_r = 0: 24/Re |u_r| = 24 nu / d.
__device__ __forceinline__ void drag_lift(const bubble_params& P, const BubbleConst& k, double d,
                                          double nu, const double ub[3], const double ul[3],
                                          const double wl[3], double FD[3], double FL[3]) {
  const double ur[3] = {ub[0] - ul[0], ub[1] - ul[1], ub[2] - ul[2]};
  const double mag = sqrt(ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2]);
  const double Re = mag * d / nu;
  double visc = k.visc48;
  if (Re < k.re_sat && Re > 0.0)
    visc = fmin(k.visc24 * (1.0 + P.cd_k * exp(0.687 * log(Re))), k.visc48);
  else if (Re == 0.0)
    visc = fmin(k.visc24, k.visc48);
  const double cdu = fmax(visc, k.shape * mag);
  double cl;
  if (k.Eod < 4.0)
    cl = fmin(0.288 * tanh(0.121 * Re), k.f_lift);
  else if (k.Eod <= 10.0)
    cl = k.f_lift;
  else
    cl = -0.29;
  const double dpre = -0.5 * P.drag_scale * cdu * P.rho_l * k.r2pi;
  for (int a = 0; a < 3; ++a) FD[a] = dpre * ur[a];
  const double cr[3] = {ur[1] * wl[2] - ur[2] * wl[1], ur[2] * wl[0] - ur[0] * wl[2],
                        ur[0] * wl[1] - ur[1] * wl[0]};
  const double lpre = -P.lift_scale * cl * P.rho_l * k.V;
  for (int a = 0; a < 3; ++a) FL[a] = lpre * cr[a];
}

// The bubble update of one lane's bubble. Returns true when the bubble's tiles are left to flag
// (several bubbles on one lattice), with its start position x0, new position xn and half-width n.
template <typename Geo>
__device__ bool ode_lane(const Geo& geo, const BubbleArgs& A, int b, double x0[3], double xn_out[3],
                         double& n_out) {
  const double* work = A.S.work + (size_t)b * kWork;
  // every load of the update at once (one round trip; all in bounds for b < nb)
  OdeIn in;
  in.st = A.S.state[b];
  in.valid = work[W_VALID];
  in.d = A.S.d[b];
  for (int a = 0; a < 3; ++a) {
    in.ul[a] = work[W_UL + a];
    in.wl[a] = work[W_WL + a];
  }
  in.ulp[0] = A.S.ulx[b];
  in.ulp[1] = A.S.uly[b];
  in.ulp[2] = A.S.ulz[b];
  in.ub[0] = A.S.ux[b];
  in.ub[1] = A.S.uy[b];
  in.ub[2] = A.S.uz[b];
  in.xn[0] = A.S.x[b];
  in.xn[1] = A.S.y[b];
  in.xn[2] = A.S.z[b];
  // the values as operands of an empty statement: the compiler keeps the loads above the branch
  // of the update instead of moving them into the branch's live path (a second round trip)
  asm volatile("" ::"v"(in.d), "v"(in.ul[0]), "v"(in.ul[1]), "v"(in.ul[2]), "v"(in.wl[0]),
               "v"(in.wl[1]), "v"(in.wl[2]), "v"(in.ulp[0]), "v"(in.ulp[1]), "v"(in.ulp[2]),
               "v"(in.ub[0]), "v"(in.ub[1]), "v"(in.ub[2]), "v"(in.xn[0]), "v"(in.xn[1]),
               "v"(in.xn[2]));
  return ode_update(geo, A, b, in, nullptr, nullptr, x0, xn_out, n_out);
}

// The update itself from its inputs; kc_in and x0_in, when given, are the closure constants and
// the window position already at hand (otherwise computed, and read from the bubble's work area).
template <typename Geo>
__device__ bool ode_update(const Geo& geo, const BubbleArgs& A, int b, const OdeIn& in,
                           const BubbleConst* kc_in, const double* x0_in, double x0[3],
                           double xn_out[3], double& n_out) {
  const ColumnView<float> col = geo.template view<float>(b);
  const Geom& G = col.G;
  const double nu = col.nu;
  const bubble_params P = geo.params(A.P, b);
  double* work = A.S.work + (size_t)b * kWork;
  const int st = in.st;
  const double valid = in.valid;
  const double d = in.d;
  const double ul[3] = {in.ul[0], in.ul[1], in.ul[2]};
  const double wl[3] = {in.wl[0], in.wl[1], in.wl[2]};
  const double ulp[3] = {in.ulp[0], in.ulp[1], in.ulp[2]};
  double ub[3] = {in.ub[0], in.ub[1], in.ub[2]};
  double xn[3] = {in.xn[0], in.xn[1], in.xn[2]};
  // the armed step record: the state before the update (what k_record's two stages copy)
  double* rec = A.rec ? A.rec + (size_t)b * R_SIZE : nullptr;
  if (rec) {
    for (int a = 0; a < 3; ++a) {
      rec[R_X + a] = xn[a];
      rec[R_UB + a] = ub[a];
      rec[R_ULP + a] = ulp[a];
      rec[R_UL + a] = ul[a];
      rec[R_WL + a] = wl[a];
    }
    rec[R_STATE] = (double)st;
    rec[R_D] = d;
    rec[R_VALID] = valid;
    rec[R_SUB] = 0.0;
  }
  auto record_position = [&](const double* xp) {
    if (A.traj) {
      const uint32_t row = *A.traj_row;
      if (row < (uint32_t)A.traj_rows)
        for (int a = 0; a < 3; ++a) A.traj[(size_t)row * 3 * A.nb + (size_t)a * A.nb + b] = xp[a];
    }
  };
  if (st == 0 || valid == 0.0) {
    record_position(xn);  // unchanged
    if (rec)
      for (int a = 0; a < 3; ++a) rec[R_PSI + a] = work[W_PSI + a];
    if (A.S.psix) {
      A.S.psix[b] = 0.0;
      A.S.psiy[b] = 0.0;
      A.S.psiz[b] = 0.0;
    }
    return false;
  }
  const int ext[3] = {G.nx, G.ny, G.nz};
  double dul[3] = {0.0, 0.0, 0.0};
  if (st == 2) {  // material derivative of u_l along the path, dt_l = 1
    dul[0] = ul[0] - ulp[0];
    dul[1] = ul[1] - ulp[1];
    dul[2] = ul[2] - ulp[2];
  }
  BubbleConst kc;
  if (kc_in)
    kc = *kc_in;
  else
    kc = bubble_constants(P, nu, d);
  const double dt = 1.0 / P.n_sub;
  const int reaction = P.coupling & LBM_REACTION_MASK;
  const double m_b = P.rho_b * kc.V;
  // sums over the sub-steps of F_D + F_L and of the net force m_b du_b/dt (reaction variants)
  double s_dl[3] = {0.0, 0.0, 0.0}, s_net[3] = {0.0, 0.0, 0.0};
  // the record keeps the velocity at the start of each sub-step and the clamp flags
  double* rec_ubs = rec && P.n_sub <= kRecordMaxSub ? rec + R_UBS : nullptr;
  uint32_t clamp0 = 0u, clamp1 = 0u, clamp2 = 0u;  // bits 0-31, 32-63, 64-95
  for (int k = 0; k < P.n_sub; ++k) {
    if (rec_ubs)
      for (int a = 0; a < 3; ++a) rec_ubs[3 * k + a] = ub[a];
    // (m_b + C_A rho_l V) du_b/dt = F_B + F_D + F_L + (1 + C_A) rho_l V D_t u_l
    double FD[3], FL[3];
    drag_lift(P, kc, d, nu, ub, ul, wl, FD, FL);
    for (int a = 0; a < 3; ++a) {
      double f = FD[a] + FL[a] + kc.va * dul[a];
      if (a == 2) f += kc.fb;
      s_dl[a] += FD[a] + FL[a];
      s_net[a] += m_b * (f * kc.inv_meff);
      ub[a] += dt * f * kc.inv_meff;
    }
    for (int a = 0; a < 3; ++a) {
      xn[a] += dt * ub[a];
      if (G.bc[2 * a] == BC_PER) {
        const double L = (double)ext[a];
        xn[a] = fmod(xn[a], L);
        if (xn[a] < 0.0) xn[a] += L;
      } else {
        bool clamped = false;
        if (xn[a] < 0.0) {
          xn[a] = 0.0;
          ub[a] = 0.0;
          clamped = true;
        }
        if (a != 2 && xn[a] > ext[a] - 1.0) {
          xn[a] = ext[a] - 1.0;
          ub[a] = 0.0;
          clamped = true;
        }
        if (clamped) {
          const int bit = 3 * k + a;
          const uint32_t m = 1u << (bit & 31);
          if (bit < 32)
            clamp0 |= m;
          else if (bit < 64)
            clamp1 |= m;
          else
            clamp2 |= m;
        }
      }
    }
  }
  if (rec_ubs) {
    for (int a = 0; a < 3; ++a) rec_ubs[3 * P.n_sub + a] = ub[a];
    rec[R_CLAMP] = (double)clamp0;
    rec[R_CLAMP + 1] = (double)clamp1;
    rec[R_CLAMP + 2] = (double)clamp2;
    rec[R_SUB] = 1.0;
  }
  // the reaction spread into the liquid (Algorithm 1, or a coupling variant)
  double psi[3];
  if (reaction == LBM_REACTION_SUBSTEP_MEAN) {
    for (int a = 0; a < 3; ++a) psi[a] = -s_dl[a] / P.n_sub;
  } else if (reaction == LBM_REACTION_NET_FORCE) {
    for (int a = 0; a < 3; ++a) psi[a] = -s_net[a] / P.n_sub;
  } else {
    double FD[3], FL[3];
    drag_lift(P, kc, d, nu, ub, ul, wl, FD, FL);
    for (int a = 0; a < 3; ++a) psi[a] = -(FD[a] + FL[a]);
  }
  A.S.x[b] = xn[0];
  A.S.y[b] = xn[1];
  A.S.z[b] = xn[2];
  record_position(xn);
  A.S.ux[b] = ub[0];
  A.S.uy[b] = ub[1];
  A.S.uz[b] = ub[2];
  A.S.ulx[b] = ul[0];
  A.S.uly[b] = ul[1];
  A.S.ulz[b] = ul[2];
  int nst = 2;
  if (G.bc[4] != BC_PER && xn[2] >= ext[2] - 1.0) nst = 0;  // reached the top layer
  A.S.state[b] = nst;
  for (int a = 0; a < 3; ++a) work[W_PSI + a] = psi[a];
  if (rec)
    for (int a = 0; a < 3; ++a) rec[R_PSI + a] = psi[a];
  if (A.S.psix) {
    A.S.psix[b] = psi[0];
    A.S.psiy[b] = psi[1];
    A.S.psiz[b] = psi[2];
  }
  if (geo.use_lists()) {  // the spreading gathers per tile: the tiles are flagged by the wavefront
    for (int a = 0; a < 3; ++a) {
      x0[a] = x0_in ? x0_in[a] : work[W_X0 + a];
      xn_out[a] = xn[a];
    }
    n_out = P.kernel_factor * d;
    return true;
  }
  return false;
}

// Bubble dynamics, one lane per bubble (Table 1, eq. (1)-(4)). With several bubbles on one
// lattice the tiles of each bubble (its force window at x0 and velocity window at the new
// position) are then flagged: each lane its own bubble's when the wavefront holds many bubbles
// (the lanes' loops run side by side), the whole wavefront one bubble after the other when it
// holds a few (the tiles of one bubble then spread over the lanes).
constexpr int kWaveFlagMaxBubbles = 16;

template <typename Geo>
__global__ __launch_bounds__(64) void k_ode(Geo geo, BubbleArgs A) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  double x0[3] = {0.0, 0.0, 0.0}, xn[3] = {0.0, 0.0, 0.0}, n = 0.0;
  const bool flag = b < A.nb && ode_lane(geo, A, b, x0, xn, n);
  if (!geo.use_lists()) return;
  const int lane = threadIdx.x;
  uint64_t todo = __ballot(flag);
  if (__popcll(todo) > kWaveFlagMaxBubbles) {
    Axis win[3];
    if (flag) {
      const ColumnView<float> col = geo.template view<float>(b);
      if (force_windows(col.G, x0, n, win)) mark_tiles<float>(col, A, win, xn, n, 0, 1);
    }
    return;
  }
  while (todo) {
    const int l = __ffsll((unsigned long long)todo) - 1;
    todo &= todo - 1;
    double y0[3], yn[3];
    for (int a = 0; a < 3; ++a) {
      y0[a] = __shfl(x0[a], l, 64);
      yn[a] = __shfl(xn[a], l, 64);
    }
    const double m = __shfl(n, l, 64);
    const ColumnView<float> col = geo.template view<float>((int)(blockIdx.x * 64) + l);
    Axis win[3];
    if (force_windows(col.G, y0, m, win)) mark_tiles<float>(col, A, win, yn, m, lane, 64);
  }
}

// ---------------------------------------------------------------------------------------------
// Backward coupling and tile flags.
// ---------------------------------------------------------------------------------------------
// Backward coupling by atomic adds: F(j) += psi W_j over the force window (eq. (21)).
template <typename T>
__device__ void spread_atomic(const Geom& G, T* __restrict__ F, const Axis win[3],
                              double (*s_w)[kSpan], const double* work, int tid) {
  const double psi0 = work[W_PSI], psi1 = work[W_PSI + 1], psi2 = work[W_PSI + 2];
  const int Kx = win[0].chi - win[0].clo + 1;
  const int Ky = win[1].chi - win[1].clo + 1;
  const int Kz = win[2].chi - win[2].clo + 1;
  const int total = Kx * Ky * Kz;
  const bool px = G.bc[0] == BC_PER, py = G.bc[2] == BC_PER, pz = G.bc[4] == BC_PER;
  for (int f = tid; f < total; f += kBlock) {
    const int i = f % Kx, r = f / Kx;
    const int j = r % Ky, k = r / Ky;
    const int vx = win[0].clo + i, vy = win[1].clo + j, vz = win[2].clo + k;
    const double W = s_w[0][vx - win[0].lo + 1] * s_w[1][vy - win[1].lo + 1] *
                     s_w[2][vz - win[2].lo + 1];
    const int x = px ? wrapi(vx, G.nx) : vx;
    const int y = py ? wrapi(vy, G.ny) : vy;
    const int z = pz ? wrapi(vz, G.nz) : vz;
    const uint32_t c = ((uint32_t)z * G.ny + y) * G.nx + x;
    atomicAdd(&F[c], (T)(psi0 * W));
    atomicAdd(&F[G.N + c], (T)(psi1 * W));
    atomicAdd(&F[2 * (size_t)G.N + c], (T)(psi2 * W));
  }
}

// Backward coupling of one bubble per workgroup by atomic adds, and the tile flags.
template <typename T, typename Geo>
__global__ __launch_bounds__(kBlock) void k_spread(Geo geo, BubbleArgs A) {
  __shared__ double s_w[3][kSpan];
  __shared__ double s_dw[3][kSpan];
  advance_traj_row(A);
  const int b = bubble_of_block(A.nb);
  const int tid = threadIdx.x;
  const ColumnView<T> col = geo.template view<T>(b);
  const double* work = A.S.work + (size_t)b * kWork;
  if (work[W_VALID] == 0.0) return;
  const double x0[3] = {work[W_X0], work[W_X0 + 1], work[W_X0 + 2]};
  const double n = A.P.kernel_factor * A.S.d[b];
  Axis win[3];
  // validated by k_interp
  if (!build_weights(col.G, x0, n, tid, s_w, s_dw, win, A.P.coupling & LBM_COUPLING_POINT_KERNEL))
    return;
  spread_atomic<T>(col.G, col.F, win, s_w, work, tid);
  const double xn[3] = {A.S.x[b], A.S.y[b], A.S.z[b]};
  mark_tiles<T>(col, A, win, xn, n, tid, kBlock);
}

// ---- deterministic backward coupling (gather per tile), for several bubbles on one lattice ----
//
// k_interp enters each bubble in the list of every tile of its force window at x0 (kTileCap
// entries per tile; the count keeps rising past a full list), the bubble update (k_ode, or
// k_interp itself with few bubbles) flags the bubble's tiles for the liquid step, and
// k_spread_gather, one wavefront per tile, sums psi_b W_b(j) over the tile's
// bubbles in bubble order in double precision with the weights k_interp stored at x0. A tile
// whose list overflowed finds its bubbles by a scan of all bubbles in index order instead, so the
// sum has the same terms in the same order either way. F(j) does not depend on the order in
// which wavefronts ran; with one bubble per cell the sum is the atomic path's single addition,
// bit for bit.
// Sum of the weights of axis a (global copy, indexed cell - lo + 1) at the window cells congruent
// to cell v (one cell unless a periodic window is wider than the lattice).
__device__ __forceinline__ double axis_weight_at(const Axis& A, const double* w_a, int v, int ext,
                                                 bool per) {
  if (!per) return (v >= A.clo && v <= A.chi) ? w_a[v - A.lo + 1] : 0.0;
  int u = A.clo + wrapi(v - A.clo, ext);  // first window cell congruent to v
  if (u > A.chi) return 0.0;
  double s = w_a[u - A.lo + 1];
  for (u += ext; u <= A.chi; u += ext) s += w_a[u - A.lo + 1];
  return s;
}

__device__ __forceinline__ bool in_tile_ranges(const TileRanges& r, int t) {
  return (r.n > 0 && t >= r.lo[0] && t <= r.hi[0]) || (r.n > 1 && t >= r.lo[1] && t <= r.hi[1]);
}

// One tile's share of the gather: the tile t of a lattice G with force field F, its list (tcount,
// tlist) and the bubbles [b0, b1) that may cover it (the overflow scan's range).
template <typename T>
struct GatherJob {
  Geom G;
  T* F;
  uint32_t* tcount;
  const uint32_t* tlist;
  uint32_t t;
  int b0, b1;
};

// Jobs of the gather. One lattice: every tile, one per workgroup (an empty list returns at once).
// Many columns: the (column, tile) pairs noted this step, over the workgroups in turn.
__device__ __forceinline__ uint32_t gather_jobs(const OneColumn& geo) {
  return (uint32_t)geo.G.tnx * geo.G.tny * (((uint32_t)geo.G.nz + kTile - 1) / kTile);
}
__device__ __forceinline__ uint32_t gather_jobs(const ManyColumns& geo) {
  return min(geo.job_count[geo.par], geo.job_cap);
}
template <typename T>
__device__ __forceinline__ GatherJob<T> gather_job(const OneColumn& geo, const BubbleArgs& A,
                                                   uint32_t j) {
  return {geo.G, static_cast<T*>(geo.F), geo.tcount, geo.tlist, j, 0, A.nb};
}
template <typename T>
__device__ __forceinline__ GatherJob<T> gather_job(const ManyColumns& geo, const BubbleArgs&,
                                                   uint32_t j) {
  const uint32_t* e = geo.jobs + 2 * ((size_t)geo.par * geo.job_cap + j);
  const ColumnDev& C = geo.cols[e[0]];
  return {C.G, static_cast<T*>(C.F), C.tcount, C.tlist, e[1], C.bubble_begin,
          C.bubble_begin + C.nb};
}

// Bubbles staged at once in the gather: 8 bubbles x kTile cells, one per lane of a wavefront.
constexpr uint32_t kGatherChunk = 64 / kTile;

// Value of v in lane l (l the same in every lane).
__device__ __forceinline__ double lane_value(double v, int l) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// One staged bubble as one lane of the wavefront holds it: the bubble's weights at the i-th cell
// of the tile along each axis, and its reaction component i mod 3.
struct GatherLane {
  double wx, wy, wz, psi;
};

__device__ __forceinline__ GatherLane gather_lane(const Geom& G, const BubbleArgs& A, uint32_t b,
                                                  bool valid, int i, const int org[3],
                                                  const bool per[3]) {
  GatherLane s = {0.0, 0.0, 0.0, 0.0};
  if (!valid) return s;
  const double* work = A.S.work + (size_t)b * kWork;
  const double x0[3] = {work[W_X0], work[W_X0 + 1], work[W_X0 + 2]};
  s.psi = work[W_PSI + i % 3];
  Axis win[3];
  force_windows(G, x0, A.P.kernel_factor * A.S.d[b], win);  // valid: the bubble was listed
  s.wx = axis_weight_at(win[0], work + W_WGT, org[0] + i, G.nx, per[0]);
  s.wy = axis_weight_at(win[1], work + W_WGT + kSpan, org[1] + i, G.ny, per[1]);
  s.wz = axis_weight_at(win[2], work + W_WGT + 2 * kSpan, org[2] + i, G.nz, per[2]);
  return s;
}

// The jobs first, first + stride, ... of the step's gather, one per wavefront (first and stride
// count wavefronts). Lane (lx, ly) = (lane mod kTile, lane / kTile) holds the tile's column of
// kTile cells along z and their 24 sums in registers. The tile's bubbles, in index order (the
// list sorted by rank, or the overflow scan compacted by ballot), are staged kGatherChunk at a
// time: lane (k, i) loads the chunk's k-th bubble and forms its weights at the tile's i-th cell of
// each axis; every lane then adds the chunk's terms in order, reading its cells' weights from the
// lanes that hold them. The terms and their order per cell are those of the eq. (21) sum in
// bubble order; only lanes whose cells exist store.
template <typename T, typename Geo>
__device__ void gather_tiles(const Geo& geo, const BubbleArgs& A, uint32_t first, uint32_t stride) {
  static_assert(kTileCap == 64 && kTile == 8, "a wavefront holds a tile's list and its 8 x 8 columns");
  const int lane = (int)(threadIdx.x & 63u);
  const int lx = lane % (int)kTile, ly = lane / (int)kTile;
  const uint64_t below = (1ull << lane) - 1ull;
  const uint32_t njobs = gather_jobs(geo);
  for (uint32_t j = first; j < njobs; j += stride) {
    const GatherJob<T> J = gather_job<T>(geo, A, j);
    const Geom& G = J.G;
    const uint32_t t = J.t;
    const uint32_t cnt = J.tcount[t];
    if (cnt == 0u) continue;  // uniform over the wavefront
    const uint32_t tx = t % (uint32_t)G.tnx, rr = t / (uint32_t)G.tnx;
    const uint32_t ty = rr % (uint32_t)G.tny, tz = rr / (uint32_t)G.tny;
    const int org[3] = {(int)(tx * kTile), (int)(ty * kTile), (int)(tz * kTile)};
    const bool per[3] = {G.bc[0] == BC_PER, G.bc[2] == BC_PER, G.bc[4] == BC_PER};
    double acc[kTile][3];
#pragma unroll
    for (int i = 0; i < (int)kTile; ++i) acc[i][0] = acc[i][1] = acc[i][2] = 0.0;
    // adds the terms of the n bubbles lanes 0..n-1 of ids name, in that order
    auto add = [&](uint32_t ids, uint32_t n) {
      for (uint32_t k0 = 0; k0 < n; k0 += kGatherChunk) {
        const uint32_t m = min(n - k0, kGatherChunk);
        const int ck = ly, ci = lx;  // this lane stages cell ci of the chunk's bubble ck
        const uint32_t b = (uint32_t)__shfl((int)ids, (int)k0 + ck, 64);
        const GatherLane st = gather_lane(G, A, b, (uint32_t)ck < m, ci, org, per);
        for (uint32_t k = 0; k < m; ++k) {
          const int l0 = (int)(k * kTile);
          const double wx = __shfl(st.wx, l0 + lx, 64);
          const double wy = __shfl(st.wy, l0 + ly, 64);
          const double psi[3] = {lane_value(st.psi, l0), lane_value(st.psi, l0 + 1),
                                 lane_value(st.psi, l0 + 2)};
#pragma unroll
          for (int i = 0; i < (int)kTile; ++i) {
            const double wz = lane_value(st.wz, l0 + i);
            const double W = wx * wy * wz;
            for (int q = 0; q < 3; ++q) acc[i][q] += psi[q] * W;
          }
        }
      }
    };
    if (cnt <= kTileCap) {
      const uint32_t n = cnt;
      const uint32_t v = (uint32_t)lane < n ? J.tlist[(size_t)t * kTileCap + lane] : 0xffffffffu;
      // rank of the lane's entry (ties, which the lists do not hold, would keep list order); the
      // lanes past the list keep their own index, so the ranks are a permutation of the lanes
      uint32_t r = 0;
      for (uint32_t i = 0; i < n; ++i) {
        const uint32_t vi = (uint32_t)__builtin_amdgcn_readlane((int)v, (int)i);
        r += (vi < v || (vi == v && i < (uint32_t)lane)) ? 1u : 0u;
      }
      if ((uint32_t)lane >= n) r = (uint32_t)lane;
      add((uint32_t)__builtin_amdgcn_ds_permute((int)(r * 4u), (int)v), n);
    } else {
      // the list overflowed: every bubble whose force window holds this tile, by a scan of the
      // lattice's bubbles in index order, 64 per pass compacted by ballot
      for (int base = J.b0; base < J.b1; base += 64) {
        const int b = base + lane;
        bool cov = false;
        if (b < J.b1) {
          const double* work = A.S.work + (size_t)b * kWork;
          if (work[W_VALID] != 0.0) {
            const double x0[3] = {work[W_X0], work[W_X0 + 1], work[W_X0 + 2]};
            Axis win[3];
            if (force_windows(G, x0, A.P.kernel_factor * A.S.d[b], win)) {
              TileRanges tr[3];
              force_tiles(G, win, tr);
              cov = in_tile_ranges(tr[0], (int)tx) && in_tile_ranges(tr[1], (int)ty) &&
                    in_tile_ranges(tr[2], (int)tz);
            }
          }
        }
        const uint64_t mask = __ballot(cov);
        const uint32_t nc = (uint32_t)__popcll(mask);
        const uint32_t pos = cov ? (uint32_t)__popcll(mask & below)
                                 : nc + (uint32_t)__popcll(~mask & below);
        add((uint32_t)__builtin_amdgcn_ds_permute((int)(pos * 4u), b), nc);
      }
    }
    const int x = org[0] + lx, y = org[1] + ly;
    if (x < G.nx && y < G.ny) {
      for (int i = 0; i < (int)kTile; ++i) {
        const int z = org[2] + i;
        if (z >= G.nz) break;
        const uint32_t c = ((uint32_t)z * G.ny + y) * G.nx + x;
        J.F[c] = (T)acc[i][0];
        J.F[G.N + c] = (T)acc[i][1];
        J.F[2 * (size_t)G.N + c] = (T)acc[i][2];
      }
    }
    // every lane has read the count
    if (lane == 0) J.tcount[t] = 0u;
  }
}

template <typename T, typename Geo>
__global__ __launch_bounds__(kBlock) void k_spread_gather(Geo geo, BubbleArgs A) {
  advance_traj_row(A);
  gather_tiles<T, Geo>(geo, A, blockIdx.x * kBlockWaves + threadIdx.x / 64, gridDim.x * kBlockWaves);
}

// Region of an overlapped step (one wavefront per bubble): the tile rows (y, z) of the bubble's
// stencil window at its current position widened by the curl ring and by kRegionMargin cells.
// They hold every tile k_spread flags in this step (the force window at this position, the
// velocity window at the position after the bubble update). A row enters the list once (its flag
// is set by an atomic exchange; the lane that finds it clear appends it).
template <typename Geo>
__global__ __launch_bounds__(64) void k_mark(Geo geo, BubbleArgs A, uint32_t* __restrict__ region,
                                             uint32_t* __restrict__ list, uint32_t* __restrict__ count,
                                             uint32_t nrows) {
  const int b = bubble_of_block(A.nb);
  if (A.S.state[b] == 0) return;
  const Geom G = geo.template view<float>(b).G;
  const double xb[3] = {A.S.x[b], A.S.y[b], A.S.z[b]};
  const double n = A.P.kernel_factor * A.S.d[b];
  const int ext[3] = {G.nx, G.ny, G.nz};
  TileRanges tr[3];
  for (int a = 1; a < 3; ++a) {
    const bool per = G.bc[2 * a] == BC_PER;
    Axis w;
    if (!axis_window(xb[a], n, ext[a], per, w)) return;  // reported by k_interp
    tr[a] = tile_ranges(w.lo - 1 - kRegionMargin, w.hi + 1 + kRegionMargin, ext[a], (int)kTile, per);
  }
  for (int rz = 0; rz < tr[2].n; ++rz)
    for (int ry = 0; ry < tr[1].n; ++ry) {
      const int ny_ = tr[1].hi[ry] - tr[1].lo[ry] + 1;
      const int nz_ = tr[2].hi[rz] - tr[2].lo[rz] + 1;
      for (int k = threadIdx.x; k < ny_ * nz_; k += 64) {
        const int ty = tr[1].lo[ry] + k % ny_;
        const int tz = tr[2].lo[rz] + k / ny_;
        const uint32_t u = (uint32_t)tz * G.tny + ty;
        if (atomicExch(&region[u], 1u) == 0u) {
          const uint32_t i = atomicAdd(count, 1u);
          if (i < nrows) list[i] = u;  // a row is listed once per step: i < nrows
        }
      }
    }
}

// Workgroups of the many-column gather (their wavefronts take the noted tiles in turn).
constexpr uint32_t kGatherMaxBlocks = 2048;

// Bubble counts up to which k_interp keeps 8 cells' loads in flight per thread: one workgroup per
// bubble, all resident at once (at 76 VGPRs six per compute unit).
constexpr int kInterpLatencyMaxBubbles = 1024;
// Bubble counts up to which k_interp also runs the bubble update (k_ode's ~200 VGPRs then limit
// it to two workgroups per compute unit): on one lattice, whose bubble kernels share the chip with
// the bulk launch, 256; for many columns, whose bubble kernels have the chip, every workgroup
// resident at once (two per compute unit).
constexpr int kFuseMaxBubbles = 256;
constexpr int kFuseMaxBubblesBatch = 512;

template <typename Geo>
constexpr int fuse_max_bubbles() {
  return std::is_same_v<Geo, OneColumn> ? kFuseMaxBubbles : kFuseMaxBubblesBatch;
}

template <typename T, typename Geo>
hipError_t launch_bubble_kernels(const Geo& geo, const BubbleArgs& A, hipStream_t stream) {
  const int nb = A.nb;
  bool exact = false;
  if constexpr (std::is_same_v<Geo, OneColumn>) exact = geo.state != nullptr;
  if (exact) {
    if constexpr (std::is_same_v<Geo, OneColumn>)
      hipLaunchKernelGGL((k_interp<T, Geo, true>), dim3(nb), dim3(kBlock), 0, stream, geo, A);
  } else if (nb <= fuse_max_bubbles<Geo>()) {
    hipLaunchKernelGGL((k_interp<T, Geo, false, 8, true>), dim3(nb), dim3(kBlock), 0, stream, geo, A);
  } else if (nb <= kInterpLatencyMaxBubbles) {
    hipLaunchKernelGGL((k_interp<T, Geo, false, 8>), dim3(nb), dim3(kBlock), 0, stream, geo, A);
  } else {
    hipLaunchKernelGGL((k_interp<T, Geo, false, 4>), dim3(nb), dim3(kBlock), 0, stream, geo, A);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const bool fused = !exact && nb <= fuse_max_bubbles<Geo>();
  if (!fused) {
    hipLaunchKernelGGL((k_ode<Geo>), dim3(div_up(nb, 64)), dim3(64), 0, stream, geo, A);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if constexpr (std::is_same_v<Geo, OneColumn>) {
    if (geo.next_region) {
      // the region of the next step, from the bubble state this update leaves
      hipLaunchKernelGGL((k_mark<OneColumn>), dim3(nb), dim3(64), 0, stream, geo, A,
                         geo.next_region, geo.next_list, geo.next_count, geo.nrows);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (geo.lists) {  // several bubbles: the lists k_interp filled, summed per tile
      const uint32_t ntiles = (uint32_t)geo.G.tnx * geo.G.tny * div_up(geo.G.nz, kTile);
      hipLaunchKernelGGL((k_spread_gather<T, OneColumn>), dim3(div_up(ntiles, kBlockWaves)),
                         dim3(kBlock), 0, stream,
                         geo, A);
      return hipGetLastError();
    }
    hipLaunchKernelGGL((k_spread<T, Geo>), dim3(nb), dim3(kBlock), 0, stream, geo, A);
    return hipGetLastError();
  } else {
    // many columns: the tiles noted this step, gathered by the workgroups in turn
    const uint32_t blocks =
        std::max(1u, std::min(div_up(geo.job_cap, (uint32_t)kBlockWaves), kGatherMaxBlocks));
    hipLaunchKernelGGL((k_spread_gather<T, ManyColumns>), dim3(blocks), dim3(kBlock), 0, stream,
                       geo, A);
    return hipGetLastError();
  }
}

// ---------------------------------------------------------------------------------------------
// Persistent batched launch: many method steps of every column in one kernel.
// ---------------------------------------------------------------------------------------------
// Barrier of every workgroup of a persistent launch (all resident: the grid is sized from the
// occupancy the kernel allows). The first thread of each workgroup makes the workgroup's writes
// visible at agent scope and counts itself in; the last arrival resets the count and advances the
// generation the others poll. The wait is bounded: after spin_limit polls a workgroup raises the
// abort word and the status, and every workgroup leaves the kernel at its next barrier, so a
// launch whose workgroups were not all resident ends (with an error) instead of hanging. Returns
// false once the launch is aborted.
__device__ bool grid_barrier(uint32_t* bar, uint32_t nblocks, uint32_t spin_limit,
                             int32_t* status) {
  __shared__ uint32_t s_go;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t go = 1u;
    const uint32_t gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();  // this workgroup's writes, before its arrival
    const uint32_t n =
        __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (n == nblocks) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&bar[1], gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint32_t polls = 0;
      // relaxed polls (an acquire per poll would invalidate the caches each time); the fence
      // below orders what follows
      while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
        if (++polls > spin_limit) {
          __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          atomicOr(status, (int32_t)STATUS_BARRIER_TIMEOUT);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __threadfence();  // the other workgroups' writes, after the barrier
    if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) go = 0u;
    s_go = go;
  }
  __syncthreads();
  return s_go != 0u;
}

// P.nsteps method steps of every column, each in three phases separated by grid barriers: the
// bubbles (forward coupling, update and tile flags, one bubble per workgroup in turn), the gather
// of the reactions per noted tile, and the liquid step per work item. The same device code as
// the per-step launches (k_interp with the fused update, k_spread_gather, k_batch_step), so the
// results are the same.
template <typename T, int FACES>
__global__ __launch_bounds__(kBlock, 2) void k_batch_persistent(ManyColumns geo, BubbleArgs A,
                                                             PersistArgs P) {
  for (int s = 0; s < P.nsteps; ++s) {
    const int odd = s & 1;
    ManyColumns g = geo;
    g.flag = P.flag0 ^ odd;
    g.par = P.cur0 ^ odd;
    if (A.nb > 0) {
      if (blockIdx.x == 0 && threadIdx.x == 0) clear_for_step(g);
      for (int b = blockIdx.x; b < A.nb; b += gridDim.x) {
        interp_bubble<T, ManyColumns, false, 8, true>(g, A, b);
        __syncthreads();  // the next bubble reuses the workgroup's shared arrays
      }
      if (!grid_barrier(P.barrier, gridDim.x, P.spin_limit, A.status)) return;
      gather_tiles<T, ManyColumns>(g, A, blockIdx.x * kBlockWaves + threadIdx.x / 64,
                                   gridDim.x * kBlockWaves);
      if (!grid_barrier(P.barrier, gridDim.x, P.spin_limit, A.status)) return;
    }
    for (uint32_t k = blockIdx.x; k < P.nitems; k += gridDim.x)
      batch_item<T, FACES>(P.cols, P.item_col, xcd_remap(k, P.nitems), P.cur0 ^ odd, g.flag,
                           P.flags);
    if (!grid_barrier(P.barrier, gridDim.x, P.spin_limit, A.status)) return;
  }
}

template <typename T, int FACES>
hipError_t launch_persistent_typed(const ManyColumns& geo, const BubbleArgs& A,
                                   const PersistArgs& P, int wgs_per_cu, uint32_t* grid,
                                   hipStream_t stream) {
  const auto kern = k_batch_persistent<T, FACES>;
  int per_cu = 0, dev = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, 0);
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (per_cu < 1 || cus < 1) return hipErrorInvalidConfiguration;
  if (wgs_per_cu > 0 && wgs_per_cu < per_cu) per_cu = wgs_per_cu;
  const uint32_t blocks = (uint32_t)per_cu * (uint32_t)cus;
  *grid = blocks;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, stream, geo, A, P);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_persistent_faces(const ManyColumns& geo, const BubbleArgs& A,
                                   const PersistArgs& P, int wgs_per_cu, uint32_t* grid,
                                   hipStream_t stream) {
  switch (P.faces) {
    case FACES_BB: return launch_persistent_typed<T, FACES_BB>(geo, A, P, wgs_per_cu, grid, stream);
    case FACES_WALLS:
      return launch_persistent_typed<T, FACES_WALLS>(geo, A, P, wgs_per_cu, grid, stream);
    default: return launch_persistent_typed<T, FACES_GENERAL>(geo, A, P, wgs_per_cu, grid, stream);
  }
}

}  // namespace

hipError_t launch_bubbles(lbm_ctx* c, const bubble_params* p, const bubble_soa* s, int32_t nb,
                          bool overlap, bool mark_ahead) {
  BubbleArgs A;
  A.P = *p;
  A.S = *s;
  A.nb = nb;
  A.status = c->status;
  A.rec = c->arm_record;  // one-shot
  c->arm_record = nullptr;
  A.traj = c->traj;
  A.traj_rows = c->traj_rows;
  A.traj_row = c->traj_row;
  // this step's mask: the one the last liquid step cleared (cleared here if no liquid step ran)
  const int m = c->hs.flag_cur ^ 1;
  if (!c->hs.flag_clean[m]) {
    const hipError_t e = launch_fill(c->tiles[m], c->ntiles, c->stream);
    if (e != hipSuccess) return e;
  }
  c->hs.flag_clean[m] = false;
  c->hs.flag_cur = m;
  if (nb == 0) return hipSuccess;
  OneColumn geo;
  geo.G = c->geom;
  geo.U = c->vel;
  geo.F = c->force;
  geo.tiles = c->tiles[m];
  geo.nu = (1.0 / c->desc.omega - 0.5) / 3.0;  // eq. (9), dx = dt_l = 1
  geo.region = nullptr;
  geo.tcount = c->tcount;
  geo.tlist = c->tlist;
  geo.lists = nb > 1;
  geo.state = (p->coupling & LBM_COUPLING_EXACT_TIME) ? c->pops[c->hs.cur] : nullptr;
  geo.clear_count = nullptr;
  geo.next_region = nullptr;
  geo.next_list = nullptr;
  geo.next_count = nullptr;
  geo.nrows = c->nrows;
  if (overlap) {
    // Region of this step (unless the previous step of this run marked it), then fork: the
    // bubble kernels run on the side stream while the bulk of the liquid step runs on the
    // caller's stream, which then waits for the bubble kernels (so that work the caller enqueues
    // next sees their results); lbm_step() updates the region. Marks left by an earlier call
    // only widen a region (the flags admit each row once), which stays correct.
    const int r = c->hs.rpar;
    hipError_t e = hipSuccess;
    if (!c->hs.marked) {
      hipLaunchKernelGGL((k_mark<OneColumn>), dim3(nb), dim3(64), 0, c->stream, geo, A,
                         c->region[r], c->region_list[r], c->region_count + r, c->nrows);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(c->ev_fork, c->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->side, c->ev_fork, 0);
    if (e != hipSuccess) return e;
    geo.region = c->region[r];
    geo.clear_count = c->region_count + (r ^ 1);
    if (mark_ahead) {
      geo.next_region = c->region[r ^ 1];
      geo.next_list = c->region_list[r ^ 1];
      geo.next_count = c->region_count + (r ^ 1);
    }
    c->hs.marked = mark_ahead;
    e = c->elem == 4 ? launch_bubble_kernels<float>(geo, A, c->side)
                     : launch_bubble_kernels<double>(geo, A, c->side);
    if (e == hipSuccess) e = hipEventRecord(c->ev_join, c->side);
    if (e == hipSuccess) e = launch_bulk(c);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->ev_join, 0);
    if (e != hipSuccess) return e;
    c->hs.pending = true;
    c->pending_nb = nb;
    return hipSuccess;
  }
  if (c->elem == 4) return launch_bubble_kernels<float>(geo, A, c->stream);
  return launch_bubble_kernels<double>(geo, A, c->stream);
}

hipError_t launch_bubbles_batch(const ManyColumns& geo, size_t elem, const bubble_params* p,
                                const bubble_soa* s, int32_t nb, int32_t* status,
                                hipStream_t stream) {
  if (nb == 0) return hipSuccess;
  BubbleArgs A;
  A.P = *p;
  A.S = *s;
  A.nb = nb;
  A.status = status;
  A.rec = nullptr;
  A.traj = nullptr;
  A.traj_rows = 0;
  A.traj_row = nullptr;
  if (elem == 4) return launch_bubble_kernels<float>(geo, A, stream);
  return launch_bubble_kernels<double>(geo, A, stream);
}

hipError_t launch_batch_persistent(const ManyColumns& geo, size_t elem, const bubble_params* p,
                                   const bubble_soa* s, int32_t nb, int32_t* status,
                                   const PersistArgs& P, int wgs_per_cu, uint32_t* grid,
                                   hipStream_t stream) {
  BubbleArgs A;
  A.P = *p;
  A.S = *s;
  A.nb = nb;
  A.status = status;
  A.rec = nullptr;
  A.traj = nullptr;
  A.traj_rows = 0;
  A.traj_row = nullptr;
  if (elem == 4) return launch_persistent_faces<float>(geo, A, P, wgs_per_cu, grid, stream);
  return launch_persistent_faces<double>(geo, A, P, wgs_per_cu, grid, stream);
}

}  // namespace lbm
