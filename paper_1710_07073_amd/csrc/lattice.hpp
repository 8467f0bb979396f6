// D3Q19 lattice, geometry and the per-cell pull (streaming with face conditions) shared by the
// device kernels of this library. Population order is the paper's (eq. (7)): six axis
// directions, twelve face diagonals, rest particle; populations are stored as g = f - w.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Velocity components (eq. (7)), paper order.
constexpr int CX[19] = {1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 0};
constexpr int CY[19] = {0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0};
constexpr int CZ[19] = {0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0};

__host__ __device__ constexpr int find_dir(int cx, int cy, int cz) {
  for (int q = 0; q < 19; ++q)
    if (CX[q] == cx && CY[q] == cy && CZ[q] == cz) return q;
  return -1;
}
__host__ __device__ constexpr int opposite(int q) { return find_dir(-CX[q], -CY[q], -CZ[q]); }
// population with the component along axis a negated (specular reflection on a wall normal to a)
__host__ __device__ constexpr int mirrored(int q, int a) {
  return find_dir(a == 0 ? -CX[q] : CX[q], a == 1 ? -CY[q] : CY[q], a == 2 ? -CZ[q] : CZ[q]);
}

// Weights (eq. (8)).
template <typename T>
__host__ __device__ constexpr T weight(int q) {
  return q < 6 ? T(1) / T(18) : (q < 18 ? T(1) / T(36) : T(1) / T(3));
}

enum : int { BC_BB = 0, BC_FS = 1, BC_PER = 2 };

// Lattice geometry passed by value to kernels.
//
// Population buffers are addressed by a layout index lc = x + nx * y + zs * z, with population q
// at element q * qs + lc. Two layouts:
//   plane-blocked (default): the 19 populations of each z-plane are 19 consecutive planes,
//     (nz, 19, ny, nx): qs = nx * ny, zs = 19 * nx * ny;
//   plain structure of arrays: (19, nz, ny, nx): qs = N, zs = nx * ny.
// Either way a run of cells along x is contiguous and every population of a cell sits at a
// fixed stride from the others. Force and velocity fields are always (3, nz, ny, nx).
struct Geom {
  int nx, ny, nz;
  uint32_t N;      // cells
  uint32_t plane;  // nx * ny
  uint32_t qs;     // element stride between populations of one cell
  uint32_t zs;     // element stride between z-planes of one population
  int bc[6];       // -x, +x, -y, +y, -z, +z
  int tnx, tny;    // tile grid (8^3 tiles) in x and y
};

inline void set_layout(Geom& G, bool plain_soa) {
  G.qs = plain_soa ? G.N : G.plane;
  G.zs = plain_soa ? G.plane : 19u * G.plane;
}

// Layout index of the cell with flat index cell = x + nx * (y + ny * z).
__device__ __forceinline__ uint32_t layout_cell(const Geom& G, uint32_t cell, uint32_t z) {
  return cell + (G.zs - G.plane) * z;
}

// Per-thread boundary information of one cell for the pull: for each axis, the offset in layout
// index of the source one cell below / above (wrapped on periodic axes) and whether that source
// lies beyond a non-periodic wall.
struct CellNbr {
  int32_t dm[3], dp[3];  // offset of the neighbour at -1 / +1 along each axis
  bool om[3], op[3];     // that neighbour is outside a wall
};

__device__ __forceinline__ CellNbr cell_neighbours(const Geom& G, int x, int y, int z) {
  CellNbr n;
  const int ext[3] = {G.nx, G.ny, G.nz};
  const int pos[3] = {x, y, z};
  const int32_t stride[3] = {1, G.nx, (int32_t)G.zs};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const bool per = G.bc[2 * a] == BC_PER;
    const bool lo = pos[a] == 0, hi = pos[a] == ext[a] - 1;
    n.dm[a] = (lo && per) ? (ext[a] - 1) * stride[a] : -stride[a];
    n.dp[a] = (hi && per) ? -(ext[a] - 1) * stride[a] : stride[a];
    n.om[a] = lo && !per;
    n.op[a] = hi && !per;
  }
  return n;
}

// Source of population Q arriving at the cell with layout index lc in the post-collision buffer:
// the streaming step eq. (16) written per destination, as the element index q_src * qs + lc_src.
// A source beyond a wall is replaced by
//   - half-way bounce-back: the opposite population of the same cell;
//   - free slip, when exactly one coordinate of the source is outside: the population with the
//     normal component mirrored, taken from the source position with the normal coordinate kept;
//   - anything else (edges and corners): bounce-back.
// Every (cell, q) of the buffer is the source of exactly one destination: the map is a
// permutation, so its transpose (the adjoint of streaming) is a conflict-free scatter.
// GENERAL = false compiles only the bounce-back/no-periodic case.
template <int Q, bool GENERAL>
__device__ __forceinline__ size_t pull_index(const Geom& G, uint32_t lc, const CellNbr& nb) {
  constexpr int cx = CX[Q], cy = CY[Q], cz = CZ[Q];
  int32_t off = 0;
  bool out[3] = {false, false, false};
  if (cx > 0) { off += nb.dm[0]; out[0] = nb.om[0]; }
  if (cx < 0) { off += nb.dp[0]; out[0] = nb.op[0]; }
  if (cy > 0) { off += nb.dm[1]; out[1] = nb.om[1]; }
  if (cy < 0) { off += nb.dp[1]; out[1] = nb.op[1]; }
  if (cz > 0) { off += nb.dm[2]; out[2] = nb.om[2]; }
  if (cz < 0) { off += nb.dp[2]; out[2] = nb.op[2]; }
  const bool any = out[0] || out[1] || out[2];
  if (!any) return (size_t)Q * G.qs + (uint32_t)((int32_t)lc + off);
  constexpr int qo = opposite(Q);
  if constexpr (GENERAL) {
    const int nout = (int)out[0] + (int)out[1] + (int)out[2];
    if (nout == 1) {
      // which face: the source lies below (c > 0) or above (c < 0) along the out axis
      const int a = out[0] ? 0 : (out[1] ? 1 : 2);
      const int c = a == 0 ? cx : (a == 1 ? cy : cz);
      if (G.bc[2 * a + (c > 0 ? 0 : 1)] == BC_FS) {
        // keep the normal coordinate: remove that axis' contribution from the offset
        const int32_t da = a == 0 ? (cx > 0 ? nb.dm[0] : nb.dp[0])
                                  : (a == 1 ? (cy > 0 ? nb.dm[1] : nb.dp[1])
                                            : (cz > 0 ? nb.dm[2] : nb.dp[2]));
        const int qm = a == 0 ? mirrored(Q, 0) : (a == 1 ? mirrored(Q, 1) : mirrored(Q, 2));
        return (size_t)qm * G.qs + (uint32_t)((int32_t)lc + off - da);
      }
    }
  }
  return (size_t)qo * G.qs + lc;
}

// Gather (pull) of population Q arriving at the cell with layout index lc from the post-collision
// buffer `src`.
template <int Q, bool GENERAL, typename T>
__device__ __forceinline__ T pull(const T* __restrict__ src, const Geom& G, uint32_t lc,
                                  const CellNbr& nb) {
  return src[pull_index<Q, GENERAL>(G, lc, nb)];
}

}  // namespace lbm
