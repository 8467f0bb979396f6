// The batched liquid step's work item (the single-lattice fused step of Sec. 2.2 and Sec. 3.3 on
// one contiguous range of a column's cells), shared by the per-step batched launch and the
// persistent batched launch.
#pragma once

#include <utility>

#include "step_cell.hpp"

namespace lbm {

// q = a / d for a < 2^24 with rd the float nearest to 1 / d: the float quotient is off by at most
// one, which one correction in each direction removes.
__device__ __forceinline__ uint32_t div_small(uint32_t a, uint32_t d, float rd) {
  uint32_t q = (uint32_t)((float)a * rd);
  if (q * d > a) --q;
  if ((q + 1) * d <= a) ++q;
  return q;
}

// The general pull (any face rule) from a global pointer.
template <typename T, int... Qs>
__device__ __forceinline__ void pull_all_g(T* g, const gmem<T>* src, const Geom& G, uint32_t lc,
                                           const CellNbr& nb, std::integer_sequence<int, Qs...>) {
  ((g[Qs] = src[pull_index<Qs, true>(G, lc, nb)]), ...);
}

// Faces of a batch (the liquid kernel's template parameter): every face of every column
// bounce-back, walls only (bounce-back or free slip), or some face periodic.
enum : int { FACES_BB = 0, FACES_WALLS = 1, FACES_GENERAL = 2 };

// The liquid step of one work item of a batch (item_col names its column) by the workgroup, one
// cell per thread per pass. The coordinates of the item's first cell are found once (uniform);
// each thread carries its own offset into x, y and z with two small divisions. With walls only,
// the cell is the single-lattice fast path (step_cell_bb: scalar bases, 32-bit byte offsets).
template <typename T, int FACES>
__device__ __forceinline__ void batch_item(const ColumnDev* __restrict__ cols,
                                           const uint32_t* __restrict__ item_col, uint32_t item,
                                           int cur, int flag, int flags) {
  const ColumnDev& C = cols[item_col[item]];
  const Geom G = C.G;
  // the column's buffers, as pointers into global memory (the table is not a kernel argument,
  // so the compiler would otherwise address them as flat memory)
  const gmem<T>* src = reinterpret_cast<const gmem<T>*>(gbytes<T>(C.pops[cur]));
  gmem<T>* dst = reinterpret_cast<gmem<T>*>(gbytes<T>(C.pops[cur ^ 1]));
  gmem<T>* F = reinterpret_cast<gmem<T>*>(gbytes<T>(C.F));
  gmem<T>* U = reinterpret_cast<gmem<T>*>(gbytes<T>(C.U));
  const gmem<uint8_t>* tiles = reinterpret_cast<const gmem<uint8_t>*>(gbytes<uint8_t>(C.tiles[flag]));
  gmem<uint8_t>* tiles_next = reinterpret_cast<gmem<uint8_t>*>(gbytes<uint8_t>(C.tiles[flag ^ 1]));
  const T omega = (T)C.omega;
  const uint32_t first = (item - C.item_begin) * C.item_cells;
  const uint32_t last = min(first + C.item_cells, G.N);
  const uint32_t z0 = first / G.plane, r0 = first - z0 * G.plane;
  const uint32_t y0 = r0 / (uint32_t)G.nx, x0 = r0 - y0 * (uint32_t)G.nx;
  const float rnx = C.rnx, rny = C.rny;
  const uint32_t fs = FACES == FACES_WALLS ? free_slip_faces(G) : 0u;
  const bool static_force = flags & LBM_FLAG_STATIC_FORCE;
  for (uint32_t k = threadIdx.x; first + k < last; k += 256) {
    const uint32_t xs = x0 + k;
    const uint32_t qy = div_small(xs, (uint32_t)G.nx, rnx);
    const uint32_t x = xs - qy * (uint32_t)G.nx;
    const uint32_t ys = y0 + qy;
    const uint32_t qz = div_small(ys, (uint32_t)G.ny, rny);
    const uint32_t y = ys - qz * (uint32_t)G.ny;
    const uint32_t z = z0 + qz;
    const uint32_t tile = ((z >> 3) * G.tny + (y >> 3)) * G.tnx + (x >> 3);
    if constexpr (FACES != FACES_GENERAL) {
      step_cell_bb<T, FACES == FACES_WALLS>((const gchar*)src, (gchar*)dst, (gchar*)F, (gchar*)U,
                                            (const gchar*)tiles, tile, G, omega, flags, (int)x,
                                            (int)y, z, fs);
    } else {
      const uint32_t cell = first + k;
      const CellNbr nb = cell_neighbours(G, (int)x, (int)y, (int)z);
      const uint32_t lc = layout_cell(G, cell, z);
      T g[19];
      pull_all_g<T>(g, src, G, lc, nb, std::make_integer_sequence<int, 19>{});
      const bool forced = static_force || tiles[tile] != 0;
      T ux, uy, uz;
      if (__any(forced)) {
        T Fx = 0, Fy = 0, Fz = 0;
        if (forced) {
          Fx = F[cell];
          Fy = F[G.N + cell];
          Fz = F[2 * (size_t)G.N + cell];
        }
        collide<T, true>(g, Fx, Fy, Fz, omega, ux, uy, uz);
      } else {
        collide<T, false>(g, T(0), T(0), T(0), omega, ux, uy, uz);
      }
#pragma unroll
      for (int q = 0; q < 19; ++q) __builtin_nontemporal_store(g[q], &dst[(size_t)q * G.qs + lc]);
      if (forced || (flags & LBM_FLAG_WRITE_U_ALL)) {
        U[cell] = ux;
        U[G.N + cell] = uy;
        U[2 * (size_t)G.N + cell] = uz;
      }
      if (forced && !static_force) {
        F[cell] = T(0);
        F[G.N + cell] = T(0);
        F[2 * (size_t)G.N + cell] = T(0);
      }
    }
    // the corner cell of each tile clears that tile in the mask of the next bubble step
    if (((x | y | z) & 7) == 0) tiles_next[tile] = 0;
  }
}

}  // namespace lbm
