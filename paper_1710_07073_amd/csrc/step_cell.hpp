// One cell of the fused liquid step on the wall fast path (eq. (13)-(16) with half-way
// bounce-back or free-slip on every face, none periodic, Sec. 3.3), shared by the bulk and region
// kernels of the single-lattice step; the liquid adjoint uses the same gather offsets.
#pragma once

#include <type_traits>
#include <utility>

#include "collide.hpp"

namespace lbm {

// Specialisation for the faces of the method's columns: every face a half-way bounce-back or a
// free-slip wall, one cell per thread, population buffer below 4 GiB. The source of a population
// is then at a fixed (uniform) offset from the destination except for lanes on a wall, so each
// gather is a scalar base plus a 32-bit byte offset selected from a few uniform values, and each
// store (populations, velocity, force) is a scalar base plus the lane's own offset: almost no
// per-lane address arithmetic is left beside the collision.
// Byte offset of the source of population Q of the cell at byte offset lc4 (layout index times the
// element size). walls: bit 0 x = 0, 1 x = nx - 1, 2 y = 0, 3 y = ny - 1, 4 z = 0, 5 z = nz - 1; the
// source x - c lies beyond the wall at x = 0 when c_x > 0, and so on. FS: some face is free slip,
// fs its faces in the same bit order. A source beyond exactly one free-slip face is replaced by the
// population with the normal component mirrored, taken from the source position with the normal
// coordinate kept; beyond a bounce-back face, an edge or a corner by the opposite population of
// the cell itself (the rules of pull_index).
template <int Q, typename T, bool FS = false>
__device__ __forceinline__ uint32_t pull_off_bb(const Geom& G, uint32_t lc4, uint32_t walls,
                                                uint32_t fs = 0u) {
  constexpr int cx = CX[Q], cy = CY[Q], cz = CZ[Q];
  constexpr uint32_t m = (cx > 0 ? 1u : 0u) | (cx < 0 ? 2u : 0u) | (cy > 0 ? 4u : 0u) |
                         (cy < 0 ? 8u : 0u) | (cz > 0 ? 16u : 0u) | (cz < 0 ? 32u : 0u);
  constexpr uint32_t esz = sizeof(T);
  // byte offsets modulo 2^32; the sum with lc4 is the true offset, below 2^32
  const uint32_t k = ((uint32_t)Q * G.qs - (uint32_t)(cx + cy * G.nx) - (uint32_t)cz * G.zs) * esz;
  const uint32_t kb = (uint32_t)opposite(Q) * G.qs * esz;
  if constexpr (!FS) {
    return lc4 + ((walls & m) ? kb : k);
  } else {
    const uint32_t hit = walls & m;
    if (!hit) return lc4 + k;
    if ((hit & (hit - 1u)) == 0u && (hit & fs)) {
      // mirrored across the one crossed face: drop that axis' shift from the offset
      const uint32_t kx = ((uint32_t)mirrored(Q, 0) * G.qs - (uint32_t)(cy * G.nx) -
                           (uint32_t)cz * G.zs) * esz;
      const uint32_t ky = ((uint32_t)mirrored(Q, 1) * G.qs - (uint32_t)cx - (uint32_t)cz * G.zs) * esz;
      const uint32_t kz = ((uint32_t)mirrored(Q, 2) * G.qs - (uint32_t)(cx + cy * G.nx)) * esz;
      return lc4 + ((hit & 3u) ? kx : ((hit & 12u) ? ky : kz));
    }
    return lc4 + kb;
  }
}

// The free-slip faces of G in the bit order of the walls mask.
__device__ __forceinline__ uint32_t free_slip_faces(const Geom& G) {
  uint32_t fs = 0u;
#pragma unroll
  for (int f = 0; f < 6; ++f)
    if (G.bc[f] == BC_FS) fs |= 1u << f;
  return fs;
}

// Byte pointers into device global memory: loads and stores through them are global
// instructions (a scalar base plus a 32-bit lane offset where the base is uniform), also when the
// base comes from a table in memory rather than a kernel argument.
using gchar = __attribute__((address_space(1))) char;
template <typename T>
using gmem = __attribute__((address_space(1))) T;

template <typename T>
__device__ __forceinline__ const gchar* gbytes(const void* p) {
  return (const gchar*)p;
}
template <typename T>
__device__ __forceinline__ gchar* gbytes(void* p) {
  return (gchar*)p;
}
template <typename T>
__device__ __forceinline__ T load_at(const gchar* b, uint32_t off) {
  return *reinterpret_cast<const gmem<T>*>(b + off);
}
template <typename T>
__device__ __forceinline__ void store_at(gchar* b, uint32_t off, T v) {
  *reinterpret_cast<gmem<T>*>(b + off) = v;
}

template <int Q, typename T, bool FS>
__device__ __forceinline__ T pull_bb(const gchar* sb, const Geom& G, uint32_t lc4, uint32_t walls,
                                     uint32_t fs) {
  return load_at<T>(sb, pull_off_bb<Q, T, FS>(G, lc4, walls, fs));
}

__device__ __forceinline__ uint32_t wall_bits(const Geom& G, int x, int y, uint32_t z) {
  return (x == 0 ? 1u : 0u) | (x == G.nx - 1 ? 2u : 0u) | (y == 0 ? 4u : 0u) |
         (y == G.ny - 1 ? 8u : 0u) | (z == 0 ? 16u : 0u) | (z == (uint32_t)G.nz - 1 ? 32u : 0u);
}

template <typename T, bool FS, int... Qs>
__device__ __forceinline__ void pull_bb_all(T* g, const gchar* sb, const Geom& G, uint32_t lc4,
                                            uint32_t walls, uint32_t fs,
                                            std::integer_sequence<int, Qs...>) {
  ((g[Qs] = pull_bb<Qs, T, FS>(sb, G, lc4, walls, fs)), ...);
}

template <typename T>
__device__ __forceinline__ T* at_bytes(T* base, uint32_t off) {
  using B = std::conditional_t<std::is_const_v<T>, const char, char>;
  return reinterpret_cast<T*>(reinterpret_cast<B*>(base) + off);
}

// One cell of the wall fast path: gather, collision, stores. sb, db: the post-collision buffers
// (source and destination), Fb, Ub: the force and velocity fields, tb: the tile mask of the step
// (tile: the cell's tile), as global byte pointers. A flagged tile holds force (read F, write U,
// clear F); the flag is read after the 19 gathers are issued, so that its round trip overlaps
// theirs. FS: some face is free slip (fs: free_slip_faces(G)).
template <typename T, bool FS>
__device__ __forceinline__ void step_cell_bb(const gchar* sb, gchar* db, gchar* Fb, gchar* Ub,
                                             const gchar* tb, uint32_t tile, const Geom& G,
                                             T omega, int flags, int x, int y, uint32_t z,
                                             uint32_t fs) {
  const uint32_t cell = ((uint32_t)z * G.ny + y) * G.nx + x;
  constexpr uint32_t esz = sizeof(T);
  const uint32_t lc4 = layout_cell(G, cell, z) * esz;
  const uint32_t walls = wall_bits(G, x, y, z);
  T g[19];
  pull_bb_all<T, FS>(g, sb, G, lc4, walls, fs, std::make_integer_sequence<int, 19>{});
  const uint32_t c4 = cell * esz;
  const uint32_t n4 = G.N * esz;
  const bool static_force = flags & LBM_FLAG_STATIC_FORCE;
  const bool forced = static_force || tb[tile] != 0;
  const bool wave_forced = __any(forced);
  T ux, uy, uz;
  if (wave_forced) {
    T Fx = T(0), Fy = T(0), Fz = T(0);
    if (forced) {
      Fx = load_at<T>(Fb, c4);
      Fy = load_at<T>(Fb, c4 + n4);
      Fz = load_at<T>(Fb, c4 + 2 * n4);
    }
    collide<T, true>(g, Fx, Fy, Fz, omega, ux, uy, uz);
  } else {
    collide<T, false>(g, T(0), T(0), T(0), omega, ux, uy, uz);
  }
  // one scalar base and a 32-bit offset per store (a 32-bit sum cannot be widened by the compiler)
  const uint32_t qs4 = G.qs * esz;
#pragma unroll
  for (int q = 0; q < 19; ++q)
    __builtin_nontemporal_store(g[q], reinterpret_cast<gmem<T>*>(db + (lc4 + (uint32_t)q * qs4)));
  if (forced || (flags & LBM_FLAG_WRITE_U_ALL)) {
    store_at<T>(Ub, c4, ux);
    store_at<T>(Ub, c4 + n4, uy);
    store_at<T>(Ub, c4 + 2 * n4, uz);
  }
  if (forced && !static_force) {
    store_at<T>(Fb, c4, T(0));
    store_at<T>(Fb, c4 + n4, T(0));
    store_at<T>(Fb, c4 + 2 * n4, T(0));
  }
}

}  // namespace lbm
