// Fused one-pass liquid step (Sec. 2.2, eq. (13)-(16), Sec. 3.3): each thread owns one cell,
// pulls its 19 populations from the post-collision buffer of the previous step (streaming with
// the face conditions), computes the moments with the half-force correction (13), relaxes to the
// equilibrium (6) with BGK (14), adds the Guo force term (12), (15), and stores the 19
// post-collision populations into the other buffer. All in shifted variables g = f - w.
//
// Populations are addressed through the buffer layout of Geom (layout index lc); the force and
// velocity fields through the flat cell index.
//
// Memory traffic per cell: 19 loads + 19 stores of the lattice type (152 B in FP32, 304 B in
// FP64); the force (3 loads, 3 stores to clear it) and the velocity (3 stores) are touched only in
// 8^3 tiles flagged by the bubble kernel, whose mask is a byte per tile.
#include <algorithm>
#include <utility>

#include "collide.hpp"
#include "step_cell.hpp"

namespace lbm {
namespace {

// VEC consecutive cells along x per thread (VEC = 1, 2 or 4; nx % VEC == 0). Interior threads
// gather each population as one VEC-wide load: the source run is contiguous in x (shifted by
// -c_x, so not VEC-aligned when c_x != 0) and lies in one row (y - c_y, z - c_z), so a wall in y
// or z replaces the whole run. Threads whose run touches x = 0 or x = nx - 1 gather element by
// element with the full face logic.
template <typename T, int VEC>
struct VecT {
  typedef T type __attribute__((ext_vector_type(VEC)));
};

template <typename T, int VEC>
__device__ __forceinline__ void load_run(T* out, const T* p) {
  if constexpr (VEC == 1) {
    out[0] = *p;
  } else {
    typename VecT<T, VEC>::type v;
    __builtin_memcpy(&v, p, sizeof(v));
#pragma unroll
    for (int e = 0; e < VEC; ++e) out[e] = v[e];
  }
}

template <typename T, int VEC>
__device__ __forceinline__ void store_run(T* p, const T* in, bool nontemporal) {
  if constexpr (VEC == 1) {
    if (nontemporal)
      __builtin_nontemporal_store(in[0], p);
    else
      *p = in[0];
  } else {
    typename VecT<T, VEC>::type v;
#pragma unroll
    for (int e = 0; e < VEC; ++e) v[e] = in[e];
    typedef typename VecT<T, VEC>::type vt;
    if (nontemporal)
      __builtin_nontemporal_store(v, reinterpret_cast<vt*>(p));
    else
      *reinterpret_cast<vt*>(p) = v;
  }
}

template <int Q, bool GENERAL, int VEC, typename T>
__device__ __forceinline__ void pull_run(T (*g)[19], const T* __restrict__ src, const Geom& G,
                                         uint32_t lc, const CellNbr& nb) {
  constexpr int cx = CX[Q], cy = CY[Q], cz = CZ[Q];
  int32_t off = -cx;
  bool oy = false, oz = false;
  int32_t dy = 0, dz = 0;
  if (cy > 0) { dy = nb.dm[1]; oy = nb.om[1]; }
  if (cy < 0) { dy = nb.dp[1]; oy = nb.op[1]; }
  if (cz > 0) { dz = nb.dm[2]; oz = nb.om[2]; }
  if (cz < 0) { dz = nb.dp[2]; oz = nb.op[2]; }
  off += dy + dz;
  T v[VEC];
  if (!(oy || oz)) {
    load_run<T, VEC>(v, src + (size_t)Q * G.qs + (uint32_t)((int32_t)lc + off));
  } else {
    bool done = false;
    if constexpr (GENERAL) {
      if (oy != oz) {
        const int a = oy ? 1 : 2;
        const int c = a == 1 ? cy : cz;
        if (G.bc[2 * a + (c > 0 ? 0 : 1)] == BC_FS) {
          const int qm = a == 1 ? mirrored(Q, 1) : mirrored(Q, 2);
          load_run<T, VEC>(v, src + (size_t)qm * G.qs + (uint32_t)((int32_t)lc + off - (a == 1 ? dy : dz)));
          done = true;
        }
      }
    }
    if (!done) load_run<T, VEC>(v, src + (size_t)opposite(Q) * G.qs + lc);
  }
#pragma unroll
  for (int e = 0; e < VEC; ++e) g[e][Q] = v[e];
}

template <bool GENERAL, int VEC, typename T, int... Qs>
__device__ __forceinline__ void pull_runs(T (*g)[19], const T* __restrict__ src, const Geom& G,
                                          uint32_t lc, const CellNbr& nb,
                                          std::integer_sequence<int, Qs...>) {
  (pull_run<Qs, GENERAL, VEC>(g, src, G, lc, nb), ...);
}

template <typename T, int VEC, bool GENERAL>
__global__ __launch_bounds__(256) void k_step(const T* __restrict__ src, T* __restrict__ dst,
                                              T* __restrict__ F, T* __restrict__ U,
                                              const uint8_t* __restrict__ tiles,
                                              uint8_t* __restrict__ tiles_next, Geom G, T omega,
                                              int flags, uint32_t bx_blocks, uint32_t by_blocks) {
  // workgroups in launch order: the dispatcher deals consecutive ones to the eight XCDs in turn,
  // so the chip streams one compact window of planes at a time (measured faster on the fused
  // step than giving each XCD a contiguous eighth of the lattice)
  const uint32_t L = blockIdx.x;
  const uint32_t bxi = L % bx_blocks;
  const uint32_t rest = L / bx_blocks;
  const uint32_t byi = rest % by_blocks;
  const uint32_t z = rest / by_blocks;
  const int x0 = (int)(bxi * blockDim.x + threadIdx.x) * VEC;
  const int y = (int)(byi * blockDim.y + threadIdx.y);
  if (x0 >= G.nx || y >= G.ny) return;
  const uint32_t cell = ((uint32_t)z * G.ny + y) * G.nx + x0;
  const uint32_t lc = layout_cell(G, cell, z);
  T g[VEC][19];
  const bool xedge = VEC > 1 && (x0 == 0 || x0 + VEC == G.nx);
  if (VEC == 1 || xedge) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const CellNbr nb = cell_neighbours(G, x0 + e, y, (int)z);
      pull_all<GENERAL>(g[e], src, G, lc + e, nb, std::make_integer_sequence<int, 19>{});
    }
  } else {
    const CellNbr nb = cell_neighbours(G, x0, y, (int)z);
    pull_runs<GENERAL, VEC>(g, src, G, lc, nb, std::make_integer_sequence<int, 19>{});
  }

  const bool static_force = flags & LBM_FLAG_STATIC_FORCE;
  const uint32_t tile = ((z >> 3) * G.tny + ((uint32_t)y >> 3)) * G.tnx + ((uint32_t)x0 >> 3);
  bool forced = static_force;
  if (!static_force) forced = tiles[tile] != 0;
  // the corner cell of each tile clears that tile in the mask of the next bubble step
  if (((x0 | y | (int)z) & 7) == 0) tiles_next[tile] = 0;
  T ux[VEC], uy[VEC], uz[VEC];
  if (__any(forced)) {
    T Fx[VEC], Fy[VEC], Fz[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) Fx[e] = Fy[e] = Fz[e] = T(0);
    if (forced) {
      load_run<T, VEC>(Fx, F + cell);
      load_run<T, VEC>(Fy, F + G.N + cell);
      load_run<T, VEC>(Fz, F + 2 * (size_t)G.N + cell);
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) collide<T, true>(g[e], Fx[e], Fy[e], Fz[e], omega, ux[e], uy[e], uz[e]);
  } else {
#pragma unroll
    for (int e = 0; e < VEC; ++e) collide<T, false>(g[e], T(0), T(0), T(0), omega, ux[e], uy[e], uz[e]);
  }
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    T v[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) v[e] = g[e][q];
    store_run<T, VEC>(dst + (size_t)q * G.qs + lc, v, true);
  }
  if (forced || (flags & LBM_FLAG_WRITE_U_ALL)) {
    store_run<T, VEC>(U + cell, ux, false);
    store_run<T, VEC>(U + G.N + cell, uy, false);
    store_run<T, VEC>(U + 2 * (size_t)G.N + cell, uz, false);
  }
  if (forced && !static_force) {
    T zero[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) zero[e] = T(0);
    store_run<T, VEC>(F + cell, zero, false);
    store_run<T, VEC>(F + G.N + cell, zero, false);
    store_run<T, VEC>(F + 2 * (size_t)G.N + cell, zero, false);
  }
}

// The whole lattice (region == nullptr), or the bulk of an overlapped step: every cell whose tile
// row is not in the region. No face periodic; FS: some face free slip.
template <typename T, bool FS>
__global__ __launch_bounds__(256) void k_step_bb(const T* __restrict__ src, T* __restrict__ dst,
                                                 T* __restrict__ F, T* __restrict__ U,
                                                 const uint8_t* __restrict__ tiles,
                                                 uint8_t* __restrict__ tiles_next,
                                                 const uint32_t* __restrict__ region, Geom G,
                                                 T omega, int flags, uint32_t bx_blocks,
                                                 uint32_t by_blocks) {
  // workgroups in launch order: the dispatcher deals consecutive ones to the eight XCDs in turn,
  // so the chip streams one compact window of planes at a time (measured faster on the fused
  // step than giving each XCD a contiguous eighth of the lattice)
  const uint32_t L = blockIdx.x;
  const uint32_t bxi = L % bx_blocks;
  const uint32_t rest = L / bx_blocks;
  const uint32_t byi = rest % by_blocks;
  const uint32_t z = rest / by_blocks;
  const int x = (int)(bxi * blockDim.x + threadIdx.x);
  const int y = (int)(byi * blockDim.y + threadIdx.y);
  if (x >= G.nx || y >= G.ny) return;
  const uint32_t tile = ((z >> 3) * G.tny + ((uint32_t)y >> 3)) * G.tnx + ((uint32_t)x >> 3);
  if (region && region[(z >> 3) * G.tny + ((uint32_t)y >> 3)]) return;  // the region launch's
  step_cell_bb<T, FS>(gbytes<T>(src), gbytes<T>(dst), gbytes<T>(F), gbytes<T>(U),
                      gbytes<uint8_t>(tiles), tile, G, omega, flags, x, y, z,
                      FS ? free_slip_faces(G) : 0u);
  // the corner cell of each tile clears that tile in the mask of the next bubble step
  if (((x | y | (int)z) & 7) == 0) tiles_next[tile] = 0;
}

// The region of an overlapped step: the tile rows of its list, each cut into the same workgroups
// as the bulk launch (bx by by cells of one z-plane). It runs after the bubble kernels, alongside
// the bulk launch; it clears the flags of its rows.
template <typename T, bool FS>
__global__ __launch_bounds__(256) void k_region_bb(const T* __restrict__ src, T* __restrict__ dst,
                                                   T* __restrict__ F, T* __restrict__ U,
                                                   const uint8_t* __restrict__ tiles,
                                                   uint8_t* __restrict__ tiles_next,
                                                   uint32_t* __restrict__ region,
                                                   const uint32_t* __restrict__ list,
                                                   const uint32_t* __restrict__ count, Geom G,
                                                   T omega, int flags, uint32_t nrows,
                                                   uint32_t bx_blocks, uint32_t by_blocks) {
  const uint32_t n = min(*count, nrows);
  const uint32_t per = bx_blocks * by_blocks * kTile;  // workgroups per row
#pragma unroll 1
  for (uint32_t w = blockIdx.x; w < n * per; w += gridDim.x) {
    const uint32_t u = list[w / per], sub = w % per;
    const uint32_t bxi = sub % bx_blocks, rest = sub / bx_blocks;
    const uint32_t byi = rest % by_blocks, zz = rest / by_blocks;
    const uint32_t ty = u % (uint32_t)G.tny, tz = u / (uint32_t)G.tny;
    const int x = (int)(bxi * blockDim.x + threadIdx.x);
    const uint32_t yr = byi * blockDim.y + threadIdx.y;  // row within the tile row
    const int y = (int)(ty * kTile + yr);
    const uint32_t z = tz * kTile + zz;
    if (x < G.nx && y < G.ny && yr < kTile && z < (uint32_t)G.nz) {
      const uint32_t tile = ((z >> 3) * G.tny + ((uint32_t)y >> 3)) * G.tnx + ((uint32_t)x >> 3);
      step_cell_bb<T, FS>(gbytes<T>(src), gbytes<T>(dst), gbytes<T>(F), gbytes<T>(U),
                          gbytes<uint8_t>(tiles), tile, G, omega, flags, x, y, z,
                          FS ? free_slip_faces(G) : 0u);
      if (((x | y | (int)z) & 7) == 0) tiles_next[tile] = 0;
    }
    if (sub == 0 && threadIdx.x == 0 && threadIdx.y == 0) region[u] = 0u;
  }
}

template <typename T, int VEC, bool GENERAL>
hipError_t launch_typed(lbm_ctx* c, uint32_t bx) {
  const Geom& G = c->geom;
  const uint32_t by = 256 / bx;
  const uint32_t nbx = div_up(G.nx / VEC, bx), nby = div_up(G.ny, by);
  const uint32_t nblocks = nbx * nby * (uint32_t)G.nz;
  const T* src = static_cast<const T*>(c->pops[c->hs.cur]);
  T* dst = static_cast<T*>(c->pops[c->hs.cur ^ 1]);
  if (VEC == 1 && !c->periodic && bb_fast_ok(G, sizeof(T))) {
    // walls only: GENERAL then means some face is free slip
    hipLaunchKernelGGL((k_step_bb<T, GENERAL>), dim3(nblocks), dim3(bx, by), step_lds(c), c->stream, src, dst,
                       static_cast<T*>(c->force), static_cast<T*>(c->vel), c->tiles[c->hs.flag_cur],
                       c->tiles[c->hs.flag_cur ^ 1], nullptr, G, (T)c->desc.omega, c->desc.flags,
                       nbx, nby);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_step<T, VEC, GENERAL>), dim3(nblocks), dim3(bx, by), step_lds(c), c->stream, src, dst,
                     static_cast<T*>(c->force), static_cast<T*>(c->vel), c->tiles[c->hs.flag_cur],
                     c->tiles[c->hs.flag_cur ^ 1], G, (T)c->desc.omega, c->desc.flags, nbx, nby);
  return hipGetLastError();
}

template <typename T, bool GENERAL>
hipError_t launch_vec(lbm_ctx* c) {
  switch (c->step_vec) {
    case 4: return launch_typed<T, 4, GENERAL>(c, c->step_bx);
    case 2: return launch_typed<T, 2, GENERAL>(c, c->step_bx);
    default: return launch_typed<T, 1, GENERAL>(c, c->step_bx);
  }
}

// Records the caller's timing events (if any) around one launch on stream s.
template <class F>
hipError_t timed(lbm_ctx* c, hipStream_t s, F&& launch) {
  hipEvent_t a = c->t_start, b = c->t_end;
  c->t_start = c->t_end = nullptr;
  hipError_t e = a ? hipEventRecord(a, s) : hipSuccess;
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess && b) e = hipEventRecord(b, s);
  return e;
}

template <typename T, bool FS>
hipError_t launch_bulk_typed(lbm_ctx* c) {
  const Geom& G = c->geom;
  const uint32_t bx = c->step_bx, by = 256 / bx;
  const uint32_t nbx = div_up(G.nx, bx), nby = div_up(G.ny, by);
  const uint32_t nblocks = nbx * nby * (uint32_t)G.nz;
  hipLaunchKernelGGL((k_step_bb<T, FS>), dim3(nblocks), dim3(bx, by), step_lds(c), c->stream,
                     static_cast<const T*>(c->pops[c->hs.cur]), static_cast<T*>(c->pops[c->hs.cur ^ 1]),
                     static_cast<T*>(c->force), static_cast<T*>(c->vel), c->tiles[c->hs.flag_cur],
                     c->tiles[c->hs.flag_cur ^ 1], c->region[c->hs.rpar], G, (T)c->desc.omega,
                     c->desc.flags, nbx, nby);
  return hipGetLastError();
}

template <typename T, bool FS>
hipError_t launch_region_typed(lbm_ctx* c, int32_t nb, hipStream_t stream) {
  const Geom& G = c->geom;
  const uint32_t bx = c->step_bx, by = 256 / bx;
  const uint32_t bx_blocks = div_up(G.nx, bx), by_blocks = div_up(kTile, by);
  const uint64_t per = (uint64_t)bx_blocks * by_blocks * kTile;
  // about 16 rows per bubble for the stencils of d <= 5 at kernel factor 1.5; more are strided
  const uint64_t rows = std::min<uint64_t>((uint64_t)nb * 16, c->nrows);
  const uint32_t blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(rows * per, 16384));
  const int r = c->hs.rpar;
  hipLaunchKernelGGL((k_region_bb<T, FS>), dim3(blocks), dim3(bx, by), step_lds(c), stream,
                     static_cast<const T*>(c->pops[c->hs.cur]), static_cast<T*>(c->pops[c->hs.cur ^ 1]),
                     static_cast<T*>(c->force), static_cast<T*>(c->vel), c->tiles[c->hs.flag_cur],
                     c->tiles[c->hs.flag_cur ^ 1], c->region[r], c->region_list[r], c->region_count + r,
                     G, (T)c->desc.omega, c->desc.flags, c->nrows,
                     bx_blocks, by_blocks);
  return hipGetLastError();
}

}  // namespace

bool can_overlap(const lbm_ctx* c) {
  return c->side && !c->periodic && c->step_vec == 1 && bb_fast_ok(c->geom, c->elem);
}

hipError_t launch_bulk(lbm_ctx* c) {
  return timed(c, c->stream, [&] {
    if (c->elem == 4)
      return c->general ? launch_bulk_typed<float, true>(c) : launch_bulk_typed<float, false>(c);
    return c->general ? launch_bulk_typed<double, true>(c) : launch_bulk_typed<double, false>(c);
  });
}

hipError_t launch_step(lbm_ctx* c) {
  hipError_t e;
  const bool overlapped = c->hs.pending;
  if (overlapped) {
    // overlapped step: the bulk and the bubble kernels are enqueued and the caller's stream waits
    // for the bubble kernels; the region runs after the bulk, alone on the chip. (Launched on the
    // side stream right after the bubble kernels, with its row flags cleared by the next step
    // rather than by the region kernel, it was bitwise identical and 0.7 % faster on 128 x 128 x
    // 512 with one bubble, 0.4 % on 256 x 256 x 768 with 20 000: too little for flags that
    // outlive their step and must then be cleared on every switch between serial and overlapped.)
    if (c->elem == 4)
      e = c->general ? launch_region_typed<float, true>(c, c->pending_nb, c->stream)
                     : launch_region_typed<float, false>(c, c->pending_nb, c->stream);
    else
      e = c->general ? launch_region_typed<double, true>(c, c->pending_nb, c->stream)
                     : launch_region_typed<double, false>(c, c->pending_nb, c->stream);
    if (e != hipSuccess) return e;
    c->hs.pending = false;
    c->hs.rpar ^= 1;
  } else {
    e = timed(c, c->stream, [&] {
      if (c->elem == 4) return c->general ? launch_vec<float, true>(c) : launch_vec<float, false>(c);
      return c->general ? launch_vec<double, true>(c) : launch_vec<double, false>(c);
    });
  }
  if (e == hipSuccess) {
    c->hs.cur ^= 1;
    c->hs.flag_clean[c->hs.flag_cur ^ 1] = true;
    c->hs.last_overlapped = overlapped;
    ++c->hs.steps;
  }
  return e;
}

}  // namespace lbm
