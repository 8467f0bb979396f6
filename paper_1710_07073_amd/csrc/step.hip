// Fused one-pass liquid step (Sec. 2.2, eq. (13)-(16), Sec. 3.3): each thread owns one cell,
// pulls its 19 populations from the post-collision buffer of the previous step (streaming with
// the face conditions), computes the moments with the half-force correction (13), relaxes to the
// equilibrium (6) with BGK (14), adds the Guo force term (12), (15), and stores the 19
// post-collision populations into the other buffer. All in shifted variables g = f - w.
//
// Memory traffic per cell: 19 loads + 19 stores of the lattice type (152 B in FP32, 304 B in
// FP64); the force (3 loads, 3 stores to clear it) and the velocity (3 stores) are touched only in
// 8^3 tiles flagged by the bubble kernel, whose mask is a byte per tile.
#include <utility>

#include "internal.hpp"

namespace lbm {
namespace {

template <bool GENERAL, typename T, int... Qs>
__device__ __forceinline__ void pull_all(T* g, const T* __restrict__ src, const Geom& G,
                                         uint32_t cell, const CellNbr& nb,
                                         std::integer_sequence<int, Qs...>) {
  ((g[Qs] = pull<Qs, GENERAL>(src, G, cell, nb)), ...);
}

template <typename T>
__device__ __forceinline__ T recip(T v) {
  return T(1) / v;
}
template <>
__device__ __forceinline__ float recip<float>(float v) {
  return __builtin_amdgcn_rcpf(v);
}

// BGK collision with the Guo force term, in place on the 19 shifted populations. Opposite
// directions are handled as pairs: the equilibrium (6) and the force term (12) split into a part
// even in c and a part odd in c. Returns the velocity of eq. (13).
template <typename T, bool FORCED>
__device__ __forceinline__ void collide(T* g, T Fx, T Fy, T Fz, T omega, T& ux, T& uy, T& uz) {
  T drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    drho += g[q];
    if (CX[q] > 0) jx += g[q];
    if (CX[q] < 0) jx -= g[q];
    if (CY[q] > 0) jy += g[q];
    if (CY[q] < 0) jy -= g[q];
    if (CZ[q] > 0) jz += g[q];
    if (CZ[q] < 0) jz -= g[q];
  }
  const T rho = T(1) + drho;
  const T inv = recip(rho);
  if (FORCED) {
    ux = (jx + T(0.5) * Fx) * inv;
    uy = (jy + T(0.5) * Fy) * inv;
    uz = (jz + T(0.5) * Fz) * inv;
  } else {
    ux = jx * inv;
    uy = jy * inv;
    uz = jz * inv;
  }
  const T usq = ux * ux + uy * uy + uz * uz;
  const T om1 = T(1) - omega;
  const T pre = T(1) - T(0.5) * omega;
  const T uF = FORCED ? (ux * Fx + uy * Fy + uz * Fz) : T(0);
  // rest particle
  {
    constexpr int q = 18;
    const T geq = weight<T>(q) * (drho - rho * T(1.5) * usq);
    T v = om1 * g[q] + omega * geq;
    if (FORCED) v += pre * weight<T>(q) * (T(-3) * uF);
    g[q] = v;
  }
#pragma unroll
  for (int q = 0; q < 18; ++q) {
    const int qb = opposite(q);
    if (qb < q) continue;  // each pair once, from its lower index
    const T cu = T(CX[q]) * ux + T(CY[q]) * uy + T(CZ[q]) * uz;
    const T w = weight<T>(q);
    const T sym = w * (drho + rho * (T(4.5) * cu * cu - T(1.5) * usq));
    const T asym = w * rho * T(3) * cu;
    T vp = om1 * g[q] + omega * (sym + asym);
    T vm = om1 * g[qb] + omega * (sym - asym);
    if (FORCED) {
      const T cF = T(CX[q]) * Fx + T(CY[q]) * Fy + T(CZ[q]) * Fz;
      const T ssym = pre * w * (T(9) * cu * cF - T(3) * uF);
      const T sasym = pre * w * T(3) * cF;
      vp += ssym + sasym;
      vm += ssym - sasym;
    }
    g[q] = vp;
    g[qb] = vm;
  }
}

template <typename T, bool GENERAL>
__global__ __launch_bounds__(256) void k_step(const T* __restrict__ src, T* __restrict__ dst,
                                              T* __restrict__ F, T* __restrict__ U,
                                              const uint8_t* __restrict__ tiles, Geom G, T omega,
                                              int flags, uint32_t bx_blocks, uint32_t by_blocks,
                                              uint32_t nblocks) {
  const uint32_t L = xcd_remap(blockIdx.x, nblocks);
  const uint32_t bxi = L % bx_blocks;
  const uint32_t rest = L / bx_blocks;
  const uint32_t byi = rest % by_blocks;
  const uint32_t z = rest / by_blocks;
  const int x = (int)(bxi * blockDim.x + threadIdx.x);
  const int y = (int)(byi * blockDim.y + threadIdx.y);
  if (x >= G.nx || y >= G.ny) return;
  const uint32_t cell = ((uint32_t)z * G.ny + y) * G.nx + x;
  const CellNbr nb = cell_neighbours(G, x, y, (int)z);
  T g[19];
  pull_all<GENERAL>(g, src, G, cell, nb, std::make_integer_sequence<int, 19>{});

  const bool static_force = flags & LBM_FLAG_STATIC_FORCE;
  bool forced = static_force;
  if (!static_force) forced = tiles[((z >> 3) * G.tny + ((uint32_t)y >> 3)) * G.tnx + ((uint32_t)x >> 3)] != 0;
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
  for (int q = 0; q < 19; ++q) __builtin_nontemporal_store(g[q], &dst[(size_t)q * G.N + cell]);
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

template <typename T, bool GENERAL>
hipError_t launch_typed(lbm_ctx* c) {
  const Geom& G = c->geom;
  uint32_t bx = G.nx >= 256 ? 256 : (G.nx >= 128 ? 128 : 64);
  if (bx > 64 && (G.nx % bx) != 0) bx = 64;
  const uint32_t by = 256 / bx;
  const uint32_t nbx = div_up(G.nx, bx), nby = div_up(G.ny, by);
  const uint32_t nblocks = nbx * nby * (uint32_t)G.nz;
  const T* src = static_cast<const T*>(c->pops[c->cur]);
  T* dst = static_cast<T*>(c->pops[c->cur ^ 1]);
  hipLaunchKernelGGL((k_step<T, GENERAL>), dim3(nblocks), dim3(bx, by), 0, c->stream, src, dst,
                     static_cast<T*>(c->force), static_cast<T*>(c->vel), c->tiles, G,
                     (T)c->desc.omega, c->desc.flags, nbx, nby, nblocks);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step(lbm_ctx* c) {
  hipError_t e;
  if (c->elem == 4)
    e = c->general ? launch_typed<float, true>(c) : launch_typed<float, false>(c);
  else
    e = c->general ? launch_typed<double, true>(c) : launch_typed<double, false>(c);
  if (e == hipSuccess) {
    c->cur ^= 1;
    ++c->steps;
  }
  return e;
}

}  // namespace lbm
