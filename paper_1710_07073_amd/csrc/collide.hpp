// Per-cell pieces of the fused liquid step shared by the single-lattice and the batched kernels:
// the 19-population gather with face conditions, and the BGK collision with the Guo force term
// (Sec. 2.2, eq. (6), (12)-(15)), in shifted variables g = f - w.
#pragma once

#include <utility>

#include "internal.hpp"

namespace lbm {

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

// c * v for a lattice weight (or a multiple of one) c given in double. In FP32, c is carried as
// hi + lo (hi the float nearest to c, lo the float nearest to c - hi): a single rounded constant
// is off by up to 3e-8 relative, always in the same direction, and multiplied into the
// equilibrium's density and momentum every step that offset compounds. With 3w rounded, the
// equilibrium returns the momentum times 1 + 3e-8, so each collision grows the momentum by
// omega * 3e-8 (the velocity of an FP32 run then drifts from the FP64 one by 1.8e-5 relative L2
// after 1000 steps of the 128 x 128 x 512 column at omega 1.6; 2.4e-7 with the split).
template <typename T>
__device__ __forceinline__ T mul_weight(double c, T v) {
  if constexpr (sizeof(T) == 4) {
    const float hi = (float)c, lo = (float)(c - (double)hi);
    return fma(hi, v, lo * v);
  } else {
    return T(c) * v;
  }
}

// BGK collision with the Guo force term, in place on the 19 shifted populations. Opposite
// directions are handled as pairs: the equilibrium (6) and the force term (12) split into a part
// even in c and a part odd in c. Returns the velocity of eq. (13).
//
// The arithmetic is written out operation by operation (contraction off, fused multiply-adds
// explicit), so every kernel that inlines it computes the same bits whatever the surrounding code;
// with a zero force the forced variant returns the unforced result exactly (every force term is an
// exact zero added last), which lets kernels choose the variant per wavefront or per tile. In
// FP32 the equilibrium's odd part 3 w rho (c . u) is formed as 3 w (c . (j + F/2)), the momentum
// itself rather than rho times the divided velocity, and the terms linear in the density deviation
// and the momentum take their weights through mul_weight (no rounding bias); FP64 keeps the plain
// products.
template <typename T, bool FORCED>
__device__ __forceinline__ void collide(T* g, T Fx, T Fy, T Fz, T omega, T& ux, T& uy, T& uz) {
#pragma clang fp contract(off)
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
  // momentum rho u of eq. (13)
  const T mx = FORCED ? fma(T(0.5), Fx, jx) : jx;
  const T my = FORCED ? fma(T(0.5), Fy, jy) : jy;
  const T mz = FORCED ? fma(T(0.5), Fz, jz) : jz;
  ux = mx * inv;
  uy = my * inv;
  uz = mz * inv;
  const T usq = fma(ux, ux, fma(uy, uy, uz * uz));
  const T om1 = T(1) - omega;
  const T pre = T(1) - T(0.5) * omega;
  const T uF = FORCED ? fma(ux, Fx, fma(uy, Fy, uz * Fz)) : T(0);
  const T m15usq = T(-1.5) * usq;
  // rest particle
  {
    constexpr int q = 18;
    const T geq = fma(weight<T>(q) * rho, m15usq, mul_weight<T>(1.0 / 3.0, drho));
    T v = fma(omega, geq, om1 * g[q]);
    if (FORCED) v = v + pre * weight<T>(q) * (T(-3) * uF);
    g[q] = v;
  }
#pragma unroll
  for (int q = 0; q < 18; ++q) {
    const int qb = opposite(q);
    if (qb < q) continue;  // each pair once, from its lower index
    const T cu = T(CX[q]) * ux + T(CY[q]) * uy + T(CZ[q]) * uz;
    const T w = weight<T>(q);
    // w rho and w drho are common to the pairs of one weight class
    const double wd = q < 6 ? 1.0 / 18.0 : 1.0 / 36.0;
    const T sym = fma(w * rho, fma(T(4.5) * cu, cu, m15usq), mul_weight<T>(wd, drho));
    T asym;
    if constexpr (sizeof(T) == 4) {
      const T cm = T(CX[q]) * mx + T(CY[q]) * my + T(CZ[q]) * mz;
      asym = mul_weight<T>(3.0 * wd, cm);
    } else {
      asym = (T(3) * w) * rho * cu;
    }
    T vp = fma(omega, sym + asym, om1 * g[q]);
    T vm = fma(omega, sym - asym, om1 * g[qb]);
    if (FORCED) {
      const T cF = T(CX[q]) * Fx + T(CY[q]) * Fy + T(CZ[q]) * Fz;
      const T ssym = pre * w * fma(T(9) * cu, cF, T(-3) * uF);
      const T sasym = pre * (T(3) * w) * cF;
      vp = vp + (ssym + sasym);
      vm = vm + (ssym - sasym);
    }
    g[q] = vp;
    g[qb] = vm;
  }
}

}  // namespace lbm
