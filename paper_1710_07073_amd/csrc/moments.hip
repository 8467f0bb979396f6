// Macroscopic fields and global sums of the current state (eq. (10)), the pre-collision
// population view, and a plain fill kernel. The stored buffer holds post-collision populations,
// so both gathers apply the streaming step (with the face conditions) on the fly.
#include <utility>

#include "collide.hpp"

namespace lbm {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Grid-stride over cells; per-block partial sums of (sum drho, sum rho u) in double precision.
template <typename T, bool GENERAL>
__global__ __launch_bounds__(kThreads) void k_moments(const T* __restrict__ src, T* __restrict__ rho,
                                                      T* __restrict__ u, double* __restrict__ partials,
                                                      Geom G) {
  __shared__ double s[4][kThreads / 64];
  double acc[4] = {0, 0, 0, 0};
  const uint32_t stride = gridDim.x * kThreads;
  for (uint32_t cell = blockIdx.x * kThreads + threadIdx.x; cell < G.N; cell += stride) {
    const uint32_t x = cell % G.nx, y = (cell / G.nx) % G.ny, z = cell / G.plane;
    const CellNbr nb = cell_neighbours(G, (int)x, (int)y, (int)z);
    T g[19];
    pull_all<GENERAL>(g, src, G, layout_cell(G, cell, z), nb, std::make_integer_sequence<int, 19>{});
    double drho = 0, m[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < 19; ++q) {
      drho += (double)g[q];
      if (CX[q]) m[0] += CX[q] * (double)g[q];
      if (CY[q]) m[1] += CY[q] * (double)g[q];
      if (CZ[q]) m[2] += CZ[q] * (double)g[q];
    }
    if (rho) rho[cell] = (T)(1.0 + drho);
    if (u) {
      const double r = 1.0 + drho;
      u[cell] = (T)(m[0] / r);
      u[G.N + cell] = (T)(m[1] / r);
      u[2 * (size_t)G.N + cell] = (T)(m[2] / r);
    }
    acc[0] += drho;
    acc[1] += m[0];
    acc[2] += m[1];
    acc[3] += m[2];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double v = wave_sum(acc[k]);
    if ((threadIdx.x & 63) == 0) s[k][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double v = 0;
    for (int w = 0; w < kThreads / 64; ++w) v += s[threadIdx.x][w];
    partials[blockIdx.x * 4 + threadIdx.x] = v;
  }
}

// One block: fixed-order sum of the partials (deterministic), result[0] = N + sum drho.
__global__ __launch_bounds__(kThreads) void k_reduce(const double* __restrict__ partials, int nblocks,
                                                     double ncells, double* __restrict__ result) {
  __shared__ double s[4][kThreads / 64];
  double acc[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += kThreads)
    for (int k = 0; k < 4; ++k) acc[k] += partials[b * 4 + k];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double v = wave_sum(acc[k]);
    if ((threadIdx.x & 63) == 0) s[k][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double v = 0;
    for (int w = 0; w < kThreads / 64; ++w) v += s[threadIdx.x][w];
    result[threadIdx.x] = threadIdx.x == 0 ? ncells + v : v;
  }
}

template <typename T, bool GENERAL>
__global__ __launch_bounds__(kThreads) void k_populations(const T* __restrict__ src, T* __restrict__ out,
                                                          Geom G) {
  const uint32_t cell = blockIdx.x * kThreads + threadIdx.x;
  if (cell >= G.N) return;
  const uint32_t x = cell % G.nx, y = (cell / G.nx) % G.ny, z = cell / G.plane;
  const CellNbr nb = cell_neighbours(G, (int)x, (int)y, (int)z);
  T g[19];
  pull_all<GENERAL>(g, src, G, layout_cell(G, cell, z), nb, std::make_integer_sequence<int, 19>{});
  // exported in the plain (19, nz, ny, nx) order whatever the buffer layout
#pragma unroll
  for (int q = 0; q < 19; ++q) out[(size_t)q * G.N + cell] = g[q];
}

__global__ __launch_bounds__(kThreads) void k_fill(uint32_t* __restrict__ p, size_t words) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < words; i += stride) p[i] = 0u;
}

__global__ void k_fill_bytes(uint8_t* __restrict__ p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

template <typename T, bool GENERAL>
hipError_t moments_typed(lbm_ctx* c, void* rho, void* u) {
  const uint32_t blocks = c->nred;
  c->bins_clean = false;
  hipLaunchKernelGGL((k_moments<T, GENERAL>), dim3(blocks), dim3(kThreads), 0, c->stream,
                     static_cast<const T*>(c->pops[c->hs.cur]), static_cast<T*>(rho),
                     static_cast<T*>(u), c->partials, c->geom);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kThreads), 0, c->stream, c->partials, (int)blocks,
                     (double)c->geom.N, c->result);
  return hipGetLastError();
}

template <typename T, bool GENERAL>
hipError_t populations_typed(lbm_ctx* c, void* out) {
  hipLaunchKernelGGL((k_populations<T, GENERAL>), dim3(div_up(c->geom.N, kThreads)), dim3(kThreads),
                     0, c->stream, static_cast<const T*>(c->pops[c->hs.cur]), static_cast<T*>(out),
                     c->geom);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_moments(lbm_ctx* c, void* rho, void* u, bool) {
  if (c->elem == 4)
    return c->general ? moments_typed<float, true>(c, rho, u) : moments_typed<float, false>(c, rho, u);
  return c->general ? moments_typed<double, true>(c, rho, u) : moments_typed<double, false>(c, rho, u);
}

hipError_t launch_populations(lbm_ctx* c, void* out) {
  if (c->elem == 4)
    return c->general ? populations_typed<float, true>(c, out) : populations_typed<float, false>(c, out);
  return c->general ? populations_typed<double, true>(c, out)
                    : populations_typed<double, false>(c, out);
}

hipError_t launch_fill(void* ptr, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const size_t words = bytes / 4;
  if (words) {
    size_t blocks = (words + kThreads - 1) / kThreads;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill, dim3((uint32_t)blocks), dim3(kThreads), 0, s,
                       static_cast<uint32_t*>(ptr), words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const size_t tail = bytes - words * 4;
  if (tail) {
    hipLaunchKernelGGL(k_fill_bytes, dim3(1), dim3(64), 0, s, static_cast<uint8_t*>(ptr) + words * 4,
                       tail);
    return hipGetLastError();
  }
  return hipSuccess;
}

}  // namespace lbm
