// Host-side context and kernel launch entry points shared by the translation units of the
// library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/lbm.h"
#include "graph.hpp"
#include "lattice.hpp"

struct lbm_ctx {
  lbm_desc desc;
  lbm::Geom geom;
  bool general;     // any free-slip or periodic face
  size_t elem;      // 4 or 8
  void* pops[2];    // population buffers; pops[cur] holds the current post-collision state
  int cur;
  void* force;
  void* vel;
  // Two tile masks, one byte per 8^3 tile (force present / velocity needed). bubbles_step()
  // writes mask[flag_cur ^ 1] and makes it current; each liquid step reads mask[flag_cur] and
  // clears the other one for the next bubble step.
  uint8_t* tiles[2];
  int flag_cur;
  bool flag_clean[2];
  uint32_t ntiles;
  double* partials; // moments reduction partials (4 doubles per block)
  double* result;   // 4 doubles
  int32_t* status;  // kernel error word
  uint32_t nred;    // number of reduction partial slots
  hipStream_t stream;
  int64_t steps;
  int step_vec;      // cells per thread along x in the liquid step (1, 2, 4)
  uint32_t step_bx;  // threads per workgroup along x (the workgroup has 256 threads)
  lbm::StepGraph graph;  // captured method steps (lbm_run)
};

namespace lbm {

// Geometry and fields of the lattice a bubble lives in, as seen by the bubble kernels.
template <typename T>
struct ColumnView {
  Geom G;
  const T* U;
  T* F;
  uint8_t* tiles;
  double nu;
};

// A single lattice (lbm_ctx).
struct OneColumn {
  Geom G;
  void* U;
  void* F;
  uint8_t* tiles;
  double nu;
  template <typename T>
  __device__ ColumnView<T> view(int) const {
    return {G, static_cast<const T*>(U), static_cast<T*>(F), tiles, nu};
  }
};

// One column of a batch, in device memory: geometry, relaxation rate, buffers, and its share of
// the work items of the batched liquid step and of the bubble arrays.
struct ColumnDev {
  Geom G;
  double omega, nu;
  void* pops[2];
  void* F;
  void* U;
  uint8_t* tiles[2];
  uint32_t item_begin;  // first work item of this column
  uint32_t items;       // work items of this column
  uint32_t item_cells;  // cells per work item
  int32_t bubble_begin, nb;
  int32_t pad;
};

// Many columns: each bubble's column comes from a per-bubble index.
struct ManyColumns {
  const ColumnDev* cols;
  const int32_t* bubble_col;
  int flag;
  template <typename T>
  __device__ ColumnView<T> view(int b) const {
    const ColumnDev& c = cols[bubble_col[b]];
    return {c.G, static_cast<const T*>(c.U), static_cast<T*>(c.F), c.tiles[flag], c.nu};
  }
};

constexpr uint32_t kTile = 8;
constexpr uint32_t kRedBlocks = 1024;  // upper bound of moments reduction blocks

enum : int32_t { STATUS_STENCIL_TOO_LARGE = 1 };

// step.hip
hipError_t launch_step(lbm_ctx* c);
// bubbles.hip
hipError_t launch_bubbles(lbm_ctx* c, const bubble_params* p, const bubble_soa* s, int32_t nb);
hipError_t launch_bubbles_batch(const ColumnDev* cols, const int32_t* bubble_col, int flag,
                                size_t elem, const bubble_params* p, const bubble_soa* s,
                                int32_t nb, int32_t* status, hipStream_t stream);
// moments.hip
hipError_t launch_moments(lbm_ctx* c, void* rho, void* u, bool sums);
hipError_t launch_populations(lbm_ctx* c, void* out);
hipError_t launch_fill(void* ptr, size_t bytes, hipStream_t s);

inline uint32_t div_up(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

// Default launch shape of the liquid step: whole rows per workgroup where they fit.
inline void default_launch(int nx, size_t elem, int* vec, uint32_t* bx) {
  (void)elem;
  *vec = 1;
  *bx = 64;
  for (uint32_t b : {256u, 128u}) {
    if ((uint32_t)nx >= b && nx % b == 0) {
      *bx = b;
      break;
    }
  }
}

// Map a hardware workgroup index to a logical one so that the workgroups the dispatcher sends to
// one XCD (index modulo 8) form a contiguous range of the domain: neighbouring rows then share
// that XCD's L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t i, uint32_t n) {
  constexpr uint32_t X = 8;
  const uint32_t q = n / X, r = n % X;
  const uint32_t k = i % X, j = i / X;
  return k * q + (k < r ? k : r) + j;
}

}  // namespace lbm
