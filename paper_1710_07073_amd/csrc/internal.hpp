// Host-side context and kernel launch entry points shared by the translation units of the
// library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/lbm.h"
#include "graph.hpp"
#include "lattice.hpp"

namespace lbm {
// Host-side step state of a context: which buffers and masks the next launches use.
struct HostState {
  int cur;                // pops[cur] holds the current post-collision state
  int flag_cur;           // current force / velocity tile mask
  bool flag_clean[2];     // tile mask known to be all zero
  int rpar;               // parity of the next overlapped step (its region flags, list, counter)
  bool pending;           // bubbles_step() enqueued the bulk; lbm_step() must update the region
  bool marked;            // the region of the next overlapped step is marked (within lbm_run)
  bool last_overlapped;   // the last liquid step was overlapped (its region list is current)
  int64_t steps;
};
}  // namespace lbm

struct lbm_ctx {
  lbm_desc desc;
  lbm::Geom geom;
  bool general;     // any free-slip or periodic face
  bool periodic;    // any periodic face
  size_t elem;      // 4 or 8
  void* pops[2];    // population buffers; pops[hs.cur] holds the current post-collision state
  void* force;
  void* vel;
  // Two tile masks, one byte per 8^3 tile (force present / velocity needed). bubbles_step()
  // writes mask[flag_cur ^ 1] and makes it current; each liquid step reads mask[flag_cur] and
  // clears the other one for the next bubble step.
  uint8_t* tiles[2];
  // Region of an overlapped step: the rows of tiles near bubbles (a row: 8 y by 8 z cells across
  // the whole x extent, so that the region launch reads long coalesced runs like the bulk), which
  // the liquid step updates only after the bubble kernels; the rest of the lattice (the bulk) is
  // updated while they run. Per step parity, a flag per row (nonzero: in the region), a compact
  // list of the region's rows and its length. The region launch clears the flags it used; the
  // first bubble kernel of a step clears the other parity's counter (its region launch is done).
  uint32_t* region[2];
  uint32_t* region_list[2];
  uint32_t* region_count;  // [2]
  // per-tile bubble lists of the deterministic force spreading: bubbles per tile (zero between
  // steps) and kTileCap list entries per tile
  uint32_t* tcount;
  uint32_t* tlist;
  lbm::HostState hs;
  bool overlap;               // overlap enabled (lbm_set_overlap)
  hipStream_t side;           // null if it could not be created (overlap then unavailable)
  hipEvent_t ev_fork, ev_join;
  // caller's events recorded around the next bulk (or whole-lattice) liquid launch, one-shot
  hipEvent_t t_start, t_end;
  hipEvent_t ta_start, ta_end;  // one-shot events around the next adjoint liquid launch
  // caller's step record the next bubble half fills (lbm_record_next_bubble_half), one-shot
  double* arm_record;
  int32_t pending_nb;  // bubbles of the pending overlapped step
  uint32_t ntiles;
  uint32_t nrows;  // tile rows (y, z tile coordinates)
  double* partials; // moments reduction partials (4 doubles per block); adjoint dL/domega bins
  bool bins_clean;   // the first 64 partials are zero (the adjoint's bins)
  double* result;   // 4 doubles
  int32_t* status;  // kernel error word
  uint32_t nred;    // number of reduction partial slots
  hipStream_t stream;
  int step_vec;      // cells per thread along x in the liquid step (1, 2, 4)
  uint32_t step_bx;  // threads per workgroup along x (the workgroup has 256 threads)
  int32_t step_wgs;  // at most this many liquid-step workgroups per compute unit (0: no cap)
  uint32_t lds_per_cu;  // LDS bytes of one compute unit
  lbm::GraphCache<lbm::HostState> graph;  // captured method steps (lbm_run), with the host state
                                          // their replay leaves
  // device address of the library's own per-bubble workspace on this context's device
  // (bubbles_step_static_work), null if it could not be resolved
  double* static_work;
  // trajectory recording (lbm_record_positions): rows of 3 x nb positions, the device row counter
  double* traj;
  int32_t traj_rows;
  uint32_t* traj_row;
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
  const uint32_t* region;  // region flags of an overlapped step (tiles the spread may force), or null
};

// A single lattice (lbm_ctx). tcount/tlist: the per-tile bubble lists of the deterministic
// spreading (kTileCap entries per tile; a count above kTileCap marks an overflowed list).
struct OneColumn {
  Geom G;
  void* U;
  void* F;
  uint8_t* tiles;
  double nu;
  const uint32_t* region;
  uint32_t* tcount;
  uint32_t* tlist;
  bool lists;  // several bubbles: spread through the per-tile lists
  // exact-time coupling: the current state (post-collision buffer), else null
  const void* state;
  // overlapped steps: the counter k_interp clears (null: none), and where the region of the next
  // step is marked after the bubble update (next_region null: not here)
  uint32_t* clear_count;
  uint32_t* next_region;
  uint32_t* next_list;
  uint32_t* next_count;
  uint32_t nrows;
  template <typename T>
  __device__ ColumnView<T> view(int) const {
    return {G, static_cast<const T*>(U), static_cast<T*>(F), tiles, nu, region};
  }
  // the deterministic spreading: per-tile lists of this lattice (every tile is gathered, so the
  // tiles entered need no note)
  __device__ bool use_lists() const { return lists; }
  // the bubble constants of bubble b: the shared ones
  __device__ bubble_params params(const bubble_params& P, int) const { return P; }
  __device__ uint32_t* tcount_of(int) const { return tcount; }
  __device__ uint32_t* tlist_of(int) const { return tlist; }
  __device__ void note_tile(int, uint32_t) const {}
  __device__ void clear_other_jobs() const {}
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
  // per-tile bubble lists of the deterministic spreading (kTileCap entries per tile)
  uint32_t* tcount;
  uint32_t* tlist;
  float rnx, rny;  // 1 / nx and 1 / ny rounded to float (cell coordinates of the batched step)
  double g, sigma;  // the column's bubbles' gravity and surface tension (0: the shared value)
};

// Many columns: each bubble's column comes from a per-bubble index. The spreading gathers in
// bubble order per tile from each column's lists; the tiles entered in a step are noted as jobs
// (column, tile) for the gather, in a list per step parity (par): each step's first bubble kernel
// empties the other parity's list, which the next step fills.
struct ManyColumns {
  const ColumnDev* cols;
  const int32_t* bubble_col;
  int flag;
  uint32_t* jobs;       // [2][job_cap][2]: (column, tile)
  uint32_t* job_count;  // [2]
  uint32_t job_cap;
  int par;
  template <typename T>
  __device__ ColumnView<T> view(int b) const {
    const ColumnDev& c = cols[bubble_col[b]];
    return {c.G, static_cast<const T*>(c.U), static_cast<T*>(c.F), c.tiles[flag], c.nu, nullptr};
  }
  __device__ bool use_lists() const { return true; }
  // the bubble constants of bubble b: the shared ones with its column's g and sigma where set
  __device__ bubble_params params(const bubble_params& P, int b) const {
    bubble_params q = P;
    const ColumnDev& c = cols[bubble_col[b]];
    if (c.g != 0.0) q.g = c.g;
    if (c.sigma != 0.0) q.sigma = c.sigma;
    return q;
  }
  __device__ uint32_t* tcount_of(int b) const { return cols[bubble_col[b]].tcount; }
  __device__ uint32_t* tlist_of(int b) const { return cols[bubble_col[b]].tlist; }
  // tile t of bubble b's column received its first bubble of the step
  __device__ void note_tile(int b, uint32_t t) const {
    const uint32_t i = atomicAdd(&job_count[par], 1u);
    if (i < job_cap) {
      uint32_t* j = jobs + 2 * ((size_t)par * job_cap + i);
      j[0] = (uint32_t)bubble_col[b];
      j[1] = t;
    }
  }
  __device__ void clear_other_jobs() const { job_count[par ^ 1] = 0u; }
};

constexpr uint32_t kTile = 8;

// Slots of the per-bubble workspace (bubble_soa.work) the bubble kernels pass between them:
// interpolated u_l and curl w_l, position at interpolation, reaction psi, window valid.
constexpr int W_UL = 0, W_WL = 3, W_X0 = 6, W_PSI = 9, W_VALID = 12;
// From W_WGT: the three axes' stencil weights at x0, LBM_MAX_STENCIL + 2 doubles per axis, indexed
// like the LDS copies of the bubble kernels (cell - lo + 1).
constexpr int W_WGT = 16;
static_assert(W_WGT + 3 * (LBM_MAX_STENCIL + 2) <= LBM_BUBBLE_WORK, "bubble workspace too small");
// Step record of one bubble (LBM_BUBBLE_RECORD doubles): the values the adjoint of the bubble half
// needs, with the sub-step velocities and clamp flags of up to kRecordMaxSub sub-steps.
constexpr int R_X = 0, R_UB = 3, R_ULP = 6, R_STATE = 9, R_UL = 10, R_WL = 13, R_PSI = 16,
              R_VALID = 19, R_D = 20, R_SUB = 21, R_UBS = 24, kRecordMaxSub = 32,
              R_CLAMP = R_UBS + 3 * (kRecordMaxSub + 1), R_SIZE = LBM_BUBBLE_RECORD;
static_assert(R_CLAMP + 3 <= R_SIZE, "bubble record too small");
// Bubbles a tile's list holds in the deterministic spreading.
constexpr uint32_t kTileCap = 64;
constexpr uint32_t kRedBlocks = 1024;  // upper bound of moments reduction blocks

enum : int32_t { STATUS_STENCIL_TOO_LARGE = 1, STATUS_REGION_MISS = 2, STATUS_BARRIER_TIMEOUT = 4 };

// A persistent batched launch: nsteps method steps of every column in one kernel (see
// launch_batch_persistent). Step s uses tile mask flag0 ^ (s & 1), reads population buffer
// cur0 ^ (s & 1) and note list parity cur0 ^ (s & 1).
struct PersistArgs {
  const ColumnDev* cols;
  const uint32_t* item_col;
  uint32_t nitems;
  int cur0, flag0, flags, nsteps, faces;
  uint32_t* barrier;    // [0] arrivals, [1] generation, [2] abort; zero at launch
  uint32_t spin_limit;  // polls a workgroup waits at a barrier before it aborts the launch
};

// Cells the region of an overlapped step extends beyond a bubble's stencil window widened by the
// curl ring: covers the bubble's displacement in one step.
constexpr int kRegionMargin = 2;

// Lattices from this size on overlap the bubble kernels with the liquid step by default.
constexpr uint32_t kOverlapMinCells = 1u << 22;

// A valid bubble_params.coupling: known bits and a known reaction.
inline bool coupling_ok(int32_t c) {
  const int32_t known = LBM_REACTION_MASK | LBM_COUPLING_POINT_KERNEL | LBM_COUPLING_EXACT_TIME;
  return (c & ~known) == 0 && (c & LBM_REACTION_MASK) <= LBM_REACTION_NET_FORCE;
}

// Byte offsets of every population (and field) element fit in 32 bits.
inline bool bb_fast_ok(const Geom& G, size_t esz) { return (size_t)19 * G.N * esz <= 0xffffffffull; }

// step.hip
hipError_t launch_step(lbm_ctx* c);
// The liquid step can be split into bulk and region launches (all faces bounce-back, one cell
// per thread, buffers below 4 GiB).
bool can_overlap(const lbm_ctx* c);
// Bulk part of the liquid step of an overlapped step (on the caller's stream).
hipError_t launch_bulk(lbm_ctx* c);
// bubbles.hip
// mark_ahead (overlapped steps of lbm_run only): also mark the region of the next step, after the
// bubble update, on the side stream
hipError_t launch_bubbles(lbm_ctx* c, const bubble_params* p, const bubble_soa* s, int32_t nb,
                          bool overlap, bool mark_ahead);
hipError_t launch_bubbles_batch(const ManyColumns& geo, size_t elem, const bubble_params* p,
                                const bubble_soa* s, int32_t nb, int32_t* status,
                                hipStream_t stream);
// The persistent launch of P.nsteps method steps (bubble half and liquid step of every column).
// wgs_per_cu: workgroups per compute unit (0: as many as fit); *grid receives the workgroups
// launched. The barrier words must be zero (the caller clears them before each launch).
hipError_t launch_batch_persistent(const ManyColumns& geo, size_t elem, const bubble_params* p,
                                   const bubble_soa* s, int32_t nb, int32_t* status,
                                   const PersistArgs& P, int wgs_per_cu, uint32_t* grid,
                                   hipStream_t stream);
// moments.hip
hipError_t launch_moments(lbm_ctx* c, void* rho, void* u, bool sums);
hipError_t launch_populations(lbm_ctx* c, void* out);
hipError_t launch_fill(void* ptr, size_t bytes, hipStream_t s);

inline uint32_t div_up(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

// Default launch shape of the liquid step: whole rows per workgroup where they fit.
// Workgroups per compute unit the liquid-step launches are held to by default: fewer waves in
// flight stream the populations faster (128 x 128 x 512: FP32 method step 228.8 us uncapped,
// 218 us at 4-5; FP64 liquid step 443.8 us at the 4 its registers allow, 417 us at 3).
constexpr int32_t kDefaultStepWgsF32 = 5;
constexpr int32_t kDefaultStepWgsF64 = 3;

// Workgroups per compute unit of the FP32 batched step (64 uneven columns: 1.716 ms uncapped,
// 1.55 ms at 2-3; its 95 VGPRs allow 5).
constexpr int32_t kDefaultBatchWgsF32 = 3;

// Dynamic LDS a launch requests (the step kernels use none) so that at most wgs of its
// workgroups fit on one compute unit with lds_per_cu bytes of LDS; LDS is allocated in 512-byte
// granules, at most 64 KB per workgroup.
inline size_t occupancy_lds(uint32_t lds_per_cu, int32_t wgs) {
  if (wgs <= 0 || lds_per_cu == 0) return 0;
  size_t s = (size_t)lds_per_cu / (size_t)wgs / 512 * 512;
  return s > 65536 ? 65536 : s;
}

inline size_t step_lds(const lbm_ctx* c) { return occupancy_lds(c->lds_per_cu, c->step_wgs); }

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
