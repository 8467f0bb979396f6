// Batched columns: many independent lattices of uneven size and relaxation rate (the paper's
// grid-independence and stability sweeps, Sec. 4.2-4.3) advanced together. One liquid-step launch
// covers every column through a table of work items (contiguous cell ranges of one column); the
// bubbles of all columns go through the same three bubble kernels as a single lattice. Repeated
// steps are captured once into a HIP graph and replayed (graph.hpp).
#include <math.h>

#include <algorithm>
#include <new>
#include <string.h>
#include <vector>

#include "batch_cell.hpp"
#include "collide.hpp"
#include "graph.hpp"

struct lbm_batch {
  int ncols;
  int32_t precision;
  size_t elem;
  bool general;
  int faces;  // FACES_* of the liquid kernel
  int flags;
  std::vector<lbm_column> cols;       // as given
  std::vector<lbm::ColumnDev> host;   // device-side table, host copy
  lbm::ColumnDev* dev;                // device table (scratch)
  std::vector<uint32_t> item_col;     // column of each work item, host copy
  uint32_t* item_col_dev;             // the same (scratch), room for items of 256 cells
  int32_t* bubble_col;                // bubble -> column (scratch)
  int32_t nb_total;
  uint32_t nitems;
  int cur;          // population buffer holding the current state, same for all columns
  int flag_cur;     // current tile mask, same for all columns
  bool flag_clean[2];
  int32_t* status;
  bool persistent;      // method steps as persistent launches (lbm_batch_set_persistent)
  uint32_t* barrier;    // grid-barrier words of the persistent launch
  uint32_t last_grid;   // workgroups of the last persistent launch
  uint32_t* jobs;       // tile jobs of the deterministic spreading, two step parities
  uint32_t* job_count;  // [2]
  uint32_t job_cap;     // tiles of all columns: each is noted at most once per step
  double* partials;
  double* result;
  uint32_t nred;
  hipStream_t stream;
  int64_t steps;
  int32_t step_wgs;     // at most this many liquid-step workgroups per compute unit (0: no cap)
  uint32_t lds_per_cu;  // LDS bytes of one compute unit
  lbm::StepGraph graph;
};

namespace lbm {
namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

constexpr uint32_t kSumBlocks = 16;  // workgroups per column of the per-column sums

// One liquid step of every column: a workgroup per work item.
template <typename T, int FACES>
__global__ __launch_bounds__(256) void k_batch_step(const ColumnDev* __restrict__ cols,
                                                    const uint32_t* __restrict__ item_col,
                                                    uint32_t nitems, int cur, int flag, int flags) {
  // each XCD takes a contiguous range of items (measured faster here than launch order, unlike
  // the single-lattice step)
  batch_item<T, FACES>(cols, item_col, xcd_remap(blockIdx.x, nitems), cur, flag, flags);
}

// Per-column sums (eq. (10)) of the current state: kSumBlocks workgroups per column accumulate
// (sum drho, sum rho u) of their share of the cells in double precision; k_batch_sums_reduce adds
// the shares of each column in a fixed order.
template <typename T, bool GENERAL>
__global__ __launch_bounds__(256) void k_batch_sums(const ColumnDev* __restrict__ cols, int cur,
                                                    double* __restrict__ partials) {
  __shared__ double s_red[4][4];
  const uint32_t col = blockIdx.x / kSumBlocks, part = blockIdx.x % kSumBlocks;
  const ColumnDev& C = cols[col];
  const Geom G = C.G;
  const T* __restrict__ src = static_cast<const T*>(C.pops[cur]);
  double acc[4] = {0, 0, 0, 0};
  for (uint32_t cell = part * 256 + threadIdx.x; cell < G.N; cell += kSumBlocks * 256) {
    const uint32_t x = cell % G.nx, y = (cell / G.nx) % G.ny, z = cell / G.plane;
    const CellNbr nb = cell_neighbours(G, (int)x, (int)y, (int)z);
    T g[19];
    pull_all<GENERAL>(g, src, G, layout_cell(G, cell, z), nb, std::make_integer_sequence<int, 19>{});
#pragma unroll
    for (int q = 0; q < 19; ++q) {
      const double v = (double)g[q];
      acc[0] += v;
      acc[1] += CX[q] * v;
      acc[2] += CY[q] * v;
      acc[3] += CZ[q] * v;
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double v = acc[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) s_red[k][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 4)
    partials[(size_t)blockIdx.x * 4 + threadIdx.x] =
        s_red[threadIdx.x][0] + s_red[threadIdx.x][1] + s_red[threadIdx.x][2] + s_red[threadIdx.x][3];
}

__global__ void k_batch_sums_reduce(const ColumnDev* __restrict__ cols, int ncols,
                                    const double* __restrict__ partials, double* __restrict__ result) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncols) return;
  double s[4] = {0, 0, 0, 0};
  for (uint32_t p = 0; p < kSumBlocks; ++p)
    for (int k = 0; k < 4; ++k) s[k] += partials[((size_t)col * kSumBlocks + p) * 4 + k];
  result[(size_t)col * 4] = (double)cols[col].G.N + s[0];
  for (int k = 1; k < 4; ++k) result[(size_t)col * 4 + k] = s[k];
}

template <typename T, bool GENERAL>
__global__ __launch_bounds__(256) void k_batch_populations(const ColumnDev* __restrict__ col, int cur,
                                                           T* __restrict__ out) {
  const Geom G = col->G;
  const uint32_t cell = blockIdx.x * 256 + threadIdx.x;
  if (cell >= G.N) return;
  const T* __restrict__ src = static_cast<const T*>(col->pops[cur]);
  const uint32_t x = cell % G.nx, y = (cell / G.nx) % G.ny, z = cell / G.plane;
  const CellNbr nb = cell_neighbours(G, (int)x, (int)y, (int)z);
  T g[19];
  pull_all<GENERAL>(g, src, G, layout_cell(G, cell, z), nb, std::make_integer_sequence<int, 19>{});
  // exported in the plain (19, nz, ny, nx) order whatever the buffer layout
#pragma unroll
  for (int q = 0; q < 19; ++q) out[(size_t)q * G.N + cell] = g[q];
}

bool column_ok(const lbm_column& c) {
  if (c.nx < 1 || c.ny < 1 || c.nz < 1 || c.reserved != 0) return false;
  if (!(c.omega > 0.0 && c.omega < 2.0)) return false;
  if (!(c.g >= 0.0 && c.g < INFINITY) || !(c.sigma >= 0.0 && c.sigma < INFINITY)) return false;
  if (c.nb < 0 || c.bubble_begin < 0) return false;
  for (int a = 0; a < 3; ++a) {
    const int lo = c.bc[2 * a], hi = c.bc[2 * a + 1];
    if (lo < 0 || lo > 2 || hi < 0 || hi > 2) return false;
    if ((lo == LBM_BC_PERIODIC) != (hi == LBM_BC_PERIODIC)) return false;
  }
  const double cells = (double)c.nx * c.ny * c.nz;
  return cells * 19.0 < 2147483648.0;
}

struct BatchLayout {
  std::vector<size_t> pops0, pops1, force, vel, tiles0, tiles1, tcount, tlist;
  std::vector<uint32_t> ntiles;
  size_t pool, table, bcol, jobs, job_count, item_col, barrier, partials, result, status, scratch;
  uint32_t total_tiles, max_items;
  int32_t nb_total;
};

bool layout_batch(const lbm_column* cols, int ncols, size_t elem, BatchLayout& L) {
  L.pool = 0;
  size_t tiles = 0;
  L.nb_total = 0;
  for (int c = 0; c < ncols; ++c) {
    const lbm_column& k = cols[c];
    if (!column_ok(k)) return false;
    // columns own consecutive, non-overlapping bubble ranges in column order
    if (k.bubble_begin != L.nb_total) return false;
    L.nb_total += k.nb;
    const size_t n = (size_t)k.nx * k.ny * k.nz;
    L.pops0.push_back(L.pool);
    L.pool = align_up(L.pool + 19 * n * elem);
    L.pops1.push_back(L.pool);
    L.pool = align_up(L.pool + 19 * n * elem);
    L.force.push_back(L.pool);
    L.pool = align_up(L.pool + 3 * n * elem);
    L.vel.push_back(L.pool);
    L.pool = align_up(L.pool + 3 * n * elem);
    const uint32_t nt = div_up(k.nx, kTile) * div_up(k.ny, kTile) * div_up(k.nz, kTile);
    L.ntiles.push_back(nt);
    L.tiles0.push_back(tiles);
    tiles = align_up(tiles + nt);
    L.tiles1.push_back(tiles);
    tiles = align_up(tiles + nt);
  }
  // per-tile bubble lists of each column (counts zero between steps)
  L.total_tiles = 0;
  for (int c = 0; c < ncols; ++c) {
    L.tcount.push_back(tiles);
    tiles = align_up(tiles + (size_t)L.ntiles[c] * sizeof(uint32_t));
    L.tlist.push_back(tiles);
    tiles = align_up(tiles + (size_t)L.ntiles[c] * kTileCap * sizeof(uint32_t));
    L.total_tiles += L.ntiles[c];
  }
  L.jobs = tiles;
  L.job_count = align_up(L.jobs + (size_t)2 * L.total_tiles * 2 * sizeof(uint32_t));
  L.max_items = 0;
  for (int c = 0; c < ncols; ++c)
    L.max_items += div_up((uint32_t)cols[c].nx * cols[c].ny * cols[c].nz, 256u);
  L.item_col = align_up(L.job_count + 2 * sizeof(uint32_t));
  L.barrier = align_up(L.item_col + (size_t)L.max_items * sizeof(uint32_t));
  L.table = align_up(L.barrier + 4 * sizeof(uint32_t));
  L.bcol = align_up(L.table + (size_t)ncols * sizeof(ColumnDev));
  L.partials = align_up(L.bcol + (size_t)(L.nb_total > 0 ? L.nb_total : 1) * sizeof(int32_t));
  const size_t nparts = std::max<size_t>(kRedBlocks, (size_t)ncols * kSumBlocks);
  L.result = align_up(L.partials + nparts * 4 * sizeof(double));
  L.status = align_up(L.result + (size_t)ncols * 4 * sizeof(double));
  L.scratch = align_up(L.status + sizeof(int32_t));
  return true;
}

// One cell per thread, no loop: on the 64-column sweep 256-cell items measured 1.72 ms per step
// against 1.91 (512), 2.25 (1024) and 2.40 (2048); on one 128 x 128 x 512 column 5.9 TB/s
// against 5.5 (1024) and 4.9 (16384).
uint32_t default_item_cells(const lbm_column& c) {
  (void)c;
  return 256;
}

void assign_items(lbm_batch* b) {
  uint32_t item = 0;
  b->item_col.clear();
  for (int c = 0; c < b->ncols; ++c) {
    ColumnDev& D = b->host[c];
    D.item_begin = item;
    D.items = div_up(D.G.N, D.item_cells);
    item += D.items;
    b->item_col.insert(b->item_col.end(), D.items, (uint32_t)c);
  }
  b->nitems = item;
}

hipError_t upload_table(lbm_batch* b) {
  hipError_t e = hipMemcpyAsync(b->dev, b->host.data(), b->host.size() * sizeof(ColumnDev),
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->item_col_dev, b->item_col.data(), b->item_col.size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice, b->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(b->stream);
}

template <typename T, int FACES>
hipError_t batch_step_faces(lbm_batch* b) {
  hipLaunchKernelGGL((k_batch_step<T, FACES>), dim3(b->nitems), dim3(256),
                     occupancy_lds(b->lds_per_cu, b->step_wgs), b->stream, b->dev, b->item_col_dev,
                     b->nitems, b->cur, b->flag_cur, b->flags);
  return hipGetLastError();
}

template <typename T>
hipError_t batch_step_typed(lbm_batch* b) {
  switch (b->faces) {
    case FACES_BB: return batch_step_faces<T, FACES_BB>(b);
    case FACES_WALLS: return batch_step_faces<T, FACES_WALLS>(b);
    default: return batch_step_faces<T, FACES_GENERAL>(b);
  }
}

// One method step of every column: bubble half, then the liquid step.
hipError_t batch_method_step(lbm_batch* b, const bubble_params* p, const bubble_soa* s, int32_t nb) {
  const int m = b->flag_cur ^ 1;
  if (!b->flag_clean[m]) {
    for (int c = 0; c < b->ncols; ++c) {
      const hipError_t e = launch_fill(b->host[c].tiles[m],
                                       (size_t)b->host[c].G.tnx * b->host[c].G.tny *
                                           div_up(b->host[c].G.nz, kTile),
                                       b->stream);
      if (e != hipSuccess) return e;
    }
  }
  b->flag_clean[m] = false;
  b->flag_cur = m;
  ManyColumns geo;
  geo.cols = b->dev;
  geo.bubble_col = b->bubble_col;
  geo.flag = m;
  geo.jobs = b->jobs;
  geo.job_count = b->job_count;
  geo.job_cap = b->job_cap;
  geo.par = b->cur;  // alternates every step, like the tile jobs' lists
  hipError_t e = launch_bubbles_batch(geo, b->elem, p, s, nb, b->status, b->stream);
  if (e != hipSuccess) return e;
  e = b->elem == 4 ? batch_step_typed<float>(b) : batch_step_typed<double>(b);
  if (e != hipSuccess) return e;
  b->cur ^= 1;
  b->flag_clean[b->flag_cur ^ 1] = true;
  ++b->steps;
  return hipSuccess;
}

// Polls of a persistent launch's barrier before it aborts (about a second of waiting).
constexpr uint32_t kBarrierSpinLimit = 1u << 20;

// n method steps of every column as one persistent launch.
hipError_t batch_persistent_steps(lbm_batch* b, const bubble_params* p, const bubble_soa* s,
                                  int32_t nb, int32_t n) {
  if (n <= 0) return hipSuccess;
  const int m0 = b->flag_cur ^ 1;  // tile mask of the first step
  if (!b->flag_clean[m0]) {
    for (int c = 0; c < b->ncols; ++c) {
      const hipError_t e = launch_fill(b->host[c].tiles[m0],
                                       (size_t)b->host[c].G.tnx * b->host[c].G.tny *
                                           div_up(b->host[c].G.nz, kTile),
                                       b->stream);
      if (e != hipSuccess) return e;
    }
  }
  hipError_t e = launch_fill(b->barrier, 4 * sizeof(uint32_t), b->stream);
  if (e != hipSuccess) return e;
  ManyColumns geo;
  geo.cols = b->dev;
  geo.bubble_col = b->bubble_col;
  geo.flag = m0;
  geo.jobs = b->jobs;
  geo.job_count = b->job_count;
  geo.job_cap = b->job_cap;
  geo.par = b->cur;
  PersistArgs P;
  P.cols = b->dev;
  P.item_col = b->item_col_dev;
  P.nitems = b->nitems;
  P.cur0 = b->cur;
  P.flag0 = m0;
  P.flags = b->flags;
  P.nsteps = n;
  P.faces = b->faces;
  P.barrier = b->barrier;
  P.spin_limit = kBarrierSpinLimit;
  e = launch_batch_persistent(geo, b->elem, p, s, nb, b->status, P, b->step_wgs, &b->last_grid,
                              b->stream);
  if (e != hipSuccess) return e;
  for (int32_t i = 0; i < n; ++i) {  // the host step state the n steps leave
    const int m = b->flag_cur ^ 1;
    b->flag_clean[m] = false;
    b->flag_cur = m;
    b->cur ^= 1;
    b->flag_clean[b->flag_cur ^ 1] = true;
    ++b->steps;
  }
  return hipSuccess;
}

lbm_status to_status(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EDEVICE; }

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" {

lbm_status lbm_batch_bytes_required(const lbm_column* cols, int32_t ncols, int32_t precision,
                                    size_t* pool_bytes, size_t* scratch_bytes) {
  if (!cols || ncols < 1) return LBM_EINVAL;
  if (precision != LBM_FP32_SHIFTED && precision != LBM_FP64_SHIFTED) return LBM_EINVAL;
  BatchLayout L;
  if (!layout_batch(cols, ncols, precision == LBM_FP32_SHIFTED ? 4 : 8, L)) return LBM_EINVAL;
  if (pool_bytes) *pool_bytes = L.pool;
  if (scratch_bytes) *scratch_bytes = L.scratch;
  return LBM_OK;
}

lbm_status lbm_batch_init(const lbm_column* cols, int32_t ncols, int32_t precision, int32_t flags,
                          void* pool, void* scratch, void* stream, lbm_batch** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  if (!cols || ncols < 1 || !pool || !scratch) return LBM_EINVAL;
  if (precision != LBM_FP32_SHIFTED && precision != LBM_FP64_SHIFTED) return LBM_EINVAL;
  if (flags & ~(LBM_FLAG_STATIC_FORCE | LBM_FLAG_WRITE_U_ALL | LBM_FLAG_PLAIN_SOA)) return LBM_EINVAL;
  const size_t elem = precision == LBM_FP32_SHIFTED ? 4 : 8;
  BatchLayout L;
  if (!layout_batch(cols, ncols, elem, L)) return LBM_EINVAL;
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return LBM_EDEVICE;
  b->ncols = ncols;
  b->precision = precision;
  b->elem = elem;
  b->flags = flags;
  b->general = false;
  b->faces = FACES_BB;
  b->cols.assign(cols, cols + ncols);
  b->nb_total = L.nb_total;
  b->stream = static_cast<hipStream_t>(stream);
  // FP32: at most kDefaultBatchWgsF32 step workgroups per compute unit (FP64 is held to 3 by its
  // registers)
  b->step_wgs = elem == 4 ? lbm::kDefaultBatchWgsF32 : 0;
  {
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
            hipSuccess)
      lds = 0;
    b->lds_per_cu = lds > 0 ? (uint32_t)lds : 0u;
  }
  b->cur = 0;
  b->flag_cur = 0;
  b->flag_clean[0] = b->flag_clean[1] = true;
  b->steps = 0;
  uint8_t* P = static_cast<uint8_t*>(pool);
  uint8_t* S = static_cast<uint8_t*>(scratch);
  b->dev = reinterpret_cast<ColumnDev*>(S + L.table);
  b->item_col_dev = reinterpret_cast<uint32_t*>(S + L.item_col);
  b->bubble_col = reinterpret_cast<int32_t*>(S + L.bcol);
  b->partials = reinterpret_cast<double*>(S + L.partials);
  b->result = reinterpret_cast<double*>(S + L.result);
  b->status = reinterpret_cast<int32_t*>(S + L.status);
  b->jobs = reinterpret_cast<uint32_t*>(S + L.jobs);
  b->job_count = reinterpret_cast<uint32_t*>(S + L.job_count);
  b->job_cap = L.total_tiles;
  b->persistent = false;
  b->barrier = reinterpret_cast<uint32_t*>(S + L.barrier);
  b->last_grid = 0;
  b->nred = kRedBlocks;
  b->host.resize(ncols);
  std::vector<int32_t> bcol(L.nb_total > 0 ? L.nb_total : 1, 0);
  hipError_t e = launch_fill(pool, L.pool, b->stream);
  if (e == hipSuccess) e = launch_fill(scratch, L.scratch, b->stream);
  for (int c = 0; c < ncols && e == hipSuccess; ++c) {
    const lbm_column& k = cols[c];
    ColumnDev& D = b->host[c];
    memset(&D, 0, sizeof(D));
    D.G.nx = k.nx;
    D.G.ny = k.ny;
    D.G.nz = k.nz;
    D.G.N = (uint32_t)k.nx * k.ny * k.nz;
    D.G.plane = (uint32_t)k.nx * k.ny;
    set_layout(D.G, (flags & LBM_FLAG_PLAIN_SOA) != 0);
    for (int f = 0; f < 6; ++f) {
      D.G.bc[f] = k.bc[f];
      if (k.bc[f] != LBM_BC_BOUNCE_BACK) b->general = true;
      if (k.bc[f] == LBM_BC_FREE_SLIP) b->faces = std::max(b->faces, (int)FACES_WALLS);
      if (k.bc[f] == LBM_BC_PERIODIC) b->faces = FACES_GENERAL;
    }
    // the wall fast path addresses populations by 32-bit byte offsets
    if (!bb_fast_ok(D.G, elem)) b->faces = FACES_GENERAL;
    D.rnx = 1.0f / (float)k.nx;
    D.rny = 1.0f / (float)k.ny;
    D.G.tnx = (int)div_up(k.nx, kTile);
    D.G.tny = (int)div_up(k.ny, kTile);
    D.omega = k.omega;
    D.nu = (1.0 / k.omega - 0.5) / 3.0;  // eq. (9), dx = dt_l = 1
    D.g = k.g;
    D.sigma = k.sigma;
    D.pops[0] = P + L.pops0[c];
    D.pops[1] = P + L.pops1[c];
    D.F = P + L.force[c];
    D.U = P + L.vel[c];
    D.tiles[0] = S + L.tiles0[c];
    D.tiles[1] = S + L.tiles1[c];
    D.tcount = reinterpret_cast<uint32_t*>(S + L.tcount[c]);
    D.tlist = reinterpret_cast<uint32_t*>(S + L.tlist[c]);
    D.item_cells = default_item_cells(k);
    D.bubble_begin = k.bubble_begin;
    D.nb = k.nb;
    for (int i = 0; i < k.nb; ++i) bcol[k.bubble_begin + i] = c;
  }
  if (e == hipSuccess) {
    assign_items(b);
    e = upload_table(b);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->bubble_col, bcol.data(), bcol.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    delete b;
    return LBM_EDEVICE;
  }
  *out = b;
  return LBM_OK;
}

lbm_status lbm_batch_set_items(lbm_batch* b, const int32_t* item_cells) {
  if (!b || !item_cells) return LBM_EINVAL;
  for (int c = 0; c < b->ncols; ++c)
    if (item_cells[c] < 256 || item_cells[c] > (1 << 16) || item_cells[c] % 256) return LBM_EINVAL;
  for (int c = 0; c < b->ncols; ++c) b->host[c].item_cells = (uint32_t)item_cells[c];
  assign_items(b);
  b->graph.reset();
  return to_status(upload_table(b));
}

lbm_status lbm_batch_set_step_occupancy(lbm_batch* b, int32_t workgroups_per_cu) {
  if (!b || workgroups_per_cu < 0 || workgroups_per_cu > 32) return LBM_EINVAL;
  b->step_wgs = workgroups_per_cu;
  b->graph.reset();  // captured launches hold the old setting
  return LBM_OK;
}

lbm_status lbm_batch_get_step_occupancy(lbm_batch* b, int32_t* workgroups_per_cu) {
  if (!b || !workgroups_per_cu) return LBM_EINVAL;
  *workgroups_per_cu = b->step_wgs;
  return LBM_OK;
}

lbm_status lbm_batch_get_items(lbm_batch* b, int32_t* item_cells) {
  if (!b || !item_cells) return LBM_EINVAL;
  for (int c = 0; c < b->ncols; ++c) item_cells[c] = (int32_t)b->host[c].item_cells;
  return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, const bubble_params* p, const bubble_soa* s, int32_t nb,
                          int32_t nsteps) {
  if (!b || !p || !s || nb != b->nb_total || nsteps < 0) return LBM_EINVAL;
  if (nb > 0 && (b->flags & LBM_FLAG_STATIC_FORCE)) return LBM_EINVAL;
  if (p->n_sub < 1 || !lbm::coupling_ok(p->coupling) || !(p->kernel_factor > 0.0) ||
      !(p->sigma > 0.0))
    return LBM_EINVAL;
  if (p->coupling & LBM_COUPLING_EXACT_TIME) return LBM_EUNSUPPORTED;
  if (nb > 0 && (!s->x || !s->y || !s->z || !s->ux || !s->uy || !s->uz || !s->d || !s->ulx ||
                 !s->uly || !s->ulz || !s->state || !s->work))
    return LBM_EINVAL;
  if (b->persistent) return to_status(batch_persistent_steps(b, p, s, nb, nsteps));
  for (int32_t i = 0; i < nsteps; ++i) {
    const hipError_t e = batch_method_step(b, p, s, nb);
    if (e != hipSuccess) return LBM_EDEVICE;
  }
  return LBM_OK;
}

lbm_status lbm_batch_set_persistent(lbm_batch* b, int32_t enable) {
  if (!b) return LBM_EINVAL;
  b->persistent = enable != 0;
  b->graph.reset();  // captured launches hold the other mode
  return LBM_OK;
}

lbm_status lbm_batch_get_persistent(lbm_batch* b, int32_t* enabled, int32_t* grid) {
  if (!b) return LBM_EINVAL;
  if (enabled) *enabled = b->persistent ? 1 : 0;
  if (grid) *grid = (int32_t)b->last_grid;
  return LBM_OK;
}

lbm_status lbm_batch_run(lbm_batch* b, const bubble_params* p, const bubble_soa* s, int32_t nb,
                         int32_t nsteps, int32_t graph_steps) {
  if (!b || !p || !s || nb != b->nb_total || nsteps < 0) return LBM_EINVAL;
  if (graph_steps < 0 || graph_steps % 2) return LBM_EINVAL;
  if (graph_steps == 0 || nsteps < graph_steps || !b->stream)
    return lbm_batch_step(b, p, s, nb, nsteps);
  // validate once through the eager entry point's checks
  const lbm_status st = lbm_batch_step(b, p, s, nb, 0);
  if (st != LBM_OK) return st;
  auto enqueue = [&](int n) -> hipError_t {
    if (b->persistent) return batch_persistent_steps(b, p, s, nb, n);  // one launch
    for (int i = 0; i < n; ++i) {
      const hipError_t e = batch_method_step(b, p, s, nb);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  int32_t done = 0;
  while (nsteps - done >= graph_steps) {
    const uint32_t mode = (b->flag_clean[0] ? 1u : 0u) | (b->flag_clean[1] ? 2u : 0u) |
                          (b->persistent ? 4u : 0u);
    const GraphKey key = GraphKey::of(p, s, nb, b->cur, b->flag_cur, graph_steps, mode);
    const int cur0 = b->cur, flag0 = b->flag_cur;
    const bool clean0[2] = {b->flag_clean[0], b->flag_clean[1]};
    const int64_t steps0 = b->steps;
    bool captured = false;
    hipError_t e = b->graph.ensure(key, b->stream, [&]() { return enqueue(graph_steps); }, &captured);
    // a capture only records the launches (and a failed one ran nothing): rewind the host-side
    // step state, then replay
    b->cur = cur0;
    b->flag_cur = flag0;
    b->flag_clean[0] = clean0[0];
    b->flag_clean[1] = clean0[1];
    b->steps = steps0;
    if (e != hipSuccess) return LBM_EDEVICE;
    e = b->graph.launch(b->stream);
    if (e != hipSuccess) return LBM_EDEVICE;
    for (int i = 0; i < graph_steps; ++i) {  // advance the host state as the steps did
      const int m = b->flag_cur ^ 1;
      b->flag_clean[m] = false;
      b->flag_cur = m;
      b->cur ^= 1;
      b->flag_clean[b->flag_cur ^ 1] = true;
      ++b->steps;
    }
    (void)captured;
    done += graph_steps;
  }
  if (nsteps > done) return lbm_batch_step(b, p, s, nb, nsteps - done);
  return LBM_OK;
}

lbm_status lbm_batch_sums(lbm_batch* b, double* sums) {
  if (!b || !sums) return LBM_EINVAL;
  const uint32_t blocks = (uint32_t)b->ncols * kSumBlocks;
  if (b->elem == 4) {
    if (b->general)
      hipLaunchKernelGGL((k_batch_sums<float, true>), dim3(blocks), dim3(256), 0, b->stream, b->dev,
                         b->cur, b->partials);
    else
      hipLaunchKernelGGL((k_batch_sums<float, false>), dim3(blocks), dim3(256), 0, b->stream, b->dev,
                         b->cur, b->partials);
  } else {
    if (b->general)
      hipLaunchKernelGGL((k_batch_sums<double, true>), dim3(blocks), dim3(256), 0, b->stream, b->dev,
                         b->cur, b->partials);
    else
      hipLaunchKernelGGL((k_batch_sums<double, false>), dim3(blocks), dim3(256), 0, b->stream, b->dev,
                         b->cur, b->partials);
  }
  if (hipGetLastError() != hipSuccess) return LBM_EDEVICE;
  hipLaunchKernelGGL(k_batch_sums_reduce, dim3(div_up((uint32_t)b->ncols, 64)), dim3(64), 0, b->stream,
                     b->dev, b->ncols, b->partials, b->result);
  if (hipGetLastError() != hipSuccess) return LBM_EDEVICE;
  if (hipMemcpyAsync(sums, b->result, (size_t)b->ncols * 4 * sizeof(double), hipMemcpyDeviceToHost,
                     b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return LBM_EDEVICE;
  for (int i = 0; i < 4 * b->ncols; ++i)
    if (!isfinite(sums[i])) return LBM_EDIVERGED;
  return LBM_OK;
}

lbm_status lbm_batch_populations(lbm_batch* b, int32_t col, void* out) {
  if (!b || col < 0 || col >= b->ncols || !out) return LBM_EINVAL;
  const ColumnDev* dc = b->dev + col;
  const uint32_t N = b->host[col].G.N;
  if (b->elem == 4) {
    if (b->general)
      hipLaunchKernelGGL((k_batch_populations<float, true>), dim3(div_up(N, 256)), dim3(256), 0,
                         b->stream, dc, b->cur, static_cast<float*>(out));
    else
      hipLaunchKernelGGL((k_batch_populations<float, false>), dim3(div_up(N, 256)), dim3(256), 0,
                         b->stream, dc, b->cur, static_cast<float*>(out));
  } else {
    if (b->general)
      hipLaunchKernelGGL((k_batch_populations<double, true>), dim3(div_up(N, 256)), dim3(256), 0,
                         b->stream, dc, b->cur, static_cast<double*>(out));
    else
      hipLaunchKernelGGL((k_batch_populations<double, false>), dim3(div_up(N, 256)), dim3(256), 0,
                         b->stream, dc, b->cur, static_cast<double*>(out));
  }
  return to_status(hipGetLastError());
}

lbm_status lbm_batch_column(lbm_batch* b, int32_t col, void** state, void** force, void** vel) {
  if (!b || col < 0 || col >= b->ncols) return LBM_EINVAL;
  if (state) *state = b->host[col].pops[b->cur];
  if (force) *force = b->host[col].F;
  if (vel) *vel = b->host[col].U;
  return LBM_OK;
}

lbm_status lbm_batch_check(lbm_batch* b) {
  if (!b) return LBM_EINVAL;
  int32_t st = 0;
  if (hipMemcpyAsync(&st, b->status, sizeof(st), hipMemcpyDeviceToHost, b->stream) != hipSuccess)
    return LBM_EDEVICE;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return LBM_EDEVICE;
  if (st != 0) {
    if (launch_fill(b->status, 256, b->stream) != hipSuccess) return LBM_EDEVICE;
    // a persistent launch that could not hold all its workgroups resident aborted its steps
    return (st & STATUS_BARRIER_TIMEOUT) ? LBM_EDEVICE : LBM_EINVAL;
  }
  return LBM_OK;
}

lbm_status lbm_batch_destroy(lbm_batch* b) {
  delete b;
  return LBM_OK;
}

}  // extern "C"
