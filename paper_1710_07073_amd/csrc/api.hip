// C ABI (include/lbm.h): argument checking, the context, the scratch layout and the launches.
#include <math.h>
#include <algorithm>
#include <mutex>
#include <new>
#include <string.h>
#include <vector>

#include "internal.hpp"

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t tiles[2], region[2], region_list[2], region_count, tcount, tlist, partials, result,
      status, traj_row, total;
  uint32_t ntiles, nred, tnx, tny, tnz;
};

bool desc_ok(const lbm_desc* d) {
  if (!d) return false;
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) return false;
  if (d->precision != LBM_FP32_SHIFTED && d->precision != LBM_FP64_SHIFTED) return false;
  if (!(d->omega > 0.0 && d->omega < 2.0)) return false;
  if (d->flags & ~(LBM_FLAG_STATIC_FORCE | LBM_FLAG_WRITE_U_ALL | LBM_FLAG_PLAIN_SOA)) return false;
  if (d->reserved != 0) return false;
  for (int a = 0; a < 3; ++a) {
    const int lo = d->bc[2 * a], hi = d->bc[2 * a + 1];
    if (lo < 0 || lo > 2 || hi < 0 || hi > 2) return false;
    if ((lo == LBM_BC_PERIODIC) != (hi == LBM_BC_PERIODIC)) return false;
  }
  // cell indices are 32-bit and every population offset q * N + cell must fit in 31 bits
  const double cells = (double)d->nx * d->ny * d->nz;
  if (cells * 19.0 >= 2147483648.0) return false;
  return true;
}

Layout layout_of(const lbm_desc* d) {
  Layout L;
  L.tnx = lbm::div_up(d->nx, lbm::kTile);
  L.tny = lbm::div_up(d->ny, lbm::kTile);
  L.tnz = lbm::div_up(d->nz, lbm::kTile);
  L.ntiles = L.tnx * L.tny * L.tnz;
  const uint32_t cells = (uint32_t)d->nx * d->ny * d->nz;
  L.nred = lbm::div_up(cells, 256);
  if (L.nred > lbm::kRedBlocks) L.nred = lbm::kRedBlocks;
  L.tiles[0] = 0;
  L.tiles[1] = align_up(L.ntiles);
  const size_t nrows = (size_t)L.tny * L.tnz;
  L.region[0] = align_up(L.tiles[1] + L.ntiles);
  L.region[1] = align_up(L.region[0] + nrows * 4);
  L.region_list[0] = align_up(L.region[1] + nrows * 4);
  L.region_list[1] = align_up(L.region_list[0] + nrows * 4);
  L.region_count = align_up(L.region_list[1] + nrows * 4);
  L.tcount = align_up(L.region_count + 2 * sizeof(uint32_t));
  L.tlist = align_up(L.tcount + (size_t)L.ntiles * 4);
  L.partials = align_up(L.tlist + (size_t)L.ntiles * lbm::kTileCap * 4);
  L.result = align_up(L.partials + (size_t)L.nred * 4 * sizeof(double));
  L.status = align_up(L.result + 4 * sizeof(double));
  L.traj_row = align_up(L.status + sizeof(int32_t));
  L.total = align_up(L.traj_row + sizeof(uint32_t));
  return L;
}

lbm_status from_hip(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EDEVICE; }

}  // namespace

// Per-bubble workspace of bubbles_step_static_work(): every GPU the library runs on holds its own
// copy until the process ends. In host code this name is only a handle for the runtime: kernels
// receive the device address that static_work_address() resolves per device, never the name.
static __device__ __align__(256) double scratch[LBM_STATIC_WORK_BUBBLES * LBM_BUBBLE_WORK];

namespace {

constexpr int kMaxDevices = 64;
std::mutex static_work_mu;
double* static_work_ptr[kMaxDevices];  // device address of `scratch` per device, once resolved

// Device address of `scratch` on device dev, which must be the current device; resolved on the
// first call for that device. Null if dev is out of range or the runtime cannot resolve it.
double* static_work_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(static_work_mu);
  if (!static_work_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p)
      static_work_ptr[dev] = static_cast<double*>(p);
  }
  return static_work_ptr[dev];
}

}  // namespace

extern "C" {

lbm_status lbm_bytes_required(const lbm_desc* desc, size_t* pop_buffer_bytes, size_t* field_bytes,
                              size_t* scratch_bytes) {
  if (!desc_ok(desc)) return LBM_EINVAL;
  const size_t cells = (size_t)desc->nx * desc->ny * desc->nz;
  const size_t elem = desc->precision == LBM_FP32_SHIFTED ? 4 : 8;
  if (pop_buffer_bytes) *pop_buffer_bytes = 19 * cells * elem;
  if (field_bytes) *field_bytes = 3 * cells * elem;
  if (scratch_bytes) *scratch_bytes = layout_of(desc).total;
  return LBM_OK;
}

lbm_status lbm_init(const lbm_desc* desc, void* pops_a, void* pops_b, void* force, void* vel,
                    void* scratch, void* stream, lbm_ctx** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  if (!desc_ok(desc) || !pops_a || !pops_b || !force || !vel || !scratch) return LBM_EINVAL;
  if (pops_a == pops_b) return LBM_EINVAL;
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_EDEVICE;
  c->desc = *desc;
  const Layout L = layout_of(desc);
  lbm::Geom& G = c->geom;
  G.nx = desc->nx;
  G.ny = desc->ny;
  G.nz = desc->nz;
  G.N = (uint32_t)desc->nx * desc->ny * desc->nz;
  G.plane = (uint32_t)desc->nx * desc->ny;
  lbm::set_layout(G, (desc->flags & LBM_FLAG_PLAIN_SOA) != 0);
  for (int f = 0; f < 6; ++f) G.bc[f] = desc->bc[f];
  G.tnx = (int)L.tnx;
  G.tny = (int)L.tny;
  c->general = false;
  c->periodic = false;
  for (int f = 0; f < 6; ++f) {
    if (desc->bc[f] != LBM_BC_BOUNCE_BACK) c->general = true;
    if (desc->bc[f] == LBM_BC_PERIODIC) c->periodic = true;
  }
  c->elem = desc->precision == LBM_FP32_SHIFTED ? 4 : 8;
  c->pops[0] = pops_a;
  c->pops[1] = pops_b;
  c->hs = lbm::HostState{};
  c->hs.flag_clean[0] = c->hs.flag_clean[1] = true;
  c->force = force;
  c->vel = vel;
  uint8_t* s = static_cast<uint8_t*>(scratch);
  c->tiles[0] = s + L.tiles[0];
  c->tiles[1] = s + L.tiles[1];
  c->region[0] = reinterpret_cast<uint32_t*>(s + L.region[0]);
  c->region[1] = reinterpret_cast<uint32_t*>(s + L.region[1]);
  c->region_list[0] = reinterpret_cast<uint32_t*>(s + L.region_list[0]);
  c->region_list[1] = reinterpret_cast<uint32_t*>(s + L.region_list[1]);
  c->region_count = reinterpret_cast<uint32_t*>(s + L.region_count);
  c->tcount = reinterpret_cast<uint32_t*>(s + L.tcount);
  c->tlist = reinterpret_cast<uint32_t*>(s + L.tlist);
  c->ntiles = L.ntiles;
  c->nrows = L.tny * L.tnz;
  c->partials = reinterpret_cast<double*>(s + L.partials);
  c->result = reinterpret_cast<double*>(s + L.result);
  c->status = reinterpret_cast<int32_t*>(s + L.status);
  c->traj = nullptr;
  c->traj_rows = 0;
  c->traj_row = reinterpret_cast<uint32_t*>(s + L.traj_row);
  c->nred = L.nred;
  c->bins_clean = false;
  c->stream = static_cast<hipStream_t>(stream);
  lbm::default_launch(G.nx, c->elem, &c->step_vec, &c->step_bx);
  c->step_wgs = c->elem == 4 ? lbm::kDefaultStepWgsF32 : lbm::kDefaultStepWgsF64;
  c->static_work = nullptr;
  {
    int dev = 0, lds = 0;
    const bool have_dev = hipGetDevice(&dev) == hipSuccess;
    if (!have_dev ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
            hipSuccess)
      lds = 0;  // no cap
    c->lds_per_cu = lds > 0 ? (uint32_t)lds : 0u;
    // the context's device is current here: resolve the library's workspace array on it
    if (have_dev) c->static_work = static_work_address(dev);
  }
  // side stream and events of the overlapped step (default priority); without them the step
  // runs on the caller's stream only. The events order kernels of this device only: every kernel
  // dispatch already releases its writes and acquires at its start, so the events carry no
  // system-scope fence of their own (a cache writeback costing about 10 us per event).
  // on by default where the liquid step is long enough to hide the bubble kernels (its fixed cost,
  // the region launch and the two cross-stream waits, is about 35 us per step)
  c->overlap = G.N >= lbm::kOverlapMinCells;
  c->side = nullptr;
  c->ev_fork = c->ev_join = nullptr;
  c->t_start = c->t_end = nullptr;
  c->ta_start = c->ta_end = nullptr;
  c->arm_record = nullptr;
  const unsigned ev_flags = hipEventDisableTiming | hipEventDisableSystemFence;
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) c->side = nullptr;
  if (c->side && (hipEventCreateWithFlags(&c->ev_fork, ev_flags) != hipSuccess ||
                  hipEventCreateWithFlags(&c->ev_join, ev_flags) != hipSuccess)) {
    for (hipEvent_t ev : {c->ev_fork, c->ev_join})
      if (ev) (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(c->side);
    c->side = nullptr;
  }
  const size_t cells = G.N;
  hipError_t e = lbm::launch_fill(pops_a, 19 * cells * c->elem, c->stream);
  if (e == hipSuccess) e = lbm::launch_fill(pops_b, 19 * cells * c->elem, c->stream);
  if (e == hipSuccess) e = lbm::launch_fill(force, 3 * cells * c->elem, c->stream);
  if (e == hipSuccess) e = lbm::launch_fill(vel, 3 * cells * c->elem, c->stream);
  if (e == hipSuccess) e = lbm::launch_fill(scratch, L.total, c->stream);
  if (e != hipSuccess) {
    lbm_destroy(c);
    return LBM_EDEVICE;
  }
  *out = c;
  return LBM_OK;
}

lbm_status lbm_set_stream(lbm_ctx* ctx, void* stream) {
  if (!ctx || ctx->hs.pending) return LBM_EINVAL;
  ctx->stream = static_cast<hipStream_t>(stream);
  return LBM_OK;
}

lbm_status lbm_set_overlap(lbm_ctx* ctx, int32_t enable) {
  if (!ctx || ctx->hs.pending) return LBM_EINVAL;
  ctx->overlap = enable != 0;
  return LBM_OK;
}

lbm_status lbm_time_next_step(lbm_ctx* ctx, void* start, void* end) {
  if (!ctx) return LBM_EINVAL;
  ctx->t_start = static_cast<hipEvent_t>(start);
  ctx->t_end = static_cast<hipEvent_t>(end);
  return LBM_OK;
}

lbm_status lbm_record_positions(lbm_ctx* ctx, double* traj, int32_t rows) {
  if (!ctx || rows < 0 || (traj && rows == 0) || ctx->hs.pending) return LBM_EINVAL;
  ctx->traj = traj;
  ctx->traj_rows = traj ? rows : 0;
  ctx->graph.reset();  // captured bubble kernels hold the previous setting
  if (traj && lbm::launch_fill(ctx->traj_row, sizeof(uint32_t), ctx->stream) != hipSuccess)
    return LBM_EDEVICE;
  return LBM_OK;
}

lbm_status lbm_step_tiles(lbm_ctx* ctx, uint8_t* tiles, int64_t* ntiles) {
  if (!ctx || !ntiles) return LBM_EINVAL;
  *ntiles = (int64_t)ctx->ntiles;
  if (!tiles) return LBM_OK;
  // the mask the last bubble half flagged, which its lbm_step() reads
  return hipMemcpyAsync(tiles, ctx->tiles[ctx->hs.flag_cur], ctx->ntiles, hipMemcpyDeviceToDevice,
                        ctx->stream) == hipSuccess
             ? LBM_OK
             : LBM_EDEVICE;
}

lbm_status lbm_record_next_bubble_half(lbm_ctx* ctx, double* record) {
  if (!ctx) return LBM_EINVAL;
  ctx->arm_record = record;  // null disarms
  return LBM_OK;
}

lbm_status lbm_region_cells(lbm_ctx* ctx, int64_t* cells) {
  if (!ctx || !cells) return LBM_EINVAL;
  *cells = 0;
  if (ctx->hs.pending) return LBM_EINVAL;
  if (!ctx->hs.last_overlapped) return LBM_OK;  // a serial step came after it
  // the list of the last overlapped step stays until the next step of the same parity
  const int r = ctx->hs.rpar ^ 1;
  uint32_t count = 0;
  if (hipMemcpyAsync(&count, ctx->region_count + r, sizeof(count), hipMemcpyDeviceToHost,
                     ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess)
    return LBM_EDEVICE;
  if (count > ctx->nrows) return LBM_EDEVICE;
  std::vector<uint32_t> list(count);
  if (count && (hipMemcpyAsync(list.data(), ctx->region_list[r], count * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
                hipStreamSynchronize(ctx->stream) != hipSuccess))
    return LBM_EDEVICE;
  const lbm::Geom& G = ctx->geom;
  const int kt = (int)lbm::kTile;
  int64_t n = 0;
  for (const uint32_t u : list) {
    if (u >= ctx->nrows) return LBM_EDEVICE;
    const int ty = (int)(u % (uint32_t)G.tny), tz = (int)(u / (uint32_t)G.tny);
    const int64_t ey = std::min(kt, G.ny - ty * kt), ez = std::min(kt, G.nz - tz * kt);
    n += (int64_t)G.nx * ey * ez;
  }
  *cells = n;
  return LBM_OK;
}

lbm_status lbm_get_overlap(lbm_ctx* ctx, int32_t* enabled, int32_t* available) {
  if (!ctx) return LBM_EINVAL;
  if (enabled) *enabled = ctx->overlap ? 1 : 0;
  if (available) *available = lbm::can_overlap(ctx) ? 1 : 0;
  return LBM_OK;
}

lbm_status lbm_set_launch(lbm_ctx* ctx, int32_t vec, int32_t block_x) {
  if (!ctx || ctx->hs.pending) return LBM_EINVAL;
  if (vec != 1 && vec != 2 && vec != 4) return LBM_EINVAL;
  if (block_x != 16 && block_x != 32 && block_x != 64 && block_x != 128 && block_x != 256)
    return LBM_EINVAL;
  if (ctx->desc.nx % vec != 0) return LBM_EINVAL;
  ctx->step_vec = vec;
  ctx->step_bx = (uint32_t)block_x;
  return LBM_OK;
}

lbm_status lbm_set_step_occupancy(lbm_ctx* ctx, int32_t workgroups_per_cu) {
  if (!ctx || ctx->hs.pending) return LBM_EINVAL;
  if (workgroups_per_cu < 0 || workgroups_per_cu > 32) return LBM_EINVAL;
  ctx->step_wgs = workgroups_per_cu;
  return LBM_OK;
}

lbm_status lbm_get_step_occupancy(lbm_ctx* ctx, int32_t* workgroups_per_cu) {
  if (!ctx || !workgroups_per_cu) return LBM_EINVAL;
  *workgroups_per_cu = ctx->step_wgs;
  return LBM_OK;
}

lbm_status lbm_get_launch(lbm_ctx* ctx, int32_t* vec, int32_t* block_x) {
  if (!ctx || !vec || !block_x) return LBM_EINVAL;
  *vec = ctx->step_vec;
  *block_x = (int32_t)ctx->step_bx;
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* ctx, int32_t nsteps) {
  if (!ctx || nsteps < 0) return LBM_EINVAL;
  for (int32_t i = 0; i < nsteps; ++i) {
    const hipError_t e = lbm::launch_step(ctx);
    if (e != hipSuccess) return LBM_EDEVICE;
  }
  return LBM_OK;
}

namespace {
// in_run: a step of lbm_run, where no caller code runs between steps, so that an overlapped step
// may mark the region of the next one while its bulk runs (from the bubble state it leaves).
lbm_status bubble_half(lbm_ctx* ctx, const bubble_params* p, const bubble_soa* s, int32_t nb,
                       bool in_run) {
  if (!ctx || !p || !s || nb < 0) return LBM_EINVAL;
  if (ctx->desc.flags & LBM_FLAG_STATIC_FORCE) return LBM_EINVAL;
  if (p->n_sub < 1 || !lbm::coupling_ok(p->coupling)) return LBM_EINVAL;
  if (!(p->kernel_factor > 0.0) || !(p->sigma > 0.0) || !(p->rho_l > 0.0)) return LBM_EINVAL;
  if (nb > 0) {
    if (!s->x || !s->y || !s->z || !s->ux || !s->uy || !s->uz || !s->d || !s->ulx || !s->uly ||
        !s->ulz || !s->state || !s->work)
      return LBM_EINVAL;
    const bool any_psi = s->psix || s->psiy || s->psiz;
    const bool all_psi = s->psix && s->psiy && s->psiz;
    if (any_psi && !all_psi) return LBM_EINVAL;
  }
  if (ctx->hs.pending) return LBM_EINVAL;  // the previous bubble half still awaits its lbm_step
  // the caller may have moved bubbles since a previous run marked ahead: mark afresh
  if (!in_run) ctx->hs.marked = false;
  const bool overlap = ctx->overlap && nb > 0 && lbm::can_overlap(ctx);
  return from_hip(lbm::launch_bubbles(ctx, p, s, nb, overlap, in_run));
}
}  // namespace

lbm_status bubbles_step(lbm_ctx* ctx, const bubble_params* p, const bubble_soa* s, int32_t nb) {
  return bubble_half(ctx, p, s, nb, false);
}

lbm_status bubbles_step_static_work(lbm_ctx* ctx, const bubble_params* p, const bubble_soa* s,
                                    int32_t nb) {
  if (!ctx || !s || nb < 0 || nb > LBM_STATIC_WORK_BUBBLES) return LBM_EINVAL;
  if (!ctx->static_work) return LBM_EDEVICE;
  bubble_soa w = *s;
  w.work = ctx->static_work;
  return bubble_half(ctx, p, &w, nb, false);
}

lbm_status lbm_check(lbm_ctx* ctx) {
  if (!ctx) return LBM_EINVAL;
  int32_t st = 0;
  if (hipMemcpyAsync(&st, ctx->status, sizeof(st), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess)
    return LBM_EDEVICE;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return LBM_EDEVICE;
  if (st != 0) {
    if (lbm::launch_fill(ctx->status, sizeof(int32_t) * 64, ctx->stream) != hipSuccess)
      return LBM_EDEVICE;
    return (st & lbm::STATUS_STENCIL_TOO_LARGE) ? LBM_EINVAL : LBM_EUNSUPPORTED;
  }
  return LBM_OK;
}

lbm_status moments(lbm_ctx* ctx, void* rho_out, void* u_out, double* sums_out) {
  if (!ctx) return LBM_EINVAL;
  if (lbm::launch_moments(ctx, rho_out, u_out, sums_out != nullptr) != hipSuccess) return LBM_EDEVICE;
  if (!sums_out) return LBM_OK;
  double r[4];
  if (hipMemcpyAsync(r, ctx->result, sizeof(r), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess)
    return LBM_EDEVICE;
  const lbm_status st = lbm_check(ctx);  // synchronises; reports and clears a kernel error
  if (st == LBM_EDEVICE) return st;
  for (int k = 0; k < 4; ++k) sums_out[k] = r[k];
  // a diverged liquid also gives its bubbles non-finite positions (a kernel error): the
  // divergence is the cause and is what gets reported
  for (int k = 0; k < 4; ++k)
    if (!isfinite(r[k])) return LBM_EDIVERGED;
  return st;
}

lbm_status lbm_populations(lbm_ctx* ctx, void* out) {
  if (!ctx || !out) return LBM_EINVAL;
  return from_hip(lbm::launch_populations(ctx, out));
}

lbm_status lbm_bind_buffers(lbm_ctx* ctx, void* state, void* next_state, void* vel) {
  if (!ctx || ctx->hs.pending) return LBM_EINVAL;
  void* cur = state ? state : ctx->pops[ctx->hs.cur];
  void* nxt = next_state ? next_state : ctx->pops[ctx->hs.cur ^ 1];
  if (cur == nxt) return LBM_EINVAL;
  ctx->pops[ctx->hs.cur] = cur;
  ctx->pops[ctx->hs.cur ^ 1] = nxt;
  if (vel) ctx->vel = vel;
  ctx->graph.reset();  // captured launches name the old buffers
  return LBM_OK;
}

lbm_status lbm_state_buffer(lbm_ctx* ctx, void** out) {
  if (!ctx || !out) return LBM_EINVAL;
  *out = ctx->pops[ctx->hs.cur];
  return LBM_OK;
}

lbm_status lbm_checkpoint(lbm_ctx* ctx, void* state_out, void* vel_out) {
  if (!ctx || !state_out || !vel_out || ctx->hs.pending) return LBM_EINVAL;
  const size_t n = (size_t)ctx->geom.N * ctx->elem;
  hipError_t e = hipMemcpyAsync(state_out, ctx->pops[ctx->hs.cur], 19 * n, hipMemcpyDeviceToDevice,
                                ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(vel_out, ctx->vel, 3 * n, hipMemcpyDeviceToDevice, ctx->stream);
  return e == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_restore(lbm_ctx* ctx, const void* state, const void* vel) {
  if (!ctx || !state || !vel || ctx->hs.pending) return LBM_EINVAL;
  const size_t n = (size_t)ctx->geom.N * ctx->elem;
  hipError_t e = hipMemcpyAsync(ctx->pops[ctx->hs.cur], state, 19 * n, hipMemcpyDeviceToDevice,
                                ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->vel, vel, 3 * n, hipMemcpyDeviceToDevice, ctx->stream);
  // the next overlapped step marks its region from the bubbles it is given
  ctx->hs.marked = false;
  return e == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_run(lbm_ctx* ctx, const bubble_params* p, const bubble_soa* s, int32_t nb,
                   int32_t nsteps, int32_t graph_steps) {
  if (!ctx || !p || !s || nb < 0 || nsteps < 0) return LBM_EINVAL;
  if (graph_steps < 0 || graph_steps % 2 || ctx->hs.pending) return LBM_EINVAL;
  // an armed step record belongs to one call of bubbles_step (a graph would replay it)
  if (ctx->arm_record) return LBM_EINVAL;
  ctx->hs.marked = false;  // the bubble state may have changed since the last call
  auto one = [&]() -> lbm_status {
    lbm_status st = bubble_half(ctx, p, s, nb, true);
    if (st != LBM_OK) return st;
    return lbm_step(ctx, 1);
  };
  if (graph_steps == 0 || nsteps < graph_steps || !ctx->stream) {
    for (int32_t i = 0; i < nsteps; ++i) {
      const lbm_status st = one();
      if (st != LBM_OK) return st;
    }
    return LBM_OK;
  }
  int32_t done = 0;
  while (nsteps - done >= graph_steps) {
    // the captured launches depend on the host step state (buffer and mask parities, which
    // masks are clean, overlap): the key holds all of it, and the state after the captured
    // steps is recorded with the graph
    const lbm::HostState pre = ctx->hs;
    const uint32_t mode = (pre.flag_clean[0] ? 1u : 0u) | (pre.flag_clean[1] ? 2u : 0u) |
                          ((uint32_t)pre.rpar << 4) | (ctx->overlap ? 32u : 0u) |
                          (pre.marked ? 64u : 0u) |
                          ((uint32_t)ctx->step_vec << 8) | (ctx->step_bx << 12) |
                          ((uint32_t)ctx->step_wgs << 24);
    const lbm::GraphKey key = lbm::GraphKey::of(p, s, nb, pre.cur, pre.flag_cur, graph_steps, mode);
    lbm_status st_cap = LBM_OK;
    bool captured = false;
    hipError_t e = ctx->graph.ensure(key, ctx->stream,
                                     [&]() -> hipError_t {
                                       for (int i = 0; i < graph_steps; ++i) {
                                         st_cap = one();
                                         if (st_cap != LBM_OK) return hipErrorInvalidValue;
                                       }
                                       return hipSuccess;
                                     },
                                     &captured);
    if (st_cap != LBM_OK || e != hipSuccess) {
      ctx->hs = pre;  // a failed capture ran nothing: back to the state before it
      return st_cap != LBM_OK ? st_cap : LBM_EDEVICE;
    }
    if (captured) ctx->graph.post() = ctx->hs;  // the capture only recorded the launches
    if (ctx->graph.launch(ctx->stream) != hipSuccess) return LBM_EDEVICE;
    ctx->hs = ctx->graph.post();
    ctx->hs.steps = pre.steps + graph_steps;
    done += graph_steps;
  }
  for (int32_t i = done; i < nsteps; ++i) {
    const lbm_status st = one();
    if (st != LBM_OK) return st;
  }
  return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx* ctx) {
  if (!ctx) return LBM_OK;
  lbm_status st = LBM_OK;
  if (ctx->side) {
    // a bulk launch may still be running (bubbles_step without its lbm_step)
    if (hipStreamSynchronize(ctx->side) != hipSuccess) st = LBM_EDEVICE;
    (void)hipEventDestroy(ctx->ev_fork);
    (void)hipEventDestroy(ctx->ev_join);
    (void)hipStreamDestroy(ctx->side);
  }
  delete ctx;
  return st;
}

const char* lbm_status_string(lbm_status status) {
  switch (status) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_EUNSUPPORTED: return "unsupported";
    case LBM_EDEVICE: return "device error";
    case LBM_EDIVERGED: return "diverged (non-finite sums)";
  }
  return "unknown status";
}

}  // extern "C"
