"""ctypes binding of the C ABI in ``include/lbm.h`` (same names, argument marshalling only).

Every step of the method runs in the HIP kernels of ``_lib/liblbm.so``; this module converts
Python arguments to C structs and pointers and raises on error codes. Loading fails loudly when
the library has not been built. PyTorch is used only by :mod:`.sim` for device memory and
streams.
"""
from __future__ import annotations

import ctypes as ct
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_EUNSUPPORTED, LBM_EDEVICE, LBM_EDIVERGED = 0, -1, -2, -3, -4
LBM_FP32_SHIFTED, LBM_FP64_SHIFTED = 1, 2
LBM_BC_BOUNCE_BACK, LBM_BC_FREE_SLIP, LBM_BC_PERIODIC = 0, 1, 2
LBM_FLAG_STATIC_FORCE, LBM_FLAG_WRITE_U_ALL, LBM_FLAG_PLAIN_SOA = 1, 2, 4
LBM_MAX_STENCIL = 64
LBM_BUBBLE_WORK = 216
LBM_BUBBLE_RECORD = 128
LBM_BUBBLE_ADJ = 12
LBM_STATIC_WORK_BUBBLES = 1024
# coupling variants (bubble_params.coupling)
LBM_REACTION_MASK, LBM_REACTION_SUBSTEP_MEAN, LBM_REACTION_NET_FORCE = 3, 1, 2
LBM_COUPLING_POINT_KERNEL, LBM_COUPLING_EXACT_TIME = 4, 8

# every symbol include/lbm.h declares
EXPORTS = ("lbm_bytes_required", "lbm_init", "lbm_set_stream", "lbm_set_launch", "lbm_get_launch",
           "lbm_set_step_occupancy", "lbm_get_step_occupancy",
           "lbm_set_overlap", "lbm_get_overlap", "lbm_time_next_step", "lbm_time_next_adjoint_liquid",
           "lbm_region_cells",
           "lbm_step", "bubbles_step", "bubbles_step_static_work",
           "moments", "lbm_populations", "lbm_state_buffer", "lbm_check", "lbm_run", "lbm_destroy",
           "lbm_status_string",
           "lbm_batch_bytes_required", "lbm_batch_init", "lbm_batch_set_items", "lbm_batch_get_items",
           "lbm_batch_set_step_occupancy", "lbm_batch_get_step_occupancy",
           "lbm_batch_set_persistent", "lbm_batch_get_persistent",
           "lbm_batch_step", "lbm_batch_run", "lbm_batch_populations", "lbm_batch_sums",
           "lbm_batch_column",
           "lbm_batch_check", "lbm_batch_destroy",
           "lbm_checkpoint", "lbm_restore",
           "lbm_adjoint_liquid", "lbm_adjoint_liquid_tiles", "lbm_step_tiles",
           "lbm_adjoint_bubbles", "lbm_bubble_record",
           "lbm_record_next_bubble_half", "lbm_record_positions", "lbm_bind_buffers",
           "lbm_host_collide",
           "lbm_host_axis_weights", "lbm_host_bubble_ode", "lbm_host_bubble_ode_adjoint")


class LbmDesc(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32),
                ("precision", ct.c_int32), ("omega", ct.c_double), ("bc", ct.c_int32 * 6),
                ("flags", ct.c_int32), ("reserved", ct.c_int32)]


class BubbleParams(ct.Structure):
    _fields_ = [("g", ct.c_double), ("rho_l", ct.c_double), ("rho_b", ct.c_double),
                ("sigma", ct.c_double), ("c_a", ct.c_double), ("drag_scale", ct.c_double),
                ("lift_scale", ct.c_double), ("kernel_factor", ct.c_double), ("cd_k", ct.c_double),
                ("lift_f0", ct.c_double), ("n_sub", ct.c_int32), ("coupling", ct.c_int32)]


class BubbleSoA(ct.Structure):
    _fields_ = [(n, ct.c_void_p) for n in ("x", "y", "z", "ux", "uy", "uz", "d", "ulx", "uly", "ulz",
                                          "state", "psix", "psiy", "psiz", "work")]


class LbmColumn(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32),
                ("bubble_begin", ct.c_int32), ("nb", ct.c_int32), ("bc", ct.c_int32 * 6),
                ("reserved", ct.c_int32), ("omega", ct.c_double), ("g", ct.c_double),
                ("sigma", ct.c_double)]


class LbmError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {lbm_status_string(code)} ({code})")
        self.code = code


_lib = None


def lib():
    """Load the HIP library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} missing "
                              "(run __graft_entry__.build() or paper_1710_07073_amd/build.py)")
        L = ct.CDLL(LIB_PATH)
        P = ct.c_void_p
        L.lbm_bytes_required.argtypes = [ct.POINTER(LbmDesc), ct.POINTER(ct.c_size_t),
                                         ct.POINTER(ct.c_size_t), ct.POINTER(ct.c_size_t)]
        L.lbm_init.argtypes = [ct.POINTER(LbmDesc), P, P, P, P, P, P, ct.POINTER(P)]
        L.lbm_set_stream.argtypes = [P, P]
        L.lbm_set_launch.argtypes = [P, ct.c_int32, ct.c_int32]
        L.lbm_get_launch.argtypes = [P, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32)]
        L.lbm_set_step_occupancy.argtypes = [P, ct.c_int32]
        L.lbm_get_step_occupancy.argtypes = [P, ct.POINTER(ct.c_int32)]
        L.lbm_set_overlap.argtypes = [P, ct.c_int32]
        L.lbm_time_next_step.argtypes = [P, P, P]
        L.lbm_time_next_adjoint_liquid.argtypes = [P, P, P]
        L.lbm_region_cells.argtypes = [P, ct.POINTER(ct.c_int64)]
        L.lbm_get_overlap.argtypes = [P, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32)]
        L.lbm_step.argtypes = [P, ct.c_int32]
        L.bubbles_step.argtypes = [P, ct.POINTER(BubbleParams), ct.POINTER(BubbleSoA), ct.c_int32]
        L.bubbles_step_static_work.argtypes = [P, ct.POINTER(BubbleParams), ct.POINTER(BubbleSoA),
                                               ct.c_int32]
        L.moments.argtypes = [P, P, P, ct.POINTER(ct.c_double)]
        L.lbm_populations.argtypes = [P, P]
        L.lbm_state_buffer.argtypes = [P, ct.POINTER(P)]
        L.lbm_check.argtypes = [P]
        L.lbm_run.argtypes = [P, ct.POINTER(BubbleParams), ct.POINTER(BubbleSoA), ct.c_int32,
                              ct.c_int32, ct.c_int32]
        L.lbm_destroy.argtypes = [P]
        CP = ct.POINTER(LbmColumn)
        L.lbm_batch_bytes_required.argtypes = [CP, ct.c_int32, ct.c_int32, ct.POINTER(ct.c_size_t),
                                               ct.POINTER(ct.c_size_t)]
        L.lbm_batch_init.argtypes = [CP, ct.c_int32, ct.c_int32, ct.c_int32, P, P, P,
                                     ct.POINTER(P)]
        L.lbm_batch_set_items.argtypes = [P, ct.POINTER(ct.c_int32)]
        L.lbm_batch_get_items.argtypes = [P, ct.POINTER(ct.c_int32)]
        L.lbm_batch_set_step_occupancy.argtypes = [P, ct.c_int32]
        L.lbm_batch_get_step_occupancy.argtypes = [P, ct.POINTER(ct.c_int32)]
        L.lbm_batch_set_persistent.argtypes = [P, ct.c_int32]
        L.lbm_batch_get_persistent.argtypes = [P, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32)]
        L.lbm_batch_step.argtypes = [P, ct.POINTER(BubbleParams), ct.POINTER(BubbleSoA), ct.c_int32,
                                     ct.c_int32]
        L.lbm_batch_run.argtypes = [P, ct.POINTER(BubbleParams), ct.POINTER(BubbleSoA), ct.c_int32,
                                    ct.c_int32, ct.c_int32]
        L.lbm_batch_populations.argtypes = [P, ct.c_int32, P]
        L.lbm_batch_sums.argtypes = [P, ct.POINTER(ct.c_double)]
        L.lbm_batch_column.argtypes = [P, ct.c_int32, ct.POINTER(P), ct.POINTER(P), ct.POINTER(P)]
        L.lbm_batch_check.argtypes = [P]
        L.lbm_batch_destroy.argtypes = [P]
        D = ct.POINTER(ct.c_double)
        I = ct.POINTER(ct.c_int32)
        L.lbm_adjoint_liquid.argtypes = [P, P, P, P, P, P, P, P]
        L.lbm_adjoint_liquid_tiles.argtypes = [P, P, P, P, P, P, P, P, P]
        L.lbm_step_tiles.argtypes = [P, P, ct.POINTER(ct.c_int64)]
        L.lbm_checkpoint.argtypes = [P, P, P]
        L.lbm_restore.argtypes = [P, P, P]
        L.lbm_adjoint_bubbles.argtypes = [P, ct.POINTER(BubbleParams), P, P, P, P, P, P, ct.c_int32, P]
        L.lbm_bubble_record.argtypes = [P, ct.POINTER(BubbleSoA), ct.c_int32, ct.c_int32, P]
        L.lbm_record_next_bubble_half.argtypes = [P, P]
        L.lbm_record_positions.argtypes = [P, P, ct.c_int32]
        L.lbm_bind_buffers.argtypes = [P, P, P, P]
        L.lbm_host_collide.argtypes = [D, D, ct.c_double, D, D, D, D, D, D, D]
        L.lbm_host_axis_weights.argtypes = [ct.c_double, ct.c_double, ct.c_int32, ct.c_int32,
                                            ct.c_double, ct.c_double, I, D, D, D, D]
        L.lbm_host_bubble_ode.argtypes = [ct.POINTER(BubbleParams), ct.c_double, ct.c_double, D, D, D,
                                          D, D, I, I, D, D, D]
        L.lbm_host_bubble_ode_adjoint.argtypes = [ct.POINTER(BubbleParams), ct.c_double, ct.c_double,
                                                  D, D, D, D, D, I, I, D, D, D, D]
        L.lbm_status_string.argtypes = [ct.c_int]
        L.lbm_status_string.restype = ct.c_char_p
        for name in EXPORTS:
            if name != "lbm_status_string":
                getattr(L, name).restype = ct.c_int
        _lib = L
    return _lib


def lbm_status_string(code):
    return lib().lbm_status_string(int(code)).decode()


def _ok(code, what):
    if code != LBM_OK:
        raise LbmError(code, what)


def make_desc(shape, omega, precision, bc=(0,) * 6, flags=0):
    nx, ny, nz = shape
    return LbmDesc(int(nx), int(ny), int(nz), int(precision), float(omega),
                   (ct.c_int32 * 6)(*[int(b) for b in bc]), int(flags), 0)


def lbm_bytes_required(desc):
    a, b, c = ct.c_size_t(), ct.c_size_t(), ct.c_size_t()
    _ok(lib().lbm_bytes_required(ct.byref(desc), ct.byref(a), ct.byref(b), ct.byref(c)),
        "lbm_bytes_required")
    return a.value, b.value, c.value


def lbm_init(desc, pops_a, pops_b, force, vel, scratch, stream):
    ctx = ct.c_void_p()
    _ok(lib().lbm_init(ct.byref(desc), pops_a, pops_b, force, vel, scratch, stream,
                       ct.byref(ctx)), "lbm_init")
    return ctx


def lbm_set_stream(ctx, stream):
    _ok(lib().lbm_set_stream(ctx, stream), "lbm_set_stream")


def lbm_set_launch(ctx, vec, block_x):
    _ok(lib().lbm_set_launch(ctx, int(vec), int(block_x)), "lbm_set_launch")


def lbm_set_step_occupancy(ctx, workgroups_per_cu):
    _ok(lib().lbm_set_step_occupancy(ctx, int(workgroups_per_cu)), "lbm_set_step_occupancy")


def lbm_get_step_occupancy(ctx):
    w = ct.c_int32()
    _ok(lib().lbm_get_step_occupancy(ctx, ct.byref(w)), "lbm_get_step_occupancy")
    return w.value


def lbm_get_launch(ctx):
    v, b = ct.c_int32(), ct.c_int32()
    _ok(lib().lbm_get_launch(ctx, ct.byref(v), ct.byref(b)), "lbm_get_launch")
    return v.value, b.value


def lbm_set_overlap(ctx, enable):
    _ok(lib().lbm_set_overlap(ctx, 1 if enable else 0), "lbm_set_overlap")


def lbm_get_overlap(ctx):
    """(enabled, available)"""
    e, a = ct.c_int32(), ct.c_int32()
    _ok(lib().lbm_get_overlap(ctx, ct.byref(e), ct.byref(a)), "lbm_get_overlap")
    return bool(e.value), bool(a.value)


def lbm_time_next_step(ctx, start, end):
    """start, end: torch.cuda.Event objects (already recorded once, so that they exist) or None."""
    h = lambda e: None if e is None else ct.c_void_p(e.cuda_event)
    _ok(lib().lbm_time_next_step(ctx, h(start), h(end)), "lbm_time_next_step")


def lbm_time_next_adjoint_liquid(ctx, start, end):
    """start, end: torch.cuda.Event objects (already recorded once, so that they exist) or None."""
    h = lambda e: None if e is None else ct.c_void_p(e.cuda_event)
    _ok(lib().lbm_time_next_adjoint_liquid(ctx, h(start), h(end)), "lbm_time_next_adjoint_liquid")


def lbm_region_cells(ctx):
    n = ct.c_int64()
    _ok(lib().lbm_region_cells(ctx, ct.byref(n)), "lbm_region_cells")
    return n.value


def lbm_step(ctx, nsteps=1):
    _ok(lib().lbm_step(ctx, int(nsteps)), "lbm_step")


def bubbles_step(ctx, params, soa, nb):
    _ok(lib().bubbles_step(ctx, ct.byref(params), ct.byref(soa), int(nb)), "bubbles_step")


def bubbles_step_static_work(ctx, params, soa, nb):
    _ok(lib().bubbles_step_static_work(ctx, ct.byref(params), ct.byref(soa), int(nb)),
        "bubbles_step_static_work")


def moments(ctx, rho_ptr=None, u_ptr=None, want_sums=True):
    sums = (ct.c_double * 4)() if want_sums else None
    _ok(lib().moments(ctx, rho_ptr, u_ptr, sums), "moments")
    return list(sums) if want_sums else None


def lbm_populations(ctx, out_ptr):
    _ok(lib().lbm_populations(ctx, out_ptr), "lbm_populations")


def lbm_state_buffer(ctx):
    p = ct.c_void_p()
    _ok(lib().lbm_state_buffer(ctx, ct.byref(p)), "lbm_state_buffer")
    return p.value


def lbm_check(ctx):
    _ok(lib().lbm_check(ctx), "lbm_check")


def lbm_destroy(ctx):
    if ctx:
        lib().lbm_destroy(ctx)


def lbm_run(ctx, params, soa, nb, nsteps, graph_steps=0):
    _ok(lib().lbm_run(ctx, ct.byref(params), ct.byref(soa), int(nb), int(nsteps), int(graph_steps)),
        "lbm_run")


# ---- batched columns ----
def make_columns(specs):
    """specs: iterable of (shape, omega, bc, nb[, g, sigma]); bubble ranges are assigned
    consecutively; g, sigma (0 or absent: the batch's bubble_params values) per column."""
    specs = list(specs)
    arr = (LbmColumn * len(specs))()
    begin = 0
    for i, spec in enumerate(specs):
        shape, omega, bc, nb = spec[:4]
        g, sigma = (tuple(spec[4:6]) + (0.0, 0.0))[:2]
        nx, ny, nz = shape
        arr[i] = LbmColumn(int(nx), int(ny), int(nz), begin, int(nb),
                           (ct.c_int32 * 6)(*[int(b) for b in bc]), 0, float(omega), float(g or 0.0),
                           float(sigma or 0.0))
        begin += int(nb)
    return arr


def lbm_batch_bytes_required(cols, precision):
    a, b = ct.c_size_t(), ct.c_size_t()
    _ok(lib().lbm_batch_bytes_required(cols, len(cols), int(precision), ct.byref(a), ct.byref(b)),
        "lbm_batch_bytes_required")
    return a.value, b.value


def lbm_batch_init(cols, precision, flags, pool, scratch, stream):
    h = ct.c_void_p()
    _ok(lib().lbm_batch_init(cols, len(cols), int(precision), int(flags), pool, scratch, stream,
                             ct.byref(h)), "lbm_batch_init")
    return h


def lbm_batch_set_items(batch, item_cells):
    arr = (ct.c_int32 * len(item_cells))(*[int(v) for v in item_cells])
    _ok(lib().lbm_batch_set_items(batch, arr), "lbm_batch_set_items")


def lbm_batch_set_step_occupancy(batch, workgroups_per_cu):
    _ok(lib().lbm_batch_set_step_occupancy(batch, int(workgroups_per_cu)), "lbm_batch_set_step_occupancy")


def lbm_batch_get_step_occupancy(batch):
    w = ct.c_int32()
    _ok(lib().lbm_batch_get_step_occupancy(batch, ct.byref(w)), "lbm_batch_get_step_occupancy")
    return w.value


def lbm_batch_get_items(batch, ncols):
    arr = (ct.c_int32 * ncols)()
    _ok(lib().lbm_batch_get_items(batch, arr), "lbm_batch_get_items")
    return list(arr)


def lbm_batch_step(batch, params, soa, nb, nsteps=1):
    _ok(lib().lbm_batch_step(batch, ct.byref(params), ct.byref(soa), int(nb), int(nsteps)),
        "lbm_batch_step")


def lbm_batch_run(batch, params, soa, nb, nsteps, graph_steps=0):
    _ok(lib().lbm_batch_run(batch, ct.byref(params), ct.byref(soa), int(nb), int(nsteps),
                            int(graph_steps)), "lbm_batch_run")


def lbm_batch_populations(batch, col, out_ptr):
    _ok(lib().lbm_batch_populations(batch, int(col), out_ptr), "lbm_batch_populations")


def lbm_batch_set_persistent(batch, enable):
    _ok(lib().lbm_batch_set_persistent(batch, 1 if enable else 0), "lbm_batch_set_persistent")


def lbm_batch_get_persistent(batch):
    """(enabled, workgroups of the last persistent launch)"""
    e, g = ct.c_int32(), ct.c_int32()
    _ok(lib().lbm_batch_get_persistent(batch, ct.byref(e), ct.byref(g)), "lbm_batch_get_persistent")
    return bool(e.value), g.value


def lbm_batch_sums(batch, ncols):
    """Per-column (sum rho, sum rho u) as a (ncols, 4) array and whether any column diverged
    (non-finite sums, LBM_EDIVERGED); other errors raise."""
    import numpy as np
    out = (ct.c_double * (4 * ncols))()
    rc = lib().lbm_batch_sums(batch, out)
    if rc not in (LBM_OK, LBM_EDIVERGED):
        _ok(rc, "lbm_batch_sums")
    return np.array(out[:], dtype=np.float64).reshape(ncols, 4), rc == LBM_EDIVERGED


def lbm_batch_column(batch, col):
    a, b, c = ct.c_void_p(), ct.c_void_p(), ct.c_void_p()
    _ok(lib().lbm_batch_column(batch, int(col), ct.byref(a), ct.byref(b), ct.byref(c)),
        "lbm_batch_column")
    return a.value, b.value, c.value


def lbm_batch_check(batch):
    _ok(lib().lbm_batch_check(batch), "lbm_batch_check")


def lbm_batch_destroy(batch):
    if batch:
        lib().lbm_batch_destroy(batch)


# ---- adjoint ----
def lbm_adjoint_liquid(ctx, state, force, lam_next, lam_prev, lam_u, lam_f, grad):
    _ok(lib().lbm_adjoint_liquid(ctx, state, force, lam_next, lam_prev, lam_u, lam_f, grad),
        "lbm_adjoint_liquid")


def lbm_adjoint_liquid_tiles(ctx, state, force, lam_next, lam_prev, lam_u, lam_f, tiles, grad):
    _ok(lib().lbm_adjoint_liquid_tiles(ctx, state, force, lam_next, lam_prev, lam_u, lam_f, tiles,
                                       grad), "lbm_adjoint_liquid_tiles")


def lbm_checkpoint(ctx, state_out, vel_out):
    _ok(lib().lbm_checkpoint(ctx, state_out, vel_out), "lbm_checkpoint")


def lbm_restore(ctx, state, vel):
    _ok(lib().lbm_restore(ctx, state, vel), "lbm_restore")


def lbm_step_tiles(ctx, tiles=None):
    """Number of tiles; with a device pointer, also copies the step's tile mask there."""
    n = ct.c_int64()
    _ok(lib().lbm_step_tiles(ctx, tiles, ct.byref(n)), "lbm_step_tiles")
    return n.value


def lbm_adjoint_bubbles(ctx, params, record, vel_prev, lam_f, lam_u, lam, lam_x, nb, grad):
    _ok(lib().lbm_adjoint_bubbles(ctx, ct.byref(params), record, vel_prev, lam_f, lam_u, lam,
                                  lam_x, int(nb), grad), "lbm_adjoint_bubbles")


def lbm_bubble_record(ctx, soa, nb, stage, record):
    _ok(lib().lbm_bubble_record(ctx, ct.byref(soa), int(nb), int(stage), record), "lbm_bubble_record")


def lbm_record_next_bubble_half(ctx, record):
    _ok(lib().lbm_record_next_bubble_half(ctx, record), "lbm_record_next_bubble_half")


def lbm_record_positions(ctx, traj_ptr, rows):
    _ok(lib().lbm_record_positions(ctx, traj_ptr, int(rows)), "lbm_record_positions")


def lbm_bind_buffers(ctx, state=None, next_state=None, vel=None):
    """Device pointers (ctypes c_void_p or None to keep the current buffer)."""
    _ok(lib().lbm_bind_buffers(ctx, state, next_state, vel), "lbm_bind_buffers")


def _dp(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ct.POINTER(ct.c_double))


def host_collide(p, F, omega, lam=None, lam_u=None):
    """Host evaluation of one cell's collision (and its transposed Jacobian if lam is given)."""
    import numpy as np
    p, pp = _dp(p)
    F, Fp = _dp(F)
    out = np.zeros(19)
    u = np.zeros(3)
    mu = np.zeros(19)
    lf = np.zeros(3)
    dom = np.zeros(1)
    if lam is None:
        _ok(lib().lbm_host_collide(pp, Fp, float(omega), None, None, _dp(out)[1], _dp(u)[1], None,
                                   None, None), "lbm_host_collide")
        return out, u
    lam, lp = _dp(lam)
    lam_u, lup = _dp(lam_u)
    _ok(lib().lbm_host_collide(pp, Fp, float(omega), lp, lup, out.ctypes.data_as(ct.POINTER(ct.c_double)),
                               u.ctypes.data_as(ct.POINTER(ct.c_double)),
                               mu.ctypes.data_as(ct.POINTER(ct.c_double)),
                               lf.ctypes.data_as(ct.POINTER(ct.c_double)),
                               dom.ctypes.data_as(ct.POINTER(ct.c_double))), "lbm_host_collide")
    return out, u, mu, lf, float(dom[0])


def host_axis_weights(x, n, ext, periodic=False, s_lo=-1.0, s_hi=-1.0):
    """Host evaluation of one axis' weights: (lo, w, dw, dw/dx, d(dw)/dx), entries from lo - 1."""
    import numpy as np
    span = LBM_MAX_STENCIL + 2
    arrs = [np.zeros(span) for _ in range(4)]
    lo = ct.c_int32()
    _ok(lib().lbm_host_axis_weights(float(x), float(n), int(ext), int(bool(periodic)), float(s_lo),
                                    float(s_hi), ct.byref(lo),
                                    *[a.ctypes.data_as(ct.POINTER(ct.c_double)) for a in arrs]),
        "lbm_host_axis_weights")
    return (lo.value,) + tuple(arrs)


def host_bubble_ode(params, nu, d, x0, ub0, ul, wl, dul, ext, periodic=(0, 0, 0)):
    import numpy as np
    ins = [_dp(v) for v in (x0, ub0, ul, wl, dul)]
    e = (ct.c_int32 * 3)(*[int(v) for v in ext])
    pr = (ct.c_int32 * 3)(*[int(bool(v)) for v in periodic])
    x, ub, psi = np.zeros(3), np.zeros(3), np.zeros(3)
    _ok(lib().lbm_host_bubble_ode(ct.byref(params), float(nu), float(d), *[p for _, p in ins], e, pr,
                                  *[a.ctypes.data_as(ct.POINTER(ct.c_double)) for a in (x, ub, psi)]),
        "lbm_host_bubble_ode")
    return x, ub, psi


def host_bubble_ode_adjoint(params, nu, d, x0, ub0, ul, wl, dul, ext, periodic, lx, lub, lpsi):
    import numpy as np
    ins = [_dp(v) for v in (x0, ub0, ul, wl, dul)]
    e = (ct.c_int32 * 3)(*[int(v) for v in ext])
    pr = (ct.c_int32 * 3)(*[int(bool(v)) for v in periodic])
    lams = [_dp(v) for v in (lx, lub, lpsi)]
    out = np.zeros(18)
    _ok(lib().lbm_host_bubble_ode_adjoint(ct.byref(params), float(nu), float(d), *[p for _, p in ins],
                                          e, pr, *[p for _, p in lams],
                                          out.ctypes.data_as(ct.POINTER(ct.c_double))),
        "lbm_host_bubble_ode_adjoint")
    return out
