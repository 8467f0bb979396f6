"""Host-side checks of the C ABI that need no GPU: the library loads, exports every function that
include/lbm.h declares, and rejects bad arguments before touching the device."""
import ctypes as ct
import os
import re

import pytest

from paper_1710_07073_amd import lbm as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lbm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"^\s*(?:lbm_status|const char\*)\s+(\w+)\s*\(", src, flags=re.M))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert names == set(L.EXPORTS)
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n


def test_header_constants_match_the_binding():
    """Every #define of include/lbm.h that the binding mirrors has the same value there."""
    src = open(HEADER).read()
    defines = dict((k, int(v)) for k, v in re.findall(r"^#define\s+(LBM_\w+)\s+(\d+)\s*$", src, flags=re.M))
    assert {"LBM_REACTION_MASK", "LBM_REACTION_SUBSTEP_MEAN", "LBM_REACTION_NET_FORCE",
            "LBM_COUPLING_POINT_KERNEL", "LBM_COUPLING_EXACT_TIME", "LBM_BUBBLE_WORK",
            "LBM_MAX_STENCIL", "LBM_BUBBLE_RECORD", "LBM_BUBBLE_ADJ"} <= set(defines)
    for k, v in defines.items():
        assert getattr(L, k) == v, k


def test_status_strings():
    for code in (0, -1, -2, -3, -4):
        assert L.lbm_status_string(code)
    assert L.lbm_status_string(-99) == "unknown status"


def test_bytes_required():
    d = L.make_desc((32, 32, 64), 1.0, L.LBM_FP64_SHIFTED)
    pop, field, scratch = L.lbm_bytes_required(d)
    n = 32 * 32 * 64
    assert pop == 19 * n * 8 and field == 3 * n * 8
    assert scratch >= 4 * 4 * 8 * 1 + (32 // 8) * (32 // 8) * (64 // 8)
    d = L.make_desc((37, 23, 19), 1.2, L.LBM_FP32_SHIFTED)
    pop, field, _ = L.lbm_bytes_required(d)
    assert pop == 19 * 37 * 23 * 19 * 4 and field == 3 * 37 * 23 * 19 * 4


@pytest.mark.parametrize("kw", [
    dict(shape=(0, 4, 4)), dict(omega=0.0), dict(omega=2.0), dict(omega=float("nan")),
    dict(precision=3), dict(bc=(2, 0, 0, 0, 0, 0)), dict(bc=(0, 0, 0, 0, 0, 5)), dict(flags=8),
    dict(shape=(2048, 2048, 32)),
])
def test_bad_descriptions_are_rejected(kw):
    args = dict(shape=(8, 8, 8), omega=1.0, precision=L.LBM_FP32_SHIFTED, bc=(0,) * 6, flags=0)
    args.update(kw)
    d = L.make_desc(args["shape"], args["omega"], args["precision"], args["bc"], args["flags"])
    with pytest.raises(L.LbmError) as e:
        L.lbm_bytes_required(d)
    assert e.value.code == L.LBM_EINVAL


def test_init_rejects_missing_buffers_without_device_work():
    d = L.make_desc((8, 8, 8), 1.0, L.LBM_FP32_SHIFTED)
    fake = ct.c_void_p(0x1000)
    with pytest.raises(L.LbmError) as e:
        L.lbm_init(d, fake, None, fake, fake, fake, None)
    assert e.value.code == L.LBM_EINVAL
    with pytest.raises(L.LbmError) as e:  # aliased population buffers
        L.lbm_init(d, fake, fake, fake, fake, fake, None)
    assert e.value.code == L.LBM_EINVAL


def test_null_context_calls_are_rejected():
    lib = L.lib()
    assert lib.lbm_step(None, 1) == L.LBM_EINVAL
    assert lib.moments(None, None, None, None) == L.LBM_EINVAL
    assert lib.lbm_check(None) == L.LBM_EINVAL
    out = ct.c_int32(-7)
    assert lib.lbm_set_step_occupancy(None, 3) == L.LBM_EINVAL
    assert lib.lbm_get_step_occupancy(None, ct.byref(out)) == L.LBM_EINVAL
    assert lib.lbm_set_overlap(None, 1) == L.LBM_EINVAL
    assert lib.lbm_record_next_bubble_half(None, None) == L.LBM_EINVAL
    assert lib.lbm_time_next_step(None, None, None) == L.LBM_EINVAL
    assert lib.lbm_time_next_adjoint_liquid(None, None, None) == L.LBM_EINVAL
    assert lib.lbm_step_tiles(None, None, None) == L.LBM_EINVAL
    assert lib.lbm_checkpoint(None, None, None) == L.LBM_EINVAL
    assert lib.lbm_restore(None, None, None) == L.LBM_EINVAL
    assert lib.lbm_batch_set_step_occupancy(None, 3) == L.LBM_EINVAL
    assert lib.lbm_batch_get_step_occupancy(None, ct.byref(out)) == L.LBM_EINVAL
    assert out.value == -7  # nothing written on rejection
    assert lib.lbm_destroy(None) == L.LBM_OK


@pytest.mark.parametrize("g,sigma,ok", [(0.0, 0.0, True), (3e-4, 1e-4, True), (-1e-5, 0.0, False),
                                        (0.0, -1.0, False), (float("nan"), 0.0, False),
                                        (0.0, float("inf"), False)])
def test_batch_column_constants_are_checked(g, sigma, ok):
    """A batched column's own gravity and surface tension: 0 takes the batch's value; negative or
    non-finite values are rejected before any device work."""
    cols = L.make_columns([((24, 24, 48), 1.2, (0,) * 6, 1, g, sigma),
                           ((16, 20, 40), 0.9, (0,) * 6, 2)])
    assert ct.sizeof(L.LbmColumn) == 72 and cols[1].bubble_begin == 1
    if ok:
        pool, scratch = L.lbm_batch_bytes_required(cols, L.LBM_FP32_SHIFTED)
        assert pool > 0 and scratch > 0
    else:
        with pytest.raises(L.LbmError) as e:
            L.lbm_batch_bytes_required(cols, L.LBM_FP32_SHIFTED)
        assert e.value.code == L.LBM_EINVAL
