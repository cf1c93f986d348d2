"""Host-side checks of the C-ABI library: it loads, exports every entry point the
header declares, and rejects bad arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

import paper_1711_00975_amd as csk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "csk.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(csk_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(csk.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(csk.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_argument_errors_are_returned_without_a_device():
    lib = csk.load_library()
    h = C.c_void_p()
    assert lib.csk_sketch_init(C.byref(h), 0, 16, 1) == csk.CSK_E_INVALID
    assert "d=0" in csk.csk_last_error()
    assert lib.csk_sketch_init(C.byref(h), 33, 16, 1) == csk.CSK_E_INVALID
    assert lib.csk_sketch_init(C.byref(h), 5, 0, 1) == csk.CSK_E_INVALID
    assert lib.csk_sketch_init(C.byref(h), 5, (1 << 30) + 1, 1) == csk.CSK_E_INVALID
    assert lib.csk_sketch_init_ex(C.byref(h), 5, 16, 1, 7, 0) == csk.CSK_E_INVALID
    assert lib.csk_sketch_init(None, 5, 16, 1) == csk.CSK_E_INVALID
    assert lib.csk_sketch_update(None, None, 0, 0.1, 100.0, None) == csk.CSK_E_INVALID
    assert lib.csk_topk(None, 1, None, None, None, None) == csk.CSK_E_INVALID
    assert lib.csk_collect_dictionary(None, 0.1, 100.0, 0, None) == csk.CSK_E_INVALID
    assert lib.csk_collect_children(None, None, 0, None) == csk.CSK_E_INVALID
    assert lib.csk_batch_create(None, None, None, 1, 0.1, 100.0, 0) == csk.CSK_E_INVALID
    assert lib.csk_batch_update(None, None, None, None) == csk.CSK_E_INVALID
    assert lib.csk_batch_topk(None, None, None, None, None, None) == csk.CSK_E_INVALID
    assert lib.csk_topk_async(None, 1, None, None, None, None) == csk.CSK_E_INVALID
    assert lib.csk_sketch_init_group(C.byref(h), 5, 16, 1, 0, 0, 0) == csk.CSK_E_INVALID
    # learned router
    assert lib.csk_mlp_create(C.byref(h), 1, 0) == csk.CSK_E_INVALID
    assert lib.csk_mlp_create(None, 1, 16) == csk.CSK_E_INVALID
    assert lib.csk_mlp_train_step(None, None, None, 1, 1e-3, None, None) == csk.CSK_E_INVALID
    assert lib.csk_gemm_bf16((1 << 20) + 1, 16, 16, None, 0, 0, None, 0, 0, None, 0, 0, 0.0, None) == csk.CSK_E_INVALID
    assert lib.csk_gemm_bf16(16, 16, 16, None, 0, 0, None, 0, 0, None, 0, 0, 0.0, None) == csk.CSK_E_INVALID
    assert lib.csk_gemm_bf16(0, 16, 16, None, 0, 0, None, 0, 0, None, 0, 0, 0.0, None) == csk.CSK_OK
    assert lib.csk_sample_counts(None, 0, 0, 0.3, 100.0, 1, 0, None, None, None) == csk.CSK_E_INVALID
    assert lib.csk_cells_clear(None, None, 5, None) == csk.CSK_E_INVALID
    assert lib.csk_cell_features(None, 1.0, 100.0, None, 5, None, None) == csk.CSK_E_INVALID
    route = lambda factor, na, slots: lib.csk_route_split(None, 0, 0.25, 50.0, factor, None, na, None, None, slots,
                                                          None, None, None, None, 0, None)
    assert route(3, 0, 1024) == csk.CSK_E_INVALID          # 3 does not divide G = 200
    assert route(4, 513, 1 << 20) == csk.CSK_E_INVALID     # more than 512 admitted cells
    assert route(4, 1, 1000) == csk.CSK_E_INVALID          # slots not a power of two
    assert route(4, 8, 512) == csk.CSK_E_INVALID           # 8 * 4^3 children above half of 512 slots
    assert route(4, 4, 512) == csk.CSK_OK
    assert route(8, 100, 1 << 20) == csk.CSK_E_INVALID     # 100 * 8^3 children above 2^15
    ws = C.c_uint64(0)
    assert lib.csk_route_split_workspace(512, 4, C.byref(ws)) == csk.CSK_OK and ws.value >= 256 * 512 * 64 * 4
    assert lib.csk_route_split_workspace(513, 4, C.byref(ws)) == csk.CSK_E_INVALID
    # a stream with too small a workspace is refused before any launch
    assert lib.csk_route_split(C.c_void_p(8), 10, 0.25, 50.0, 4, C.c_void_p(8), 4, C.c_void_p(8), C.c_void_p(8),
                               512, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), 16, None) \
        == csk.CSK_E_INVALID
    assert lib.csk_topk_with_table(None, None, None, 16, 1, None, None, None, None) == csk.CSK_E_INVALID
    assert lib.csk_exact_counts(None, 0, 0.25, 50.0, None, None, 1000, None, None) == csk.CSK_E_INVALID
    assert lib.csk_exact_counts(None, 5, 0.25, 50.0, None, None, 1024, None, None) == csk.CSK_E_INVALID
    kout = C.c_uint32(7)
    assert lib.csk_table_topk(None, None, 1024, 1, None, None, C.byref(kout), None) == csk.CSK_E_INVALID
    tot = C.c_uint64(7)
    assert lib.csk_cell_list(None, 5, 1, None, None, 0, None, None) == csk.CSK_E_INVALID
    assert lib.csk_cell_list(None, 0, 1, None, None, 0, C.byref(tot), None) == csk.CSK_OK and tot.value == 0
    assert lib.csk_cell_labels(None, 5, None, (1 << 17) + 1, 0.25, 50.0, 4, None, None) == csk.CSK_E_INVALID
    assert lib.csk_cell_labels(None, 5, None, 3, 0.25, 50.0, 3, None, None) == csk.CSK_E_INVALID
    na = C.c_uint32(7)
    assert lib.csk_route_admit(None, None, 10, (1 << 16) + 1, None, C.byref(na), None) == csk.CSK_E_INVALID
    assert lib.csk_route_admit(None, None, 0, 5, None, C.byref(na), None) == csk.CSK_OK and na.value == 0
    # invalid meshes
    for delta, L in [(0.0, 100.0), (0.3, 100.0), (1e-4, 100.0), (float("nan"), 1.0), (1.0, float("inf"))]:
        assert lib.csk_cell_keys(None, 0, delta, L, None, None) == csk.CSK_E_INVALID
    assert lib.csk_cell_keys(None, 5, 0.1, 100.0, None, None) == csk.CSK_E_INVALID
    assert lib.csk_cell_keys(None, 0, 0.1, 100.0, None, None) == csk.CSK_OK


def test_missing_library_fails_loudly(tmp_path):
    saved = csk._lib
    try:
        csk._lib = None
        with pytest.raises(RuntimeError):
            csk.load_library(str(tmp_path / "libcsk.so"))
    finally:
        csk._lib = saved
