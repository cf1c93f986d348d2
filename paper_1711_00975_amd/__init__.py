"""Streaming Count-Sketch halo finder for AMD MI355X (gfx950).

Python binding of ``libcsk.so``, the HIP library behind ``include/csk.h``.  The
functions below carry the C ABI's names and only marshal arguments: device
pointers come from PyTorch tensors (PyTorch supplies device memory and streams),
and every step of the hot path runs in the library's HIP kernels.  If the
library is missing this module raises; there is no CPU fallback.

Hot path (arXiv:1711.00975): particle -> mesh-cell key (Sec. 2.1) -> Count Sketch
Add (Sec. 2.2) -> median Estimate of each distinct cell (Sec. 2.2) -> top-k
(Sec. 2.2 UpdateHeap, Alg. 1; Sec. 3.1 item 4).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsk.so")

CSK_OK = 0
CSK_W_INCOMPLETE = 1
CSK_E_INVALID = -1
CSK_E_NOMEM = -2
CSK_E_HIP = -3
CSK_E_CAPACITY = -4
CSK_E_DOMAIN = -5
CSK_E_STATE = -6
CSK_VARIANT_COUNT_SKETCH = 0
CSK_VARIANT_COUNT_MIN = 1
CSK_MAX_ROWS = 32
CSK_MAX_WIDTH = 1 << 30
CSK_DEFAULT_CANDIDATES = 1 << 21
INT32_MIN = -(2 ** 31)

EXPORTS = ["csk_sketch_init", "csk_sketch_init_ex", "csk_sketch_init_group", "csk_sketch_destroy", "csk_sketch_update",
           "csk_sketch_update_noalloc",
           "csk_set_update_plan", "csk_set_update_tiling",
           "csk_sketch_query", "csk_cell_keys", "csk_collect",
           "csk_pack_positions", "csk_sketch_update_packed", "csk_collect_packed", "csk_cell_keys_packed", "csk_collect_dictionary", "csk_collect_children", "csk_candidates_clear",
           "csk_topk", "csk_topk_async", "csk_batch_create", "csk_batch_create_meshes", "csk_batch_update", "csk_batch_topk", "csk_batch_destroy",
           "csk_batch_reset", "csk_batch_collect",
           "csk_sample_counts", "csk_cell_features", "csk_mlp_create", "csk_mlp_destroy", "csk_mlp_params",
           "csk_mlp_grads", "csk_mlp_forward", "csk_mlp_train_step", "csk_gemm_bf16", "csk_route_split", "csk_route_split_workspace", "csk_topk_with_table",
           "csk_exact_counts", "csk_table_topk", "csk_cell_list", "csk_cells_clear", "csk_cell_labels",
           "csk_route_admit", "csk_cell_list_workspace", "csk_cell_list_async", "csk_route_score",
           "csk_route_admit_workspace", "csk_route_admit_async", "csk_route_update_workspace",
           "csk_sketch_update_routed", "csk_topk_with_table_async",
           "csk_get_counters", "csk_set_counters", "csk_reset", "csk_check", "csk_device_bytes",
           "csk_last_error"]


class CskError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"csk error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libcsk.so and declare its signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() "
                           "(or python -m paper_1711_00975_amd.build)")
    lib = C.CDLL(path)
    P, u64, u32, i32, f64 = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int32, C.c_double
    PP = C.POINTER(C.c_void_p)
    sig = {
        "csk_sketch_init": [PP, u32, u32, u64],
        "csk_sketch_init_ex": [PP, u32, u32, u64, i32, u64],
        "csk_sketch_init_group": [PP, u32, u32, u64, i32, u64, u32],
        "csk_sketch_destroy": [P],
        "csk_sketch_update": [P, P, u64, f64, f64, P],
        "csk_sketch_update_noalloc": [P, P, u64, f64, f64, P],
        "csk_set_update_tiling": [P, i32, u32, u32, i32],
        "csk_set_update_plan": [P, i32, u32],
        "csk_sketch_query": [P, P, u64, P, P],
        "csk_cell_keys": [P, u64, f64, f64, P, P],
        "csk_collect": [P, P, u64, f64, f64, i32, P],
        "csk_pack_positions": [P, u64, f64, P, P, P],
        "csk_sketch_update_packed": [P, P, u64, f64, f64, P],
        "csk_collect_packed": [P, P, u64, f64, f64, i32, P],
        "csk_cell_keys_packed": [P, u64, f64, f64, P, P],
        "csk_collect_dictionary": [P, f64, f64, i32, P],
        "csk_collect_children": [P, P, i32, P],
        "csk_candidates_clear": [P, P],
        "csk_topk": [P, u32, P, P, C.POINTER(C.c_uint32), P],
        "csk_topk_async": [P, u32, P, P, P, P],
        "csk_batch_create": [PP, P, P, u32, f64, f64, u32],
        "csk_batch_create_meshes": [PP, P, P, u32, P, P, u32],
        "csk_batch_topk": [P, P, P, P, P, P],
        "csk_batch_update": [P, P, P, P],
        "csk_batch_destroy": [P],
        "csk_batch_reset": [P, P],
        "csk_batch_collect": [P, P, P, P, P],
        "csk_sample_counts": [P, u64, u64, f64, f64, u64, u32, P, P, P],
        "csk_cell_features": [P, f64, f64, P, u64, P, P],
        "csk_mlp_create": [PP, u64, u32],
        "csk_mlp_destroy": [P],
        "csk_mlp_params": [P, P, P],
        "csk_mlp_grads": [P, P],
        "csk_mlp_forward": [P, P, u64, P, P],
        "csk_mlp_train_step": [P, P, P, u32, C.c_float, P, P],
        "csk_gemm_bf16": [u32, u32, u32, P, u64, u64, P, u64, u64, P, u64, u64, C.c_float, P],
        "csk_route_split": [P, u64, f64, f64, u32, P, u32, P, P, u32, P, P, P, P, u64, P],
        "csk_route_split_workspace": [u32, u32, C.POINTER(C.c_uint64)],
        "csk_topk_with_table": [P, P, P, u32, u32, P, P, C.POINTER(C.c_uint32), P],
        "csk_exact_counts": [P, u64, f64, f64, P, P, u32, P, P],
        "csk_table_topk": [P, P, u32, u32, P, P, C.POINTER(C.c_uint32), P],
        "csk_cell_list": [P, u64, u32, P, P, u64, C.POINTER(C.c_uint64), P],
        "csk_cells_clear": [P, P, u64, P],
        "csk_cell_labels": [P, u64, P, u32, f64, f64, u32, P, P],
        "csk_route_admit": [P, P, u64, u32, P, C.POINTER(C.c_uint32), P],
        "csk_cell_list_workspace": [u64, C.POINTER(C.c_uint64)],
        "csk_cell_list_async": [P, u64, u32, P, P, u64, P, P, u64, P],
        "csk_route_score": [P, P, f64, f64, P, P, u64, P, P],
        "csk_route_admit_workspace": [u64, u32, C.POINTER(C.c_uint64)],
        "csk_route_admit_async": [P, P, P, u64, u32, P, P, P, u64, P],
        "csk_route_update_workspace": [u32, u32, C.POINTER(C.c_uint64)],
        "csk_sketch_update_routed": [P, P, u64, f64, f64, u32, P, P, P, P, u32, P, P, u64, P],
        "csk_topk_with_table_async": [P, P, P, u32, u32, P, P, P, P],
        "csk_get_counters": [P, P, P],
        "csk_set_counters": [P, P, P],
        "csk_reset": [P, P],
        "csk_check": [P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.restype = i32
        fn.argtypes = args
    lib.csk_device_bytes.restype = u64
    lib.csk_device_bytes.argtypes = [P]
    lib.csk_last_error.restype = C.c_char_p
    lib.csk_last_error.argtypes = []
    _lib = lib
    return lib


def _check(rc: int, allow_warning: bool = False) -> int:
    if rc == CSK_OK or (allow_warning and rc > 0):
        return rc
    raise CskError(rc, load_library().csk_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dev(t, dtype, shape_last=None):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if shape_last is not None and (t.dim() != 2 or t.shape[1] != shape_last):
        raise ValueError(f"expected shape [n, {shape_last}]")
    return C.c_void_p(t.data_ptr())


# ------------------------------------------------------------- C ABI, by name

def csk_sketch_init(d: int, w: int, seed: int):
    h = C.c_void_p()
    _check(load_library().csk_sketch_init(C.byref(h), d, w, seed))
    return h


def csk_sketch_init_ex(d: int, w: int, seed: int, variant: int = CSK_VARIANT_COUNT_SKETCH,
                       max_candidates: int = 0):
    h = C.c_void_p()
    _check(load_library().csk_sketch_init_ex(C.byref(h), d, w, seed, variant, max_candidates))
    return h


def csk_sketch_init_group(d: int, w: int, seed: int, variant: int = CSK_VARIANT_COUNT_SKETCH,
                          max_candidates: int = 0, group: int = 1):
    h = C.c_void_p()
    _check(load_library().csk_sketch_init_group(C.byref(h), d, w, seed, variant, max_candidates, group))
    return h


CSK_UPDATE_AUTO, CSK_UPDATE_BINNED, CSK_UPDATE_DIRECT = 0, 1, 2
CSK_BIN_AUTO, CSK_BIN_GENERAL, CSK_BIN_SORT_WORD = 0, 1, 2


def csk_set_update_plan(h, mode: int, max_wg: int = 0) -> None:
    _check(load_library().csk_set_update_plan(h, mode, max_wg))


def csk_set_update_tiling(h, form: int = 0, threads: int = 0, rows_per_pass: int = 0, prefetch: int = 0) -> None:
    _check(load_library().csk_set_update_tiling(h, form, threads, rows_per_pass, prefetch))


def csk_sketch_destroy(h) -> None:
    _check(load_library().csk_sketch_destroy(h))


def csk_sketch_update(h, pos, delta: float, L: float, stream=None) -> None:
    import torch
    _check(load_library().csk_sketch_update(h, _dev(pos, torch.float32, 3), pos.shape[0], delta, L,
                                            _stream(stream)))


def csk_sketch_update_noalloc(h, pos, delta: float, L: float, stream=None) -> None:
    import torch
    _check(load_library().csk_sketch_update_noalloc(h, _dev(pos, torch.float32, 3), pos.shape[0], delta, L,
                                                    _stream(stream)))


def csk_sketch_query(h, keys, est, stream=None) -> None:
    import torch
    if keys.numel() != est.numel():
        raise ValueError("keys and est differ in length")
    _check(load_library().csk_sketch_query(h, _dev(keys, torch.int64), keys.numel(), _dev(est, torch.int32),
                                           _stream(stream)))


def csk_cell_keys(pos, delta: float, L: float, keys, stream=None) -> None:
    import torch
    if keys.numel() != pos.shape[0]:
        raise ValueError("keys must hold one entry per particle")
    _check(load_library().csk_cell_keys(_dev(pos, torch.float32, 3), pos.shape[0], delta, L,
                                        _dev(keys, torch.int64), _stream(stream)))


def csk_collect(h, pos, delta: float, L: float, theta: int, stream=None) -> None:
    import torch
    _check(load_library().csk_collect(h, _dev(pos, torch.float32, 3), pos.shape[0], delta, L, theta,
                                      _stream(stream)))


def pack_positions(pos, L: float, err=None, stream=None):
    """The packed stream (int64 words holding uint64: qx | qy << 21 | qz << 42, q =
    floor(p 2^21 / L); all ones outside the domain, which sets err[0] bit 0)."""
    import torch
    out = torch.empty(pos.shape[0], dtype=torch.int64, device=pos.device)
    if err is None:
        err = torch.zeros(1, dtype=torch.int32, device=pos.device)
    if pos.shape[0]:
        _check(load_library().csk_pack_positions(_dev(pos, torch.float32, 3), pos.shape[0], L, _dev(out, torch.int64),
                                                 _dev(err, torch.int32), _stream(stream)))
    return out


def csk_sketch_update_packed(h, words, delta: float, L: float, stream=None) -> None:
    import torch
    _check(load_library().csk_sketch_update_packed(h, _dev(words, torch.int64) if words.numel() else None,
                                                   words.numel(), delta, L, _stream(stream)))


def csk_collect_packed(h, words, delta: float, L: float, theta: int, stream=None) -> None:
    import torch
    _check(load_library().csk_collect_packed(h, _dev(words, torch.int64) if words.numel() else None, words.numel(),
                                             delta, L, theta, _stream(stream)))


def cell_keys_packed(words, delta: float, L: float, stream=None):
    import torch
    keys = torch.empty(words.numel(), dtype=torch.int64, device=words.device)
    if words.numel():
        _check(load_library().csk_cell_keys_packed(_dev(words, torch.int64), words.numel(), delta, L,
                                                   _dev(keys, torch.int64), _stream(stream)))
    return keys


def csk_collect_dictionary(h, delta: float, L: float, theta: int, stream=None) -> None:
    _check(load_library().csk_collect_dictionary(h, delta, L, theta, _stream(stream)))


def csk_collect_children(fine, coarse, theta: int, stream=None) -> None:
    _check(load_library().csk_collect_children(fine, coarse, theta, _stream(stream)))


def csk_candidates_clear(h, stream=None) -> None:
    _check(load_library().csk_candidates_clear(h, _stream(stream)))


def csk_topk(h, k: int, keys, est, stream=None) -> tuple[int, int]:
    """Returns (k_out, status); status is CSK_OK or CSK_W_INCOMPLETE."""
    import torch
    if keys.numel() < k or est.numel() < k:
        raise ValueError("output tensors hold fewer than k entries")
    kout = C.c_uint32(0)
    rc = _check(load_library().csk_topk(h, k, _dev(keys, torch.int64), _dev(est, torch.int32), C.byref(kout),
                                        _stream(stream)), allow_warning=True)
    return kout.value, rc


def csk_topk_async(h, k: int, keys, est, out, stream=None) -> None:
    """No host synchronization: out (device uint32 [2]) gets (number written, incomplete flag)."""
    import torch
    _check(load_library().csk_topk_async(h, k, _dev(keys, torch.int64) if k else None,
                                         _dev(est, torch.int32) if k else None, _dev(out, torch.int32),
                                         _stream(stream)))


def csk_get_counters(h, out, stream=None) -> None:
    import torch
    _check(load_library().csk_get_counters(h, _dev(out, torch.int32), _stream(stream)))


def csk_set_counters(h, src, stream=None) -> None:
    import torch
    _check(load_library().csk_set_counters(h, _dev(src, torch.int32), _stream(stream)))


def csk_reset(h, stream=None) -> None:
    _check(load_library().csk_reset(h, _stream(stream)))


def csk_check(h, stream=None) -> None:
    _check(load_library().csk_check(h, _stream(stream)))


def csk_device_bytes(h) -> int:
    return int(load_library().csk_device_bytes(h))


def csk_last_error() -> str:
    return load_library().csk_last_error().decode()


# ------------------------------------------------------------- convenience

class Batch:
    """Up to 64 sketches updated by one bin and one accumulate launch (csk_batch_*)."""

    def __init__(self, sketches, max_n, delta, L, wg_budget: int = 0):
        """delta and L: one mesh for every sketch, or one per sketch (sequences)."""
        lib = load_library()
        m = len(sketches)
        arr = (C.c_void_p * m)(*[s.h.value if isinstance(s.h, C.c_void_p) else s.h for s in sketches])
        mx = (C.c_uint64 * m)(*[int(x) for x in max_n])
        h = C.c_void_p()
        if isinstance(delta, (list, tuple)) or isinstance(L, (list, tuple)):
            ds = list(delta) if isinstance(delta, (list, tuple)) else [delta] * m
            ls = list(L) if isinstance(L, (list, tuple)) else [L] * m
            _check(lib.csk_batch_create_meshes(C.byref(h), arr, mx, m, (C.c_double * m)(*ds), (C.c_double * m)(*ls),
                                               wg_budget))
        else:
            _check(lib.csk_batch_create(C.byref(h), arr, mx, m, delta, L, wg_budget))
        self.h, self.sketches, self.count = h, list(sketches), m

    def update(self, positions, stream=None):
        """positions: one float32 [n_i][3] device tensor per sketch (n_i may be 0)."""
        import torch
        if len(positions) != self.count:
            raise ValueError("one position tensor per sketch")
        ptrs = (C.c_void_p * self.count)(*[_dev(t, torch.float32, 3) if t.shape[0] else None for t in positions])
        ns = (C.c_uint64 * self.count)(*[int(t.shape[0]) for t in positions])
        _check(load_library().csk_batch_update(self.h, ptrs, ns, _stream(stream)))

    def reset(self, stream=None):
        """Every sketch back to zero counters and an empty candidate set, in one launch."""
        _check(load_library().csk_batch_reset(self.h, _stream(stream)))

    def collect(self, positions, thetas, stream=None):
        """The candidate pass of every sketch (positions: one float32 [n_i][3] device tensor
        per sketch, thetas: one int per sketch) as one set of launches."""
        import torch
        if len(positions) != self.count or len(thetas) != self.count:
            raise ValueError("one position tensor and one threshold per sketch")
        ptrs = (C.c_void_p * self.count)(*[_dev(t, torch.float32, 3) if t.shape[0] else None for t in positions])
        ns = (C.c_uint64 * self.count)(*[int(t.shape[0]) for t in positions])
        th = (C.c_int32 * self.count)(*[int(x) for x in thetas])
        _check(load_library().csk_batch_collect(self.h, ptrs, ns, th, _stream(stream)))

    def topk(self, ks, keys, est, outs, stream=None):
        """Top-k of every sketch in one set of launches: ks (ints), keys / est (device int64 /
        int32 tensors of at least k each), outs (device int32 [2] each: count, incomplete)."""
        import torch
        m = self.count
        if not (len(ks) == len(keys) == len(est) == len(outs) == m):
            raise ValueError("one k and one output per sketch")
        kk = (C.c_uint32 * m)(*[int(k) for k in ks])
        kp = (C.c_void_p * m)(*[_dev(t, torch.int64) if k else None for t, k in zip(keys, ks)])
        ep = (C.c_void_p * m)(*[_dev(t, torch.int32) if k else None for t, k in zip(est, ks)])
        op = (C.c_void_p * m)(*[_dev(t, torch.int32) for t in outs])
        for t, k in zip(keys, ks):
            if k and t.numel() < k:
                raise ValueError("an output holds fewer than k entries")
        _check(load_library().csk_batch_topk(self.h, kk, kp, ep, op, _stream(stream)))

    def close(self):
        if self.h is not None:
            _check(load_library().csk_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sketch:
    """Owns one handle.  d rows ("t" in the paper) by w counters ("b")."""

    def __init__(self, d: int, w: int, seed: int, variant: int = CSK_VARIANT_COUNT_SKETCH,
                 max_candidates: int = 0, group: int = 1):
        """group > 1: the sketch counts super-items (cell key // group), the coarse layer
        of the hierarchical variant."""
        self.d, self.w, self.seed, self.variant, self.group = d, w, seed, variant, group
        self.h = csk_sketch_init_group(d, w, seed, variant, max_candidates, group)

    def close(self):
        if self.h is not None:
            csk_sketch_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update(self, pos, delta, L, stream=None):
        csk_sketch_update(self.h, pos, delta, L, stream)

    def update_noalloc(self, pos, delta, L, stream=None):
        csk_sketch_update_noalloc(self.h, pos, delta, L, stream)

    def query(self, keys, stream=None):
        import torch
        est = torch.empty(keys.numel(), dtype=torch.int32, device=keys.device)
        csk_sketch_query(self.h, keys, est, stream)
        return est

    def collect(self, pos, delta, L, theta=INT32_MIN, stream=None):
        csk_collect(self.h, pos, delta, L, theta, stream)

    def update_packed(self, words, delta, L, stream=None):
        csk_sketch_update_packed(self.h, words, delta, L, stream)

    def collect_packed(self, words, delta, L, theta=INT32_MIN, stream=None):
        csk_collect_packed(self.h, words, delta, L, theta, stream)

    def collect_dictionary(self, delta, L, theta=INT32_MIN, stream=None):
        csk_collect_dictionary(self.h, delta, L, theta, stream)

    def collect_children(self, coarse, theta=INT32_MIN, stream=None):
        """Children of coarse's candidate super-items with estimate >= theta join this set."""
        csk_collect_children(self.h, coarse.h, theta, stream)

    def clear_candidates(self, stream=None):
        csk_candidates_clear(self.h, stream)

    def topk(self, k, stream=None):
        """(keys int64 [k_out], est int32 [k_out], status) on the device."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        keys = torch.empty(max(k, 1), dtype=torch.int64, device=dev)
        est = torch.empty(max(k, 1), dtype=torch.int32, device=dev)
        kout, rc = csk_topk(self.h, k, keys, est, stream)
        return keys[:kout], est[:kout], rc

    def set_update_plan(self, mode, max_wg=0):
        csk_set_update_plan(self.h, mode, max_wg)

    def set_update_tiling(self, form=0, threads=0, rows_per_pass=0, prefetch=0):
        csk_set_update_tiling(self.h, form, threads, rows_per_pass, prefetch)

    def topk_async(self, k, keys, est, out, stream=None):
        """Top-k into preallocated device tensors without synchronizing (graph-capturable)."""
        csk_topk_async(self.h, k, keys, est, out, stream)

    def counters(self, stream=None):
        import torch
        out = torch.empty((self.d, self.w), dtype=torch.int32,
                          device=torch.device("cuda", torch.cuda.current_device()))
        csk_get_counters(self.h, out, stream)
        return out

    def set_counters(self, src, stream=None):
        csk_set_counters(self.h, src, stream)

    def reset(self, stream=None):
        csk_reset(self.h, stream)

    def check(self, stream=None):
        csk_check(self.h, stream)

    def device_bytes(self):
        return csk_device_bytes(self.h)


def cell_keys(pos, delta, L, stream=None):
    import torch
    keys = torch.empty(pos.shape[0], dtype=torch.int64, device=pos.device)
    csk_cell_keys(pos, delta, L, keys, stream)
    return keys


# ------------------------------------------------------------- learned router

SAMPLE_THRESHOLD = 42949672   # floor(0.01 * 2^32): the 1 % sample
N_PARAMS = 6337
FEAT = 32


def sample_counts(pos, delta_c, L, seed, counts, index0=0, threshold=SAMPLE_THRESHOLD, stream=None, bitmap=None):
    """Add the 1 % sample of pos (particles index0 ..) to counts (device uint32 [G_c^3] as int32);
    bitmap (device int32 [ceil(G_c^3 / 32)]) marks the cells first touched."""
    import torch
    _check(load_library().csk_sample_counts(_dev(pos, torch.float32, 3) if pos.shape[0] else None, pos.shape[0],
                                            index0, delta_c, L, seed, threshold, _dev(counts, torch.int32),
                                            _dev(bitmap, torch.int32) if bitmap is not None else None,
                                            _stream(stream)))


def cell_features(counts, delta_c, L, cells, stream=None):
    """float32 [m][32] features of the coarse cells `cells` (device int64 keys)."""
    import torch
    feat = torch.empty((cells.shape[0], FEAT), dtype=torch.float32, device=cells.device)
    if cells.shape[0]:
        _check(load_library().csk_cell_features(_dev(counts, torch.int32), delta_c, L, _dev(cells, torch.int64),
                                                cells.shape[0], _dev(feat, torch.float32, FEAT), _stream(stream)))
    return feat


class MLP:
    """The router's 27 -> 64 -> 64 -> 1 model (csk_mlp_*)."""

    def __init__(self, seed=1, max_batch=4096):
        h = C.c_void_p()
        _check(load_library().csk_mlp_create(C.byref(h), seed, max_batch))
        self.h, self.max_batch = h, max_batch

    def params(self):
        import numpy as np
        out = np.empty(N_PARAMS, dtype=np.float32)
        _check(load_library().csk_mlp_params(self.h, out.ctypes.data_as(C.c_void_p), None))
        return out

    def set_params(self, p):
        import numpy as np
        a = np.ascontiguousarray(p, dtype=np.float32)
        assert a.size == N_PARAMS
        _check(load_library().csk_mlp_params(self.h, None, a.ctypes.data_as(C.c_void_p)))

    def grads(self):
        import numpy as np
        out = np.empty(N_PARAMS, dtype=np.float32)
        _check(load_library().csk_mlp_grads(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def forward(self, x, stream=None):
        import torch
        z = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        if x.shape[0]:
            _check(load_library().csk_mlp_forward(self.h, _dev(x, torch.float32, FEAT), x.shape[0],
                                                  _dev(z, torch.float32), _stream(stream)))
        return z

    def train_step(self, x, y, lr, loss=None, stream=None):
        import torch
        _check(load_library().csk_mlp_train_step(self.h, _dev(x, torch.float32, FEAT), _dev(y, torch.float32),
                                                 x.shape[0], lr, _dev(loss, torch.float32) if loss is not None else None,
                                                 _stream(stream)))

    def close(self):
        if self.h is not None:
            _check(load_library().csk_mlp_destroy(self.h))
            self.h = None


def gemm_bf16(M, N, K, A, sa, B, sb, C_out, sc, beta=0.0, stream=None):
    """C = beta C + A B over strided device float32 views (strides in elements: sa = (row,
    k), sb = (k, col), sc = (row, col)) with bf16 operands and float32 sums."""
    def span(t, r, c, st):   # every element the kernel reads or writes lies inside t
        _dev(t, torch.float32)
        if r and c and (r - 1) * st[0] + (c - 1) * st[1] >= t.numel():
            raise ValueError("gemm_bf16: strides reach outside the tensor")
    import torch
    span(C_out, M, N, sc)
    if K:
        span(A, M, K, sa)
        span(B, K, N, sb)
    _check(load_library().csk_gemm_bf16(M, N, K, A.data_ptr() if K else None, sa[0], sa[1],
                                        B.data_ptr() if K else None, sb[0], sb[1], C_out.data_ptr(), sc[0], sc[1],
                                        beta, _stream(stream)))


_split_ws = {}


def route_split(pos, delta, L, factor, admitted, table_keys, table_counts, rest_pos, rest_count, err, stream=None,
                workspace=None):
    """admitted: sorted device int64 coarse keys; table_keys (int64, all ones when empty) and
    table_counts (int32) of a power-of-two size; rest_pos float32 [>= rest_count + n][3];
    rest_count int64 [1] (the rest is appended after it); err int32 [1].  workspace: a
    device uint8 tensor of csk_route_split_workspace bytes (one kept per device and size
    class when omitted)."""
    import torch
    lib = load_library()
    na = admitted.shape[0]
    need = C.c_uint64(0)
    _check(lib.csk_route_split_workspace(na, factor, C.byref(need)))
    if workspace is None:
        key = (pos.device.index, factor, max(na, 1).bit_length())
        workspace = _split_ws.get(key)
        if workspace is None or workspace.numel() < need.value:
            workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device=pos.device)
            _split_ws[key] = workspace
    _check(lib.csk_route_split(_dev(pos, torch.float32, 3) if pos.shape[0] else None, pos.shape[0], delta, L,
                               factor, _dev(admitted, torch.int64) if na else None, na,
                               _dev(table_keys, torch.int64), _dev(table_counts, torch.int32), table_keys.shape[0],
                               _dev(rest_pos, torch.float32, 3), _dev(rest_count, torch.int64),
                               _dev(err, torch.int32), workspace.data_ptr(), workspace.numel(), _stream(stream)))


def topk_with_table(sketch, table_keys, table_counts, k, stream=None):
    import torch
    dev = table_keys.device
    keys = torch.empty(max(k, 1), dtype=torch.int64, device=dev)
    est = torch.empty(max(k, 1), dtype=torch.int32, device=dev)
    kout = C.c_uint32(0)
    rc = _check(load_library().csk_topk_with_table(sketch.h, _dev(table_keys, torch.int64),
                                                   _dev(table_counts, torch.int32), table_keys.shape[0], k,
                                                   _dev(keys, torch.int64), _dev(est, torch.int32), C.byref(kout),
                                                   _stream(stream)), allow_warning=True)
    return keys[:kout.value], est[:kout.value], rc


def exact_counts(pos, delta, L, table_keys, table_counts, err, stream=None):
    """Add every particle of pos to the exact table (table_keys int64 all ones when empty,
    table_counts int32, same power-of-two size; err int32 [1])."""
    import torch
    _check(load_library().csk_exact_counts(_dev(pos, torch.float32, 3) if pos.shape[0] else None, pos.shape[0], delta,
                                           L, _dev(table_keys, torch.int64), _dev(table_counts, torch.int32),
                                           table_keys.shape[0], _dev(err, torch.int32), _stream(stream)))


def new_table(slots, device="cuda"):
    """An empty exact table (keys, counts) of `slots` entries."""
    import torch
    return (torch.full((slots,), -1, dtype=torch.int64, device=device),
            torch.zeros(slots, dtype=torch.int32, device=device))


def table_topk(table_keys, table_counts, k, stream=None):
    """(keys, counts) of the k heaviest table entries, by (count desc, key asc)."""
    import torch
    keys = torch.empty(max(k, 1), dtype=torch.int64, device=table_keys.device)
    counts = torch.empty(max(k, 1), dtype=torch.int32, device=table_keys.device)
    kout = C.c_uint32(0)
    _check(load_library().csk_table_topk(_dev(table_keys, torch.int64), _dev(table_counts, torch.int32),
                                         table_keys.shape[0], k, _dev(keys, torch.int64), _dev(counts, torch.int32),
                                         C.byref(kout), _stream(stream)))
    return keys[:kout.value], counts[:kout.value]


def cell_list(counts, min_count=1, cap=None, stream=None, out=None, bitmap=None):
    """Ascending device int64 list of the cells with counts >= min_count (only the cells
    marked in `bitmap` are examined when it is given).  With `out` (a device int64 buffer)
    the list is written there and a larger buffer is made only when it is too small;
    otherwise cap (default: count first) bounds the list."""
    import torch
    total = C.c_uint64(0)
    lib = load_library()
    bm = _dev(bitmap, torch.int32) if bitmap is not None else None
    grow = out is not None
    if out is None:
        if cap is None:
            _check(lib.csk_cell_list(_dev(counts, torch.int32), counts.numel(), min_count, bm, None, 0,
                                     C.byref(total), _stream(stream)))
            cap = total.value
        out = torch.empty(max(cap, 1), dtype=torch.int64, device=counts.device)
    else:
        cap = out.numel()
    _check(lib.csk_cell_list(_dev(counts, torch.int32), counts.numel(), min_count, bm, _dev(out, torch.int64), cap,
                             C.byref(total), _stream(stream)))
    if grow and total.value > cap:
        out = torch.empty(total.value, dtype=torch.int64, device=counts.device)
        return cell_list(counts, min_count, stream=stream, out=out, bitmap=bitmap)
    return out[:min(cap, total.value)]


def cells_clear(counts, bitmap, stream=None):
    """Zero the counts of the cells marked in bitmap, then the bitmap."""
    import torch
    _check(load_library().csk_cells_clear(_dev(counts, torch.int32), _dev(bitmap, torch.int32), counts.numel(),
                                          _stream(stream)))


def cell_labels(cells, fine_keys, delta, L, factor, stream=None):
    import torch
    labels = torch.empty(cells.shape[0], dtype=torch.float32, device=cells.device)
    if cells.shape[0]:
        _check(load_library().csk_cell_labels(_dev(cells, torch.int64), cells.shape[0],
                                              _dev(fine_keys, torch.int64) if fine_keys.shape[0] else None,
                                              fine_keys.shape[0], delta, L, factor, _dev(labels, torch.float32),
                                              _stream(stream)))
    return labels


# ---- the routed step without host synchronization: device counts, caller-held buffers

def _workspace(nbytes, device):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def cell_list_workspace_bytes(ncells):
    need = C.c_uint64(0)
    _check(load_library().csk_cell_list_workspace(ncells, C.byref(need)))
    return need.value


def cell_list_async(counts, out, total, min_count=1, bitmap=None, workspace=None, stream=None):
    """The cells with counts >= min_count into out (device int64; the first out.numel() of
    them, ascending) and their number into total (device int64 [1]), with no host
    synchronization.  workspace: device uint8 of cell_list_workspace_bytes(counts.numel())."""
    import torch
    if workspace is None:
        workspace = _workspace(cell_list_workspace_bytes(counts.numel()), counts.device)
    _check(load_library().csk_cell_list_async(_dev(counts, torch.int32), counts.numel(), min_count,
                                              _dev(bitmap, torch.int32) if bitmap is not None else None,
                                              _dev(out, torch.int64), out.numel(), _dev(total, torch.int64),
                                              workspace.data_ptr(), workspace.numel(), _stream(stream)))


def route_score(mlp, counts, delta_c, L, cells, m, logits, stream=None):
    """fp32 logits of cells[0 .. min(m, cells.numel())) (m: device int64 [1]) from their
    features, in one kernel."""
    import torch
    _check(load_library().csk_route_score(mlp.h, _dev(counts, torch.int32), delta_c, L, _dev(cells, torch.int64),
                                          _dev(m, torch.int64), cells.numel(), _dev(logits, torch.float32),
                                          _stream(stream)))


def route_admit_workspace_bytes(cap, A):
    need = C.c_uint64(0)
    _check(load_library().csk_route_admit_workspace(cap, A, C.byref(need)))
    return need.value


def route_admit_async(cells, logits, m, A, admitted, na, workspace=None, stream=None):
    """The min(A, m) best cells (m: device int64 [1]) into admitted (device int64 [A],
    ascending) and their number into na (device int32 [1])."""
    import torch
    cap = cells.numel()
    if workspace is None:
        workspace = _workspace(route_admit_workspace_bytes(cap, A), cells.device)
    _check(load_library().csk_route_admit_async(_dev(cells, torch.int64), _dev(logits, torch.float32),
                                                _dev(m, torch.int64), cap, A, _dev(admitted, torch.int64),
                                                _dev(na, torch.int32), workspace.data_ptr(), workspace.numel(),
                                                _stream(stream)))


def route_update_workspace_bytes(factor, table_slots):
    need = C.c_uint64(0)
    _check(load_library().csk_route_update_workspace(factor, table_slots, C.byref(need)))
    return need.value


def update_routed(sketch, pos, delta, L, factor, admitted, na, table_keys, table_counts, err, workspace=None,
                  stream=None):
    """Add pos to sketch except the particles of the admitted coarse cells (admitted[0 .. na),
    na device int32 [1]), which go to the exact table (cleared by the caller)."""
    import torch
    if workspace is None:
        workspace = _workspace(route_update_workspace_bytes(factor, table_keys.shape[0]), pos.device)
    n = pos.shape[0]
    _check(load_library().csk_sketch_update_routed(sketch.h, _dev(pos, torch.float32, 3) if n else None, n, delta, L,
                                                   factor, _dev(admitted, torch.int64), _dev(na, torch.int32),
                                                   _dev(table_keys, torch.int64), _dev(table_counts, torch.int32),
                                                   table_keys.shape[0], _dev(err, torch.int32), workspace.data_ptr(),
                                                   workspace.numel(), _stream(stream)))


def topk_with_table_async(sketch, table_keys, table_counts, k, keys, est, out, stream=None):
    """As topk_with_table into keys / est (device, >= k), out (device int32 [2]) = (number
    written, 1 if incomplete), with no host synchronization."""
    import torch
    _check(load_library().csk_topk_with_table_async(sketch.h, _dev(table_keys, torch.int64),
                                                    _dev(table_counts, torch.int32), table_keys.shape[0], k,
                                                    _dev(keys, torch.int64), _dev(est, torch.int32),
                                                    _dev(out, torch.int32), _stream(stream)))


def route_admit(cells, logits, A, stream=None):
    """Ascending device int64 keys of the min(A, m) cells with the highest logits."""
    import torch
    out = torch.empty(max(A, 1), dtype=torch.int64, device=cells.device)
    na = C.c_uint32(0)
    m = cells.shape[0]
    _check(load_library().csk_route_admit(_dev(cells, torch.int64) if m else None,
                                          _dev(logits, torch.float32) if m else None, m, A,
                                          _dev(out, torch.int64), C.byref(na), _stream(stream)))
    return out[:na.value]
