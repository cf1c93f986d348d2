"""CPU oracle for the streaming Count-Sketch halo-finder hot path (arXiv:1711.00975).

TEST INFRASTRUCTURE ONLY: this package is loaded by the test suite, the smoke
check and the CPU-baseline leg of the benchmark.  The product library never
imports it and shares no code with it.

Thin ctypes marshalling over ``csk_oracle.c`` (plain C): every computation lives
in that file; this module only converts numpy arrays to pointers.
"""
from __future__ import annotations

import ctypes as C
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsk_oracle.so")

OK = 0
W_INCOMPLETE = 1
E_INVALID = -1
E_DOMAIN = -5
VARIANT_CS = 0
VARIANT_CM = 1
INT32_MIN = -(2 ** 31)

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    u64, i64, u32, i32, f64 = C.c_uint64, C.c_int64, C.c_uint32, C.c_int32, C.c_double
    sig = {
        "orc_grid": (C.c_int, [f64, f64, P]),
        "orc_in_domain": (C.c_int, [C.c_float, f64]),
        "orc_cell_index": (C.c_int, [C.c_float, i64, f64, P]),
        "orc_cell_index_many": (None, [P, u64, i64, f64, P]),
        "orc_cell_key": (C.c_int, [P, i64, f64, P]),
        "orc_keys": (i64, [P, u64, f64, f64, P]),
        "orc_splitmix64_next": (u64, [P]),
        "orc_hash_tables": (None, [u64, u32, P]),
        "orc_row_hash": (u32, [P, u32, u64]),
        "orc_row_hash_many": (None, [P, u32, P, u64, P]),
        "orc_bucket": (u32, [u32, u32]),
        "orc_sign": (i32, [u32]),
        "orc_sketch_update": (i64, [P, P, u32, u32, C.c_int, P, u64, f64, f64]),
        "orc_estimate": (None, [P, P, u32, u32, C.c_int, P, u64, P]),
        "orc_histogram": (i64, [P, u64, P, P]),
        "orc_topk_sketch": (i64, [P, P, u32, u32, C.c_int, P, u64, f64, f64, i32, u64, P, P, P]),
        "orc_topk_exact": (i64, [P, P, u64, u64, P, P]),
        "orc_topk_dictionary": (i64, [P, P, u32, u32, C.c_int, i64, i32, u64, P, P, P]),
        "orc_sketch_update_keys": (None, [P, P, u32, u32, C.c_int, P, u64]),
        "orc_topk_hierarchical": (i64, [P, P, u32, u32, P, P, u32, u32, C.c_int, i64, u64, i32, i32, u64,
                                        P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def _pos(pos) -> np.ndarray:
    a = np.ascontiguousarray(pos, dtype=np.float32)
    assert a.ndim == 2 and a.shape[1] == 3, "positions are float32 [n][3]"
    return a


def grid(delta: float, L: float) -> int:
    G = C.c_int64(0)
    if _load().orc_grid(delta, L, C.byref(G)) != OK:
        raise ValueError(f"invalid mesh delta={delta} L={L}")
    return G.value


def in_domain(p: float, L: float) -> bool:
    return bool(_load().orc_in_domain(p, L))


def cell_index(p: float, G: int, L: float) -> int:
    """Exact floor(p*G/L) wrapped into [0, G); -1 outside the domain."""
    i = C.c_int64(0)
    rc = _load().orc_cell_index(C.c_float(p), G, L, C.byref(i))
    return i.value if rc == OK else -1


def cell_index_many(p, G: int, L: float) -> np.ndarray:
    a = np.ascontiguousarray(p, dtype=np.float32).ravel()
    out = np.empty(a.size, dtype=np.int64)
    _load().orc_cell_index_many(_p(a), a.size, G, L, _p(out))
    return out


def keys(pos, delta: float, L: float) -> np.ndarray:
    """Cell keys of the in-domain particles, in stream order."""
    a = _pos(pos)
    out = np.empty(max(a.shape[0], 1), dtype=np.uint64)
    m = _load().orc_keys(_p(a), a.shape[0], delta, L, _p(out))
    if m < 0:
        raise ValueError("invalid mesh")
    return out[:m].copy()


PACK_BITS = 21
PACK_OUTSIDE = np.uint64(2 ** 64 - 1)


def pack(pos, L: float) -> np.ndarray:
    """The packed stream (Sec. 4.1: three coordinates in 64 bits): word = qx | qy << 21 |
    qz << 42 with q = floor(p * 2^21 / L) exactly, wrapped as for the cell index (the cell
    index of a mesh of 2^21 cells); all ones when the particle is outside the domain.
    orc_cell_index's 128-bit arithmetic covers G = 2^21: |mantissa * G| < 2^45."""
    a = _pos(pos)
    q = cell_index_many(a.ravel(), 1 << PACK_BITS, L).reshape(-1, 3)
    out = np.full(a.shape[0], PACK_OUTSIDE, dtype=np.uint64)
    ok = (q >= 0).all(axis=1)
    qq = q[ok].astype(np.uint64)
    out[ok] = qq[:, 0] | (qq[:, 1] << np.uint64(PACK_BITS)) | (qq[:, 2] << np.uint64(2 * PACK_BITS))
    return out


def keys_packed(words, delta: float, L: float) -> np.ndarray:
    """Cell keys of the in-domain packed particles, in stream order: i = floor(q G / 2^21)."""
    G = np.uint64(grid(delta, L))
    w = np.ascontiguousarray(words, dtype=np.uint64)
    w = w[(w >> np.uint64(63)) == 0]
    mask = np.uint64((1 << PACK_BITS) - 1)
    i = [(((w >> np.uint64(sh)) & mask) * G) >> np.uint64(PACK_BITS) for sh in (0, PACK_BITS, 2 * PACK_BITS)]
    return (i[0] * G + i[1]) * G + i[2]


def topk_keys(M, T, keys_, theta, k, variant: int = VARIANT_CS):
    """Top-k over the distinct keys of a key stream: those with estimate >= theta, ordered by
    (estimate desc, key asc).  Returns (keys, est)."""
    uniq = np.unique(np.ascontiguousarray(keys_, dtype=np.uint64))
    est = estimate(M, T, uniq, variant) if uniq.size else np.empty(0, np.int32)
    sel = est.astype(np.int64) >= theta
    u, e = uniq[sel], est[sel]
    order = np.lexsort((u, -e.astype(np.int64)))[:k]
    return u[order], e[order]


def splitmix64(seed: int, count: int) -> np.ndarray:
    st = C.c_uint64(seed)
    lib = _load()
    return np.array([lib.orc_splitmix64_next(C.byref(st)) for _ in range(count)], dtype=np.uint64)


def hash_tables(seed: int, d: int) -> np.ndarray:
    T = np.empty((d, 6, 256), dtype=np.uint32)
    _load().orc_hash_tables(seed, d, _p(T))
    return T


def row_hash(T: np.ndarray, r: int, keys_) -> np.ndarray:
    k = np.ascontiguousarray(keys_, dtype=np.uint64).ravel()
    out = np.empty(k.size, dtype=np.uint32)
    _load().orc_row_hash_many(_p(np.ascontiguousarray(T)), r, _p(k), k.size, _p(out))
    return out


def bucket(h: int, w: int) -> int:
    return int(_load().orc_bucket(h, w))


def sign(h: int) -> int:
    return int(_load().orc_sign(h))


def sketch_update(M: np.ndarray, T: np.ndarray, pos, delta: float, L: float,
                  variant: int = VARIANT_CS) -> int:
    """Add every in-domain particle to M (int32 [d][w], in place). Returns #skipped."""
    assert M.dtype == np.int32 and M.ndim == 2 and M.flags["C_CONTIGUOUS"]
    d, w = M.shape
    a = _pos(pos)
    sk = _load().orc_sketch_update(_p(M), _p(np.ascontiguousarray(T)), d, w, variant,
                                   _p(a), a.shape[0], delta, L)
    if sk < 0:
        raise ValueError("invalid mesh or sketch shape")
    return int(sk)


def sketch(pos, d: int, w: int, seed: int, delta: float, L: float,
           variant: int = VARIANT_CS, threads: int = 1):
    """Counters of the whole stream.  With threads > 1 the stream is cut into
    contiguous ranges, each range gets its own zeroed sketch, and the sketches are
    summed modulo 2^32 (counters are linear in the stream, Sec. 5)."""
    T = hash_tables(seed, d)
    a = _pos(pos)
    n = a.shape[0]
    if threads <= 1 or n < 4096:
        M = np.zeros((d, w), dtype=np.int32)
        skipped = sketch_update(M, T, a, delta, L, variant)
        return M, skipped
    bounds = np.linspace(0, n, threads + 1).astype(np.int64)

    def part(i):
        Mi = np.zeros((d, w), dtype=np.int32)
        sk = sketch_update(Mi, T, a[bounds[i]:bounds[i + 1]], delta, L, variant)
        return Mi, sk

    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(part, range(threads)))
    M = np.zeros((d, w), dtype=np.int32)
    skipped = 0
    for Mi, sk in parts:
        M = (M.view(np.uint32) + Mi.view(np.uint32)).view(np.int32)
        skipped += sk
    return M, skipped


def estimate(M: np.ndarray, T: np.ndarray, keys_, variant: int = VARIANT_CS) -> np.ndarray:
    d, w = M.shape
    k = np.ascontiguousarray(keys_, dtype=np.uint64).ravel()
    out = np.empty(k.size, dtype=np.int32)
    _load().orc_estimate(_p(np.ascontiguousarray(M)), _p(np.ascontiguousarray(T)), d, w, variant,
                         _p(k), k.size, _p(out))
    return out


def histogram(keys_):
    k = np.ascontiguousarray(keys_, dtype=np.uint64).ravel()
    uniq = np.empty(max(k.size, 1), dtype=np.uint64)
    cnt = np.empty(max(k.size, 1), dtype=np.int64)
    m = _load().orc_histogram(_p(k), k.size, _p(uniq), _p(cnt))
    return uniq[:m].copy(), cnt[:m].copy()


def topk_sketch(M, T, pos, delta, L, theta, k, variant=VARIANT_CS):
    """Returns (keys, est, status)."""
    d, w = M.shape
    a = _pos(pos)
    ko = np.empty(max(k, 1), dtype=np.uint64)
    eo = np.empty(max(k, 1), dtype=np.int32)
    st = C.c_int32(0)
    m = _load().orc_topk_sketch(_p(np.ascontiguousarray(M)), _p(np.ascontiguousarray(T)), d, w,
                                variant, _p(a), a.shape[0], delta, L, theta, k,
                                _p(ko), _p(eo), C.byref(st))
    return ko[:m].copy(), eo[:m].copy(), st.value


def topk_dictionary(M, T, G, theta, k, variant=VARIANT_CS):
    """Top-k over every key of the G^3 mesh (CSFS).  Returns (keys, est, status)."""
    d, w = M.shape
    Mc = np.ascontiguousarray(M, dtype=np.int32)
    Tc = np.ascontiguousarray(T, dtype=np.uint32)
    ko = np.empty(max(k, 1), dtype=np.uint64)
    eo = np.empty(max(k, 1), dtype=np.int32)
    st = C.c_int32(0)
    m = _load().orc_topk_dictionary(_p(Mc), _p(Tc), d, w, variant, G, theta, k, _p(ko), _p(eo), C.byref(st))
    return ko[:m].copy(), eo[:m].copy(), st.value


def sketch_keys(keys_, d, w, seed, variant=VARIANT_CS):
    """Counters of a stream of item keys (uint64), each added once (Sec. 2.2 Add)."""
    T = hash_tables(seed, d)
    k = np.ascontiguousarray(keys_, dtype=np.uint64).ravel()
    M = np.zeros((d, w), dtype=np.int32)
    _load().orc_sketch_update_keys(_p(M), _p(T), d, w, variant, _p(k), k.size)
    return M


def super_sketch(pos, d, w, seed, delta, L, group, variant=VARIANT_CS):
    """Counters of the super-item stream key // group (the coarse layer of the hierarchy).
    Particles outside the domain are skipped, as in sketch()."""
    return sketch_keys(keys(pos, delta, L) // np.uint64(group), d, w, seed, variant)


def topk_hierarchical(M1, T1, M2, T2, G, group, theta1, theta2, k, variant=VARIANT_CS):
    """Count Sketch Hierarchical query (Alg. 3).  Returns (keys, est, status)."""
    d1, w1 = M1.shape
    d2, w2 = M2.shape
    a1, b1 = np.ascontiguousarray(M1, dtype=np.int32), np.ascontiguousarray(T1, dtype=np.uint32)
    a2, b2 = np.ascontiguousarray(M2, dtype=np.int32), np.ascontiguousarray(T2, dtype=np.uint32)
    ko = np.empty(max(k, 1), dtype=np.uint64)
    eo = np.empty(max(k, 1), dtype=np.int32)
    st = C.c_int32(0)
    m = _load().orc_topk_hierarchical(_p(a1), _p(b1), d1, w1, _p(a2), _p(b2), d2, w2, variant, G, group, theta1,
                                      theta2, k, _p(ko), _p(eo), C.byref(st))
    return ko[:m].copy(), eo[:m].copy(), st.value


def topk_exact(uniq, count, k):
    u = np.ascontiguousarray(uniq, dtype=np.uint64)
    c = np.ascontiguousarray(count, dtype=np.int64)
    ko = np.empty(max(k, 1), dtype=np.uint64)
    co = np.empty(max(k, 1), dtype=np.int64)
    m = _load().orc_topk_exact(_p(u), _p(c), u.size, k, _p(ko), _p(co))
    return ko[:m].copy(), co[:m].copy()
