"""Seeded synthetic particle streams (Plummer halos + uniform background).

Stand-ins for the paper's Millennium (Sec. 4.1) and Millennium XXL (Sec. 4.5)
snapshots, which are not available.  The generator lives in ``plummer.c``; this
module marshals arguments and names the workload configurations.  It holds none
of the sketch method's arithmetic, so both the GPU library and the CPU oracle can
consume what it produces.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsk_workloads.so")
GPU_LIB_PATH = os.path.join(HERE, "libcsk_workloads_gpu.so")
_lib = None
_gpu_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    P, u64, u32, f64, i64 = C.c_void_p, C.c_uint64, C.c_uint32, C.c_double, C.c_int64
    lib.wl_philox4x32_10.restype = None
    lib.wl_philox4x32_10.argtypes = [P, P, P]
    lib.wl_philox_words.restype = None
    lib.wl_philox_words.argtypes = [u64, u64, u32, u64, P]
    lib.wl_halo_catalogue.restype = None
    lib.wl_halo_catalogue.argtypes = [u64, u32, f64, f64, f64, f64, P, P]
    lib.wl_gen_exact.restype = i64
    lib.wl_gen_exact.argtypes = [u64, f64, u32, f64, f64, f64, f64, u64, P, C.c_int]
    lib.wl_gen_mixture.restype = i64
    lib.wl_gen_mixture.argtypes = [u64, u64, f64, u32, f64, f64, f64, f64, f64, u64, P, C.c_int]
    lib.wl_alias_records.restype = i64
    lib.wl_alias_records.argtypes = [u64, u32, f64, f64, f64, f64, P]
    _lib = lib
    return lib


def _p(a):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    _load().wl_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def philox_words(index0: int, n: int, stream: int, seed: int) -> np.ndarray:
    """Words index0 .. index0 + n - 1 of the Philox4x32-10 output stream: word g is word g mod 4
    of the counter (g / 4, stream, 0)."""
    out = np.empty(max(n, 1), dtype=np.uint32)
    _load().wl_philox_words(index0, n, stream, seed, _p(out))
    return out[:n]


@dataclass(frozen=True)
class Workload:
    """One synthetic stream and the sketch parameters it is measured with."""
    name: str
    n: int                 # particles
    L: float               # box side (Mpc/h)
    delta: float           # cell side (Mpc/h)
    d: int                 # sketch rows (t in the paper)
    w: int                 # counters per row (b in the paper)
    k: int                 # heavy cells wanted
    seed: int
    n_halo: int
    m_lo: float
    m_hi: float
    slope: float = 1.9
    a: float = 0.2         # Plummer scale radius (Mpc/h)
    f_bg: float = -1.0     # < 0: exact-count recipe (halo j gets floor(M_j) particles, rest uniform)
    chunk: int = 0         # particles per generated chunk (0: one piece)
    extra: dict = field(default_factory=dict)

    def generate(self, start: int = 0, count: int | None = None, out: np.ndarray | None = None,
                 threads: int = 0) -> np.ndarray:
        """float32 [count][3] positions of particles [start, start + count).  threads > 0 caps
        the generator's OpenMP threads (1 when several generators run at once)."""
        if count is None:
            count = self.n - start
        if out is None:
            out = np.empty((count, 3), dtype=np.float32)
        assert out.shape == (count, 3) and out.dtype == np.float32
        lib = _load()
        if self.f_bg < 0:
            assert start == 0 and count == self.n, "exact-count recipe is generated whole"
            lib.wl_gen_exact(self.n, self.L, self.n_halo, self.m_lo, self.m_hi, self.slope, self.a,
                             self.seed, _p(out), threads)
        else:
            lib.wl_gen_mixture(start, count, self.L, self.n_halo, self.m_lo, self.m_hi, self.slope,
                               self.a, self.f_bg, self.seed, _p(out), threads)
        return out

    def with_(self, **kw) -> "Workload":
        d = dict(self.__dict__)
        d.update(kw)
        return Workload(**d)


# 2^20 particles, L = 100 Mpc/h, 256 Plummer halos (a = 0.2), masses ~ M^-1.9 on
# [100, 1e4], remainder uniform; cell 0.1 Mpc/h (1000^3 cells), d = 5, w = 2^16, k = 100.
SMALL = Workload(name="plummer-2^20-L100-d0.1-w2^16", n=1 << 20, L=100.0, delta=0.1, d=5,
                 w=1 << 16, k=100, seed=1, n_halo=256, m_lo=100.0, m_hi=1.0e4)

# 2^30 particles in 2^26-particle chunks, L = 1000 Mpc/h, 2^20 halos with masses
# ~ M^-1.9 on [50, 1e6], 30 % uniform background; cell 0.25 Mpc/h (4000^3 cells),
# d = 5, w = 2^24, k = 1e4.
SCALE = Workload(name="plummer-2^30-L1000-d0.25-w2^24", n=1 << 30, L=1000.0, delta=0.25, d=5,
                 w=1 << 24, k=10_000, seed=1, n_halo=1 << 20, m_lo=50.0, m_hi=1.0e6, f_bg=0.3,
                 chunk=1 << 26)


def halo_catalogue(wl: Workload):
    mass = np.empty(wl.n_halo, dtype=np.float64)
    cen = np.empty((wl.n_halo, 3), dtype=np.float64)
    _load().wl_halo_catalogue(wl.seed, wl.n_halo, wl.L, wl.m_lo, wl.m_hi, wl.slope, _p(mass), _p(cen))
    return mass, cen


def batch_subvolumes(count: int = 64, seed: int = 1) -> list:
    """The batched-update workload: `count` independent sub-volumes of uneven size.

    Sub-volume s: u_s = (first Philox4x32-10 word of counter (s, 0, 3, 0) under `seed`) / 2^32,
    n_s = floor(2^(16 + 8 u_s)) particles (2^16 .. 2^24), L = 100, delta = 0.1,
    w_s = 2^(14 + round(6 (log2 n_s - 16) / 8)) (2^14 .. 2^20), d = 5, k_s = floor(0.01 w_s),
    max(1, round(256 n_s / 2^20)) Plummer halos with masses on [100, 1e4], the rest uniform
    (the exact-count recipe of SMALL), seed 1 + s.
    """
    out = []
    for s in range(count):
        u = int(philox4x32_10([s, 0, 3, 0], [seed & 0xFFFFFFFF, seed >> 32])[0]) / 2.0 ** 32
        n = int(np.floor(2.0 ** (16.0 + 8.0 * u)))
        w = 1 << (14 + int(round(6.0 * (np.log2(n) - 16.0) / 8.0)))
        out.append(Workload(name=f"subvolume-{s}", n=n, L=100.0, delta=0.1, d=5, w=w, k=max(1, w // 100),
                            seed=1 + s, n_halo=max(1, int(round(256 * n / 2 ** 20))), m_lo=100.0, m_hi=1.0e4))
    return out


def _load_gpu():
    global _gpu_lib
    if _gpu_lib is None:
        if not os.path.exists(GPU_LIB_PATH):
            raise RuntimeError(f"{GPU_LIB_PATH} is missing: build the workloads first")
        lib = C.CDLL(GPU_LIB_PATH)
        lib.wl_gen_mixture_device.restype = C.c_int
        lib.wl_gen_mixture_device.argtypes = [C.c_uint64, C.c_uint64, C.c_double, C.c_uint32, C.c_double,
                                              C.c_double, C.c_uint64, C.c_double, C.c_void_p, C.c_void_p,
                                              C.c_void_p]
        _gpu_lib = lib
    return _gpu_lib


class DeviceGenerator:
    """The mixture recipe generated on the GPU, chunk by chunk (plummer_gpu.hip): the same
    draws and alias records as Workload.generate, written straight into device memory."""

    def __init__(self, wl: Workload):
        import torch
        if wl.f_bg < 0:
            raise ValueError("the device generator implements the mixture recipe only")
        self.wl = wl
        rec = np.zeros((max(wl.n_halo, 1), 8), dtype=np.float64)
        _load().wl_alias_records(wl.seed, wl.n_halo, wl.L, wl.m_lo, wl.m_hi, wl.slope, _p(rec))
        self.rec = torch.from_numpy(rec).cuda()
        self.u_max = 1.01 ** -1.5

    def generate(self, start: int, count: int, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((count, 3), dtype=torch.float32, device="cuda")
        assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous() and out.shape[0] >= count
        s = stream.cuda_stream if stream is not None else torch.cuda.current_stream().cuda_stream
        rc = _load_gpu().wl_gen_mixture_device(start, count, self.wl.L, self.wl.n_halo, self.wl.a, self.wl.f_bg,
                                               self.wl.seed, self.u_max, self.rec.data_ptr(), out.data_ptr(), s)
        if rc != 0:
            raise RuntimeError(f"device generator launch failed ({rc})")
        return out[:count]


# 2^34 particles in 2^27-particle chunks, L = 3000 Mpc/h, 2^24 halos (masses ~ M^-1.9 on
# [50, 1e6]), 30 % uniform background; three meshes 0.25 / 0.5 / 1.0 Mpc/h, d = 5,
# w = 2^24 each, k = 1e5.  Generated on the device.
LARGE = Workload(name="plummer-2^34-L3000-d0.25/0.5/1.0-w2^24", n=1 << 34, L=3000.0, delta=0.25, d=5,
                 w=1 << 24, k=100_000, seed=1, n_halo=1 << 24, m_lo=50.0, m_hi=1.0e6, f_bg=0.3,
                 chunk=1 << 27)
