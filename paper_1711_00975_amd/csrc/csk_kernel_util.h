// csk_kernel_util.h — device helpers shared by the update kernels and the query,
// collect and top-k kernels (wave scans, appends, tabulated estimates, table staging).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csk_internal.h"

namespace csk {

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane >= (uint32_t)o) v += t;
  }
  return v;
}

// Wave-aggregated append: every lane of the wave must call it.  Returns the slot of a
// lane with pred set.
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, bool pred) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return 0;
  const uint32_t lane = lane_id();
  const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1u;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
  base = __shfl(base, (int)leader, 64);
  const uint64_t below = (lane == 0) ? 0ull : (mask & ((~0ull) >> (64 - lane)));
  return base + (uint32_t)__popcll(below);
}

// Exclusive scan of in[0..n) into out[0..n) by a block of NT threads; total -> *total.
// Contains barriers: every thread of the block must call it.
template <int NT>
__device__ __forceinline__ void block_exclusive_scan(const uint32_t* in, uint32_t* out, uint32_t n,
                                                     uint32_t* wsum, uint32_t* total) {
  constexpr int NW = NT / 64;
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (n + NT - 1) / NT;
  const uint32_t lo = min(n, tid * per), hi = min(n, lo + per);
  uint32_t s = 0;
  for (uint32_t i = lo; i < hi; ++i) s += in[i];
  const uint32_t incl = wave_incl_scan(s);
  const uint32_t wave = tid >> 6;
  if (lane_id() == 63) wsum[wave] = incl;
  __syncthreads();
  if (tid == 0) {
    uint32_t acc = 0;
    for (int w = 0; w < NW; ++w) {
      const uint32_t t = wsum[w];
      wsum[w] = acc;
      acc += t;
    }
    *total = acc;
  }
  __syncthreads();
  uint32_t run = wsum[wave] + incl - s;
  for (uint32_t i = lo; i < hi; ++i) {
    out[i] = run;
    run += in[i];
  }
  __syncthreads();
}

// Signed estimate of one row: M * sign (Count-Min: M), modulo 2^32.
__device__ __forceinline__ int32_t row_estimate(const uint32_t* tab_r, const int32_t* __restrict__ Mr,
                                                uint32_t w, uint32_t cm, uint64_t key) {
  const uint32_t h = row_hash(tab_r, key);
  const uint32_t c = (uint32_t)Mr[bucket_of(h, w)];
  const uint32_t neg = (h >> 31) & (cm ^ 1u);
  return (int32_t)(neg ? (0u - c) : c);
}

template <int MAXD>
__device__ __forceinline__ int32_t estimate_key(const uint32_t* tabs, const int32_t* __restrict__ M,
                                                uint32_t d, uint32_t w, uint32_t cm, uint64_t key) {
  int32_t v[MAXD];
#pragma unroll
  for (int r = 0; r < MAXD; ++r) {
    v[r] = ((uint32_t)r < d) ? row_estimate(tabs + r * kTableWords, M + (uint64_t)r * w, w, cm, key) : 0;
  }
  if (cm) {
    int32_t mn = v[0];
#pragma unroll
    for (int r = 1; r < MAXD; ++r)
      if ((uint32_t)r < d) mn = min(mn, v[r]);
    return mn;
  }
  return lower_median<MAXD>(v, (int)d);
}

// Stage the tables of the first `rows` rows in LDS.
__device__ __forceinline__ void load_tables(uint32_t* dst, const uint32_t* __restrict__ src, uint32_t rows) {
  for (uint32_t i = threadIdx.x; i < rows * kTableWords; i += blockDim.x) dst[i] = src[i];
}

// ------------------------------------------------------------------ candidate set

// Longest probe sequence of the candidate set.  Inserts stop at max_candidates, so the
// table (2^ceil(log2(2 max_candidates)) slots) stays at most about half full and real
// probe runs are far shorter; the cap only bounds the work when the set is over capacity.
constexpr uint32_t kMaxProbe = 4096;

// Is key already in the candidate set?  (A stale read can only miss a key.)
__device__ __forceinline__ bool set_contains(const uint64_t* set, uint32_t mask, uint64_t key) {
  uint32_t i = (uint32_t)slot_mix(key) & mask;
  for (uint32_t probe = 0; probe <= mask && probe < kMaxProbe; ++probe) {
    const uint64_t cur = set[i];
    if (cur == key) return true;
    if (cur == kEmptyKey) return false;
    i = (i + 1) & mask;
  }
  return false;
}

__device__ __forceinline__ void set_insert(uint64_t* set, uint32_t mask, uint64_t key, uint32_t* count,
                                           uint32_t max_cand, uint32_t* err) {
  uint32_t i = (uint32_t)slot_mix(key) & mask;
  for (uint32_t probe = 0; probe <= mask && probe < kMaxProbe; ++probe) {
    // A slot only ever changes from empty to a key, so a stale read can only show
    // "empty"; the compare-and-swap then tells the truth.
    const uint64_t cur = set[i];
    if (cur == key) return;
    if (cur == kEmptyKey) {
      // a new key: once the set holds max_candidates keys no more go in (capacity error)
      if (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= max_cand) {
        atomicOr(err, kErrCapacity);
        return;
      }
      const uint64_t old = atomicCAS((unsigned long long*)&set[i], (unsigned long long)kEmptyKey,
                                     (unsigned long long)key);
      if (old == kEmptyKey) {
        if (atomicAdd(count, 1u) >= max_cand) atomicOr(err, kErrCapacity);
        return;
      }
      if (old == key) return;
    }
    i = (i + 1) & mask;
  }
  atomicOr(err, kErrCapacity);
}

// ---- the admitted coarse cells of the learned router: an LDS hash of their keys (load at
// most 1/2) that maps a key to its position in the admitted list.
constexpr uint64_t kAdmEmpty = ~0ull;

__device__ __forceinline__ uint32_t adm_hash(uint64_t key) {
  return ((uint32_t)(key ^ (key >> 32)) * 0x9E3779B9u) >> 22;   // top 10 bits: kAdmHashSlots
}

// Fill the hash with admitted[0 .. na) (na <= kAdmHashSlots / 2, distinct keys); every thread
// of the block calls it; ends with a barrier.
__device__ __forceinline__ void adm_hash_fill(const uint64_t* __restrict__ admitted, uint32_t na, uint64_t* hkey,
                                              uint16_t* hidx) {
  for (uint32_t i = threadIdx.x; i < kAdmHashSlots; i += blockDim.x) hkey[i] = kAdmEmpty;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < na; i += blockDim.x) {
    const uint64_t key = admitted[i];
    uint32_t sl = adm_hash(key);
    for (uint32_t probe = 0; probe < kAdmHashSlots; ++probe) {
      if (atomicCAS((unsigned long long*)&hkey[sl], kAdmEmpty, (unsigned long long)key) == kAdmEmpty) {
        hidx[sl] = (uint16_t)i;
        break;
      }
      sl = (sl + 1) & (kAdmHashSlots - 1);
    }
  }
  __syncthreads();
}

// ---- the exclusion's table (update kernels): keys at kExSlots slots, their positions, and
// a 2^16-bit prefilter (one bit per admitted key, under a second hash).  A particle whose
// bit is clear -- nearly every one outside the admitted cells -- stops after one LDS read.
struct ExLds {
  uint64_t* key;   // kExSlots
  uint16_t* idx;   // kExSlots
  uint32_t* bits;  // kExBitWords
};

// The table at the start of an LDS array of at least kExLdsWords words (8-byte aligned).
__device__ __forceinline__ ExLds ex_lds(uint32_t* base) {
  ExLds t;
  t.key = (uint64_t*)base;
  t.idx = (uint16_t*)(base + 2 * kExSlots);
  t.bits = base + 2 * kExSlots + kExSlots / 2;
  return t;
}

__device__ __forceinline__ uint32_t ex_fold(uint64_t key) { return (uint32_t)key ^ (uint32_t)(key >> 32); }
__device__ __forceinline__ uint32_t ex_slot(uint32_t x) { return (x * 0x9E3779B9u) >> 21; }   // 11 bits
__device__ __forceinline__ uint32_t ex_bit(uint32_t x) { return (x * 0x85EBCA77u) >> 16; }    // 16 bits

// Fill the table with admitted[0 .. na) (na <= kExSlots / 4, distinct keys); every thread
// of the block calls it; ends with a barrier.
__device__ __forceinline__ void ex_fill(const uint64_t* __restrict__ admitted, uint32_t na, const ExLds& t) {
  for (uint32_t i = threadIdx.x; i < kExSlots; i += blockDim.x) t.key[i] = kAdmEmpty;
  for (uint32_t i = threadIdx.x; i < kExBitWords; i += blockDim.x) t.bits[i] = 0u;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < na; i += blockDim.x) {
    const uint64_t key = admitted[i];
    const uint32_t x = ex_fold(key), b = ex_bit(x);
    atomicOr(&t.bits[b >> 5], 1u << (b & 31u));
    uint32_t sl = ex_slot(x);
    for (uint32_t probe = 0; probe < kExSlots; ++probe) {
      if (atomicCAS((unsigned long long*)&t.key[sl], kAdmEmpty, (unsigned long long)key) == kAdmEmpty) {
        t.idx[sl] = (uint16_t)i;
        break;
      }
      sl = (sl + 1) & (kExSlots - 1);
    }
  }
  __syncthreads();
}

// Position of coarse key ck in the admitted list, or -1.
__device__ __forceinline__ int32_t ex_find(uint64_t ck, const ExLds& t) {
  const uint32_t x = ex_fold(ck), b = ex_bit(x);
  if (((t.bits[b >> 5] >> (b & 31u)) & 1u) == 0u) return -1;
  uint32_t sl = ex_slot(x);
  for (uint32_t probe = 0; probe < kExSlots; ++probe) {
    const uint64_t k = t.key[sl];
    if (k == ck) return (int32_t)t.idx[sl];
    if (k == kAdmEmpty) return -1;
    sl = (sl + 1) & (kExSlots - 1);
  }
  return -1;
}

// Coarse key of the fine cell (ix, iy, iz) (each index < G <= 2^16) and the fine cell's
// position inside its coarse cell, (x * f + y) * f + z.
__device__ __forceinline__ uint64_t adm_coarse(int32_t ix, int32_t iy, int32_t iz, const RouteExclude& ex,
                                               uint32_t& child) {
  const uint32_t f = ex.factor;
  const uint32_t cx = __umulhi((uint32_t)ix, ex.fmagic), cy = __umulhi((uint32_t)iy, ex.fmagic),
                 cz = __umulhi((uint32_t)iz, ex.fmagic);
  child = (((uint32_t)ix - cx * f) * f + ((uint32_t)iy - cy * f)) * f + ((uint32_t)iz - cz * f);
  return ((uint64_t)cx * ex.gc + cy) * ex.gc + cz;
}

// The admitted count an exclusion uses: *na clamped to na_max (bit 2 of *err when above).
__device__ __forceinline__ uint32_t adm_count(const RouteExclude& ex) {
  const uint32_t na = *ex.na;
  if (na > ex.na_max) {
    if (threadIdx.x == 0) atomicOr(ex.err, 4u);
    return ex.na_max;
  }
  return na;
}

// A buffer resource over the bytes [base, base + bytes), bytes clamped to 2^32 - 16: a load at
// an offset past them returns 0.  Its last word (0x00020000) selects the raw 32-bit data
// format of gfx9 buffers.  With one resource per tile, a lane's byte offsets are the same
// for every tile, so the loads need no per-particle address arithmetic and no clamping.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t byte_span(const void* base, uint64_t bytes) {
  const uint32_t nrec = bytes > 0xFFFFFFF0ull ? 0xFFFFFFF0u : (uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)nrec, 0x00020000);
}

// The 12-byte record (x, y, z) at byte offset voff + soff of the span (voff per lane, soff
// the same for the whole wave), one nontemporal load.
__device__ __forceinline__ void load_xyz(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float& x, float& y,
                                         float& z) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b96(r, voff, (int)soff, 2);
  x = __uint_as_float(v[0]);
  y = __uint_as_float(v[1]);
  z = __uint_as_float(v[2]);
}

static inline uint32_t grid_for(uint64_t n, uint32_t threads, uint32_t max_blocks) {
  uint64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return (uint32_t)b;
}

}  // namespace csk
