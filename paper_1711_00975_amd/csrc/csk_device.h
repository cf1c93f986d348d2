// csk_device.h — device-side building blocks shared by the csk kernels (gfx950).
//
// Mesh cell of a particle (Sec. 2.1; Sec. 3.1 stage 1), simple-tabulation row hashes
// (Sec. 2.2: t bucket hashes and t sign hashes), and the median of the signed row
// estimates (Sec. 2.2 Estimate; Alg. 4 Estimate).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csk {

constexpr int kChars = 6;              // keys < 2^48: six 8-bit characters
constexpr int kTableWords = kChars * 256;
constexpr int kSliceBits = 15;         // counters per accumulation slice = 2^15 (128 KiB of LDS)
constexpr uint32_t kSlice = 1u << kSliceBits;
constexpr uint64_t kEmptyKey = ~0ull;  // empty slot of the candidate set / invalid key
constexpr int kTabLdsRows = 8;         // rows whose tables are staged in LDS
constexpr int kFilterWords = 24576;    // LDS Bloom filter of hot (row, bucket, sign): 96 KiB
constexpr uint32_t kFilterMaxItems = kFilterWords * 32 / 6;  // denser filters are not used

// error latch bits (device word)
constexpr uint32_t kErrDomain = 1u;
constexpr uint32_t kErrCapacity = 2u;

struct Mesh {
  double L;       // box side
  double invL;    // binary64(1 / L)
  double twoL;    // domain bound: |p| < 2L
  double Gd;      // cells per side, as a double
  int32_t G;      // cells per side
};

// Exact cell index along one axis: floor(p * G / L) on the exact values, wrapped into
// [0, G).  p*G is exact in binary64 (24-bit significand times a 16-bit integer).  The
// quotient estimate floor((p*G) * (1/L)) is within one of the exact floor, because its
// relative error is a few ulp and |p*G/L| < 2^17; the sign of a single-rounded fma
// t - q*L equals the sign of the exact remainder, which fixes the estimate.
// Returns false for a non-finite p or |p| >= 2L.
__device__ __forceinline__ bool cell_index(float p, const Mesh& m, int32_t& out) {
  const double x = (double)p;
  if (!(__builtin_fabs(x) < m.twoL)) return false;
  const double t = x * m.Gd;
  double q = __builtin_floor(t * m.invL);
  if (__builtin_fma(-q, m.L, t) < 0.0) {
    q -= 1.0;
  } else if (__builtin_fma(-(q + 1.0), m.L, t) >= 0.0) {
    q += 1.0;
  }
  int32_t i = (int32_t)q;          // in [-2G, 2G)
  if (i < 0) i += m.G;
  if (i < 0) i += m.G;
  if (i >= m.G) i -= m.G;
  out = i;
  return true;
}

// Cell key (ix * G + iy) * G + iz of one particle; false if it is outside the domain.
__device__ __forceinline__ bool cell_key(float x, float y, float z, const Mesh& m, uint64_t& key) {
  int32_t ix = 0, iy = 0, iz = 0;
  const bool ok = (int)cell_index(x, m, ix) & (int)cell_index(y, m, iy) & (int)cell_index(z, m, iz);
  const uint32_t xy = (uint32_t)ix * (uint32_t)m.G + (uint32_t)iy;  // < G^2 <= 2^32
  key = (uint64_t)xy * (uint64_t)(uint32_t)m.G + (uint64_t)(uint32_t)iz;
  return ok;
}

// Tabulated word of row r: XOR over the six key bytes of T[r][c][byte_c].
// Table layout: row-major [r][c][256] uint32 (LDS or global).
__device__ __forceinline__ uint32_t row_hash(const uint32_t* __restrict__ tab_r, uint64_t key) {
  const uint32_t lo = (uint32_t)key, hi = (uint32_t)(key >> 32);
  uint32_t h = tab_r[0 * 256 + (lo & 255u)];
  h ^= tab_r[1 * 256 + ((lo >> 8) & 255u)];
  h ^= tab_r[2 * 256 + ((lo >> 16) & 255u)];
  h ^= tab_r[3 * 256 + (lo >> 24)];
  h ^= tab_r[4 * 256 + (hi & 255u)];
  h ^= tab_r[5 * 256 + ((hi >> 8) & 255u)];
  return h;
}

// Tabulated words of rows 0..DP-1 from row-interleaved tables Ti[c][v][DP] (DP = 4 or 8,
// 16-byte aligned rows): two (or one) 16-byte reads per key byte give every row at once.
template <int DP>
__device__ __forceinline__ void row_hashes(const uint32_t* __restrict__ ti, uint64_t key, uint32_t (&h)[DP]) {
  const uint32_t lo = (uint32_t)key, hi = (uint32_t)(key >> 32);
  const uint32_t byte[kChars] = {lo & 255u, (lo >> 8) & 255u, (lo >> 16) & 255u, lo >> 24, hi & 255u, (hi >> 8) & 255u};
#pragma unroll
  for (int r = 0; r < DP; ++r) h[r] = 0;
#pragma unroll
  for (int c = 0; c < kChars; ++c) {
    const uint4* e = (const uint4*)(ti + (c * 256 + byte[c]) * DP);
#pragma unroll
    for (int q = 0; q < DP / 4; ++q) {
      const uint4 v = e[q];
      h[4 * q + 0] ^= v.x;
      h[4 * q + 1] ^= v.y;
      h[4 * q + 2] ^= v.z;
      h[4 * q + 3] ^= v.w;
    }
  }
}

// Bucket hash: low 31 bits scaled onto [0, w).
__device__ __forceinline__ uint32_t bucket_of(uint32_t h, uint32_t w) {
  return (uint32_t)(((uint64_t)(h & 0x7FFFFFFFu) * (uint64_t)w) >> 31);
}

// Lower median (index floor((d-1)/2) of the ascending order) of v[0..d), d <= MAXD,
// by counting: v[i] is the answer when #{v < v[i]} <= m < #{v <= v[i]}.
template <int MAXD>
__device__ __forceinline__ int32_t lower_median(const int32_t (&v)[MAXD], int d) {
  const int m = (d - 1) >> 1;
  int32_t res = v[0];
#pragma unroll
  for (int i = 0; i < MAXD; ++i) {
    if (i < d) {
      int lt = 0, le = 0;
#pragma unroll
      for (int j = 0; j < MAXD; ++j) {
        if (j < d) {
          lt += (v[j] < v[i]);
          le += (v[j] <= v[i]);
        }
      }
      if (lt <= m && m < le) res = v[i];
    }
  }
  return res;
}

// Blocked Bloom filter over (row, bucket, sign) items: one 32-bit word, three bits.
struct FilterProbe {
  uint32_t word;
  uint32_t mask;
};

// 64-bit finaliser (MurmurHash3 fmix64) used only to place keys in the candidate set
// and items in the Bloom filter.
__device__ __forceinline__ uint64_t slot_mix(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// Probe of the filter for the item (row r, bucket b, sign bit neg): fmix32 of the item,
// word index from its high bits, three bit positions from a second multiply.
__device__ __forceinline__ FilterProbe filter_probe(uint32_t r, uint32_t b, uint32_t neg) {
  uint32_t x = ((b << 1) | neg) ^ (r * 0x9E3779B9u);
  x ^= x >> 16;
  x *= 0x85EBCA6Bu;
  x ^= x >> 13;
  x *= 0xC2B2AE35u;
  x ^= x >> 16;
  const uint32_t y = x * 0xCC9E2D51u;
  FilterProbe p;
  p.word = (uint32_t)(((uint64_t)x * (uint64_t)kFilterWords) >> 32);
  p.mask = (1u << (y >> 27)) | (1u << ((y >> 22) & 31u)) | (1u << ((y >> 17) & 31u));
  return p;
}

}  // namespace csk
