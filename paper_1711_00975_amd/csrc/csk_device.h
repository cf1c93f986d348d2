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
constexpr uint32_t kHotSlots = 1u << 19;   // exact set of hot items: 2 MiB, stays in L2
constexpr uint32_t kHotMaxItems = kHotSlots / 2;
constexpr uint32_t kHotEmpty = 0xFFFFFFFFu;

// error latch bits (device word)
constexpr uint32_t kErrDomain = 1u;
constexpr uint32_t kErrCapacity = 2u;

struct Mesh {
  double L;       // box side
  double invL;    // binary64(1 / L)
  double twoL;    // domain bound: |p| < 2L
  double Gd;      // cells per side, as a double
  int32_t G;      // cells per side
  uint32_t nch;   // key bytes that can be non-zero (keys < G^3)
  uint32_t mode;  // kMeshGeneral, kMeshExactRatio or kMeshPow2Ratio
  double R;       // G / L when it is exact (modes 1, 2)
  float Rf;       // G / L as a float (mode 2: a power of two >= 1)
  float twoLf;    // 2L as a float (mode 2: exact)
  uint32_t group; // items are cell keys divided by `group` (1: the cell keys themselves)
  double ginv;    // binary64(1 / group)
};

// Item of a cell key: key / group exactly (the super-items of the hierarchical variant,
// Sec. 2.2 item 3; group 1 leaves the key alone).  key < 2^48, so key * (1/group) in
// binary64 is within 1/16 of the quotient and one correction step gives the floor.
__device__ __forceinline__ uint64_t group_key(uint64_t key, const Mesh& m) {
  if (m.group == 1u) return key;
  uint64_t q = (uint64_t)((double)key * m.ginv);
  const int64_t r = (int64_t)(key - q * (uint64_t)m.group);
  if (r < 0) --q;
  else if (r >= (int64_t)m.group) ++q;
  return q;
}

// How a mesh's cell index is computed (every mode gives floor(p * G / L) exactly):
//   general     floor estimate of p*G*(1/L) corrected by the signs of two fma residuals
//   exact ratio R = G/L is a double with at most 29 significant bits, so p*R is exact in
//               binary64 and floor(p*R) is the answer
//   pow2 ratio  R = 2^k, k >= 0, and 2L is a float: p*R is exact in binary32
constexpr uint32_t kMeshGeneral = 0;
constexpr uint32_t kMeshExactRatio = 1;
constexpr uint32_t kMeshPow2Ratio = 2;
// The stream is packed: one 64-bit word per particle holding three 21-bit fixed-point
// coordinates q = floor(p * 2^21 / L) (x in bits 0-20, y in 21-41, z in 42-62; all ones:
// outside the domain).  The cell index on a mesh of G cells is floor(q * G / 2^21).
constexpr uint32_t kMeshPacked = 3;
constexpr uint32_t kPackBits = 21;
constexpr uint64_t kPackedOutside = ~0ull;

// Exact cell index along one axis: floor(p * G / L) on the exact values, wrapped into
// [0, G).  p*G is exact in binary64 (24-bit significand times a 16-bit integer).  The
// quotient estimate q = floor((p*G) * (1/L)) is within one of the exact floor, because
// its relative error is a few ulp and |p*G/L| < 2^17; the signs of the single-rounded
// fma residuals t - q*L and t - (q+1)*L equal the signs of the exact ones and move q
// to the floor.  Branch-free; the result is meaningful only when it returns true
// (p finite and |p| < 2L).
template <uint32_t MODE>
__device__ __forceinline__ bool cell_index_m(float p, const Mesh& m, int32_t& out) {
  int32_t i;
  bool ok;
  if (MODE == kMeshPow2Ratio) {
    ok = __builtin_fabsf(p) < m.twoLf;
    // floor and conversion in one instruction, defined for every input (out-of-range
    // values clamp, NaN gives 0), so no select is needed for the particles that fail ok
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(i) : "v"(p * m.Rf));
  } else if (MODE == kMeshExactRatio) {
    const double x = (double)p;
    ok = __builtin_fabs(x) < m.twoL;
    // the conversion as one instruction, defined for every input (as above)
    asm("v_cvt_i32_f64 %0, %1" : "=v"(i) : "v"(__builtin_floor(x * m.R)));
  } else {
    const double x = (double)p;
    ok = __builtin_fabs(x) < m.twoL;
    const double t = x * m.Gd;
    const double q = __builtin_floor(t * m.invL);
    const double r0 = __builtin_fma(-q, m.L, t);
    const double r1 = __builtin_fma(-(q + 1.0), m.L, t);
    i = ok ? (int32_t)q : 0;  // in [-2G, 2G)
    i += (r1 >= 0.0) ? 1 : 0;
    i -= (r0 < 0.0) ? 1 : 0;
  }
  // i in [-2G, 2G) into [0, G) with unsigned minima: u = i + 2G is in [0, 4G), and
  // min(u, u - 2G) (u - 2G = i as unsigned, huge when i < 0) is in [0, 2G); then
  // min(u, u - G) is in [0, G)
  uint32_t u = (uint32_t)i + 2u * (uint32_t)m.G;
  u = __builtin_elementwise_min(u, (uint32_t)i);
  u = __builtin_elementwise_min(u, u - (uint32_t)m.G);
  out = (int32_t)u;
  return ok;
}

// GROUPED = false: the caller has checked that the mesh's group is 1, so the division
// of group_key() is left out of the code altogether (a uniform branch on the group was
// compiled into a computed-and-discarded division per particle).
template <uint32_t MODE, bool GROUPED = true>
__device__ __forceinline__ bool cell_key_m(float x, float y, float z, const Mesh& m, uint64_t& key) {
  int32_t ix, iy, iz;
  const bool ok = (int)cell_index_m<MODE>(x, m, ix) & (int)cell_index_m<MODE>(y, m, iy) &
                  (int)cell_index_m<MODE>(z, m, iz);
  const uint32_t xy = (uint32_t)ix * (uint32_t)m.G + (uint32_t)iy;  // < G^2 <= 2^32
  const uint64_t k = (uint64_t)xy * (uint64_t)(uint32_t)m.G + (uint64_t)(uint32_t)iz;
  key = GROUPED ? group_key(k, m) : k;
  return ok;
}

__device__ __forceinline__ bool cell_index(float p, const Mesh& m, int32_t& out) {
  if (m.mode == kMeshPow2Ratio) return cell_index_m<kMeshPow2Ratio>(p, m, out);
  if (m.mode == kMeshExactRatio) return cell_index_m<kMeshExactRatio>(p, m, out);
  return cell_index_m<kMeshGeneral>(p, m, out);
}

// Cell key (ix * G + iy) * G + iz of one particle (divided by the mesh's group); false
// if it is outside the domain.
__device__ __forceinline__ bool cell_key(float x, float y, float z, const Mesh& m, uint64_t& key) {
  int32_t ix, iy, iz;
  const bool ok = (int)cell_index(x, m, ix) & (int)cell_index(y, m, iy) & (int)cell_index(z, m, iz);
  const uint32_t xy = (uint32_t)ix * (uint32_t)m.G + (uint32_t)iy;  // < G^2 <= 2^32
  key = group_key((uint64_t)xy * (uint64_t)(uint32_t)m.G + (uint64_t)(uint32_t)iz, m);
  return ok;
}

// Cell key of a packed particle: i = floor(q * G / 2^21) = umulhi(q * 2^11, G) exactly
// (q < 2^21, G < 2^16); false for the outside marker (the key is then still a key of
// the mesh, so table lookups stay in range).
template <bool GROUPED = true>
__device__ __forceinline__ bool packed_key(uint64_t w, const Mesh& m, uint64_t& key) {
  constexpr uint32_t mask = (1u << kPackBits) - 1u;
  const uint32_t G = (uint32_t)m.G;
  const uint32_t ix = __umulhi(((uint32_t)w & mask) << (32 - kPackBits), G);
  const uint32_t iy = __umulhi(((uint32_t)(w >> kPackBits) & mask) << (32 - kPackBits), G);
  const uint32_t iz = __umulhi(((uint32_t)(w >> (2 * kPackBits)) & mask) << (32 - kPackBits), G);
  const uint64_t k = (uint64_t)(ix * G + iy) * G + iz;
  key = GROUPED ? group_key(k, m) : k;
  return (w >> 63) == 0;
}

// Cell key of particle i of a stream in the mesh's form: float (x, y, z) triples, or
// packed words when the mesh mode says so.
__device__ __forceinline__ bool particle_key(const float* __restrict__ pos, uint64_t i, const Mesh& m,
                                             uint64_t& key) {
  if (m.mode == kMeshPacked) return packed_key(((const uint64_t*)pos)[i], m, key);
  return cell_key(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], m, key);
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

// Row words of rows 0..DP-1 from row-interleaved tables Ti[c][v][DP] (DP = 4, 6 or 8),
// read with 16-byte (DP = 4, 8) or 8-byte (DP = 6) LDS loads.  Only key bytes below
// `nch` are looked up; stage_tables() folds the constant contribution of the other
// bytes (always 0 for keys < G^3 <= 2^(8 nch)) into the entries of byte nch - 1.
template <int DP>
__device__ __forceinline__ void row_hashes(const uint32_t* __restrict__ ti, uint64_t key, uint32_t nch,
                                           uint32_t (&h)[DP]) {
  const uint32_t lo = (uint32_t)key, hi = (uint32_t)(key >> 32);
  const uint32_t byte[kChars] = {lo & 255u, (lo >> 8) & 255u, (lo >> 16) & 255u, lo >> 24, hi & 255u, (hi >> 8) & 255u};
#pragma unroll
  for (int r = 0; r < DP; ++r) h[r] = 0;
#pragma unroll
  for (int c = 0; c < kChars; ++c) {
    if ((uint32_t)c < nch) {
      const uint32_t* e = ti + (c * 256 + byte[c]) * DP;
      if (DP % 4 == 0) {
#pragma unroll
        for (int q = 0; q < DP / 4; ++q) {
          const uint4 v = ((const uint4*)e)[q];
          h[4 * q + 0] ^= v.x;
          h[4 * q + 1] ^= v.y;
          h[4 * q + 2] ^= v.z;
          h[4 * q + 3] ^= v.w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < DP / 2; ++q) {
          const uint2 v = ((const uint2*)e)[q];
          h[2 * q + 0] ^= v.x;
          h[2 * q + 1] ^= v.y;
        }
      }
    }
  }
}

// The same over exactly KB key bytes, with no branch on the mesh: every LDS load of a key is
// issued before any is waited for.  The tables must have been staged with fold point KB
// (stage_tables(..., KB)), and KB must be at least the mesh's nch: bytes nch..KB-1 of every
// key are 0 and look up the value-0 entries, which is what the full hash does.
template <int DP, int KB>
__device__ __forceinline__ void row_hashes_kb(const uint32_t* __restrict__ ti, uint64_t key, uint32_t (&h)[DP]) {
  static_assert(KB >= 1 && KB <= kChars, "key bytes");
  const uint32_t lo = (uint32_t)key, hi = (uint32_t)(key >> 32);
  const uint32_t byte[kChars] = {lo & 255u, (lo >> 8) & 255u, (lo >> 16) & 255u, lo >> 24, hi & 255u, (hi >> 8) & 255u};
  if constexpr (DP % 4 == 0) {
    uint4 v[KB][DP / 4];
#pragma unroll
    for (int c = 0; c < KB; ++c)
#pragma unroll
      for (int q = 0; q < DP / 4; ++q) v[c][q] = ((const uint4*)(ti + (c * 256 + byte[c]) * DP))[q];
    // three-input XORs (truth table 0x96), two entries folded in per instruction
    auto xor3 = [](uint32_t a, uint32_t b, uint32_t c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96); };
#pragma unroll
    for (int q = 0; q < DP / 4; ++q) {
      uint4 x = v[0][q];
      int c = 1;
#pragma unroll
      for (; c + 1 < KB; c += 2) {
        x.x = xor3(x.x, v[c][q].x, v[c + 1][q].x);
        x.y = xor3(x.y, v[c][q].y, v[c + 1][q].y);
        x.z = xor3(x.z, v[c][q].z, v[c + 1][q].z);
        x.w = xor3(x.w, v[c][q].w, v[c + 1][q].w);
      }
      if (c < KB) {
        x.x ^= v[c][q].x;
        x.y ^= v[c][q].y;
        x.z ^= v[c][q].z;
        x.w ^= v[c][q].w;
      }
      h[4 * q + 0] = x.x;
      h[4 * q + 1] = x.y;
      h[4 * q + 2] = x.z;
      h[4 * q + 3] = x.w;
    }
  } else {
    static_assert(DP % 2 == 0, "8-byte entries");
    uint2 v[KB][DP / 2];
#pragma unroll
    for (int c = 0; c < KB; ++c)
#pragma unroll
      for (int q = 0; q < DP / 2; ++q) v[c][q] = ((const uint2*)(ti + (c * 256 + byte[c]) * DP))[q];
#pragma unroll
    for (int q = 0; q < DP / 2; ++q) {
      uint2 x = v[0][q];
#pragma unroll
      for (int c = 1; c < KB; ++c) {
        x.x ^= v[c][q].x;
        x.y ^= v[c][q].y;
      }
      h[2 * q + 0] = x.x;
      h[2 * q + 1] = x.y;
    }
  }
}

// Key bytes the branch-free hashing looks up for a mesh with nch possible key bytes: 5 for
// keys below 2^40 (G <= 10321), else 6.
__host__ __device__ __forceinline__ uint32_t key_bytes_kb(uint32_t nch) { return nch <= 5u ? 5u : 6u; }

// Number of key bytes that can be non-zero for a mesh of G cells per side.
__host__ __device__ __forceinline__ uint32_t key_chars(int32_t G) {
  const uint64_t top = (uint64_t)G * (uint64_t)G * (uint64_t)G;  // keys are < G^3
  uint32_t n = 1;
  while (n < (uint32_t)kChars && ((top - 1) >> (8 * n)) != 0) ++n;
  return n;
}

// Copy the interleaved tables of key bytes 0..bytes-1 (bytes >= nch) into LDS; entries of
// byte nch - 1 absorb the XOR of the value-0 entries of bytes nch..5.  Ends with a barrier.
template <int DP>
__device__ __forceinline__ void stage_tables(uint32_t* ti, const uint32_t* __restrict__ src, uint32_t nch,
                                             uint32_t bytes = kChars) {
  for (uint32_t i = threadIdx.x; i < (uint32_t)(256 * DP) * bytes; i += blockDim.x) {
    uint32_t v = src[i];
    const uint32_t c = i / (256 * DP);
    if (c == nch - 1) {
      const uint32_t r = i % DP;
      for (uint32_t c2 = nch; c2 < (uint32_t)kChars; ++c2) v ^= src[(c2 * 256) * DP + r];
    }
    ti[i] = v;
  }
  __syncthreads();
}

template <int D>
struct RowPad {
  static constexpr int value = (D <= 4) ? 4 : (D <= 6 ? 6 : 8);
};

// Bucket hash: low 31 bits scaled onto [0, w), i.e. floor(h31 * w / 2^31), taken as the
// high word of (h31 << 1) * w.  For w = 2^lw (lw_shift = 32 - lw) it is a plain shift.
__device__ __forceinline__ uint32_t bucket_of(uint32_t h, uint32_t w) {
  return __umulhi(h << 1, w);
}
__device__ __forceinline__ uint32_t bucket_of(uint32_t h, uint32_t w, uint32_t lw_shift) {
  return lw_shift ? (h << 1) >> lw_shift : __umulhi(h << 1, w);
}
// The same with the choice made at compile time (POW2: w = 2^lw, lw_shift = 32 - lw).
template <bool POW2>
__device__ __forceinline__ uint32_t bucket_of_t(uint32_t h, uint32_t w, uint32_t lw_shift) {
  return POW2 ? (h << 1) >> lw_shift : __umulhi(h << 1, w);
}

// How the kernels that hash all rows at once get bucket and sign:
//   kHashMulHi   any w: bucket = high word of (h31 << 1) * w (row-interleaved tables)
//   kHashShift   w = 2^lw: bucket = (h << 1) >> (32 - lw) (row-interleaved tables)
//   kHashPacked  w = 2^lw with lw + 1 <= F = floor(128 / d), d = 5..8: each table entry
//                keeps only the top F bits of every row's word, packed into 128 bits
//                (row r at bit r * F), so one 16-byte LDS load per key byte serves all
//                rows.  XOR acts bit by bit, so the packed fields of the XOR are the top
//                F bits of each row's XOR: the bucket bits (30 .. 31 - lw) and the sign
//                bit 31 are exactly those of the full word.
constexpr int kHashMulHi = 0;
constexpr int kHashShift = 1;
constexpr int kHashPacked = 2;
constexpr int packed_bits(int d) { return 128 / d; }

// Field r (F bits at bit r * F) of a 128-bit value held in four words.
template <int F>
__device__ __forceinline__ uint32_t packed_field(const uint32_t (&q)[4], int r) {
  const int o = r * F, wi = o >> 5, sh = o & 31;
  const uint32_t v = (sh + F <= 32) ? (q[wi] >> sh) : __builtin_amdgcn_alignbit(q[wi + 1], q[wi], (uint32_t)sh);
  return (F >= 32) ? v : (v & ((1u << F) - 1u));
}

// Table entry width (words) that a kernel hashing all D rows at once stages in LDS.
template <int D, int HM>
struct HashWords {
  static constexpr int value = (HM == kHashPacked) ? 4 : RowPad<D>::value;
};

// Bucket and sign bit (1 = negative) of every row of `key` from LDS tables staged for
// mode HM (see kHashMulHi / kHashShift / kHashPacked).
template <int D, int HM>
__device__ __forceinline__ void rows_bucket_sign(const uint32_t* __restrict__ ti, uint64_t key, uint32_t nch,
                                                 uint32_t w, uint32_t wshift, uint32_t (&b)[D], uint32_t (&neg)[D]) {
  constexpr int DP = HashWords<D, HM>::value;
  uint32_t h[DP];
  row_hashes<DP>(ti, key, nch, h);
  if constexpr (HM == kHashPacked) {
    constexpr int F = packed_bits(D);
    static_assert(D >= 5 && D <= 8 && F <= 25, "packed fields need d = 5..8");
    const uint32_t q[4] = {h[0], h[1], h[2], h[3]};
#pragma unroll
    for (int r = 0; r < D; ++r) {
      const uint32_t f = packed_field<F>(q, r);
      neg[r] = f >> (F - 1);
      b[r] = (f << (33 - F)) >> wshift;   // (h << 1) >> wshift with bits below the field cleared
    }
  } else {
#pragma unroll
    for (int r = 0; r < D; ++r) {
      b[r] = bucket_of_t<HM == kHashShift>(h[r], w, wshift);
      neg[r] = h[r] >> 31;
    }
  }
}

// rows_bucket_sign over exactly KB key bytes (row_hashes_kb): tables staged with fold
// point KB, or unstaged tables with KB = 6.
template <int D, int HM, int KB>
__device__ __forceinline__ void rows_bucket_sign_kb(const uint32_t* __restrict__ ti, uint64_t key, uint32_t w,
                                                    uint32_t wshift, uint32_t (&b)[D], uint32_t (&neg)[D]) {
  constexpr int DP = HashWords<D, HM>::value;
  uint32_t h[DP];
  row_hashes_kb<DP, KB>(ti, key, h);
  if constexpr (HM == kHashPacked) {
    constexpr int F = packed_bits(D);
    const uint32_t q[4] = {h[0], h[1], h[2], h[3]};
#pragma unroll
    for (int r = 0; r < D; ++r) {
      const uint32_t f = packed_field<F>(q, r);
      neg[r] = f >> (F - 1);
      b[r] = (f << (33 - F)) >> wshift;
    }
  } else {
#pragma unroll
    for (int r = 0; r < D; ++r) {
      b[r] = bucket_of_t<HM == kHashShift>(h[r], w, wshift);
      neg[r] = h[r] >> 31;
    }
  }
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

// Home slot of a cell key in the router's exact table (linear probing, empty = all ones).
__device__ __forceinline__ uint32_t table_slot(uint64_t key, uint32_t mask) {
  uint64_t x = key;
  x ^= x >> 33;
  x *= 0xFF51AFD7ED558CCDull;
  x ^= x >> 33;
  return (uint32_t)x & mask;
}

// Hot item (row r < 8, bucket b < 2^28 - 1, sign bit) packed in 32 bits (never kHotEmpty).
__device__ __forceinline__ uint32_t hot_item(uint32_t r, uint32_t b, uint32_t neg) {
  return (r << 29) | (b << 1) | neg;
}

__device__ __forceinline__ uint32_t hot_slot(uint32_t item) {
  uint32_t x = item;
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x & (kHotSlots - 1);
}

// Field-probe filter (d <= 5, w = 2^lw, lw <= 24).  Each row r has a fixed GF(2)-linear
// map L_r of 25 bits plus a salt c_r; the probe field of item (r, b, neg) is
// f = L_r((neg << lw) | b) ^ c_r: word = f mod 2^15 of a 2^15-word filter, two bit
// positions from bits 15-19 and 20-24.  The bucket and the sign are bit selections of
// the row's tabulated word, so f is itself a tabulation: the collect kernel reads it
// from probe tables (four words per key-byte entry, row r's field at bit 25 r) with one
// 16-byte LDS load per key byte and no per-row hashing.  The filter build computes f
// from the columns of L_r (kFieldCols words per row: 25 columns, then the salt).
constexpr int kFieldBits = 25;
constexpr int kFieldCols = kFieldBits + 1;
constexpr uint32_t kFieldFilterWords = 1u << 15;     // 128 KiB of LDS
constexpr uint32_t kFieldFilterMaxItems = kFieldFilterWords * 32 / 4;
constexpr uint32_t kFilterAllocWords = kFieldFilterWords > (uint32_t)kFilterWords ? kFieldFilterWords
                                                                                   : (uint32_t)kFilterWords;

// Probe of the field-probe filter for a 25-bit field f (bits above 24 ignored): the word
// from bits 10..24, the two bit positions from bits 0..4 and 5..9.
__device__ __forceinline__ FilterProbe field_probe(uint32_t f) {
  FilterProbe p;
  p.word = (f >> 10) & (kFieldFilterWords - 1u);
  p.mask = (1u << (f & 31u)) | (1u << ((f >> 5) & 31u));
  return p;
}

// 1 when both bits of field_probe(f) are set in the filter words filt, else 0: the word
// shifted down by each bit position and anded (no mask to build and compare; a shift takes
// the low five bits of its amount, so bits 0..4 need no extraction).
__device__ __forceinline__ uint32_t field_hit(const uint32_t* filt, uint32_t f) {
  const uint32_t x = filt[(f >> 10) & (kFieldFilterWords - 1u)];
  return (x >> (f & 31u)) & (x >> ((f >> 5) & 31u)) & 1u;
}

// f = L_r(x) ^ c_r from the row's columns (build side; x < 2^25).
__device__ __forceinline__ uint32_t item_field(const uint32_t* __restrict__ cols_r, uint32_t x) {
  uint32_t f = cols_r[kFieldBits];
  for (int i = 0; i < kFieldBits; ++i) f ^= ((x >> i) & 1u) ? cols_r[i] : 0u;
  return f;
}

// Bits of field r (F bits at bit r * F) of a four-word XOR, not masked above F.
template <int F>
__device__ __forceinline__ uint32_t field_bits(const uint32_t (&q)[4], int r) {
  const int o = r * F, wi = o >> 5, sh = o & 31;
  return (sh + F <= 32) ? (q[wi] >> sh) : __builtin_amdgcn_alignbit(q[wi + 1], q[wi], (uint32_t)sh);
}

// Probe of the filter for the item (row r, bucket b, sign bit neg).  Buckets are already
// uniform hash outputs, so the probe only spreads them: u = (b << bnorm) ^ row salt puts
// the bucket bits at the top of a word (bnorm = 32 - bits(w - 1)); the word comes from
// the top of u, the three bit positions from its low bits mixed with the sign.
__device__ __forceinline__ FilterProbe filter_probe(uint32_t r, uint32_t b, uint32_t neg, uint32_t bnorm) {
  const uint32_t u = (b << bnorm) ^ (r * 0x9E3779B9u);
  const uint32_t v = (b ^ (neg ? 0x5A5A5A5Au : 0u)) ^ (r * 0x7F4A7C15u) ^ (u >> 17);
  FilterProbe p;
  p.word = (uint32_t)(((uint64_t)u * (uint64_t)kFilterWords) >> 32);
  p.mask = (1u << (v & 31u)) | (1u << ((v >> 5) & 31u)) | (1u << ((v >> 10) & 31u));
  return p;
}

}  // namespace csk
