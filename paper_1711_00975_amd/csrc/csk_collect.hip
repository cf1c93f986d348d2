// csk_collect.hip — the candidate pass (Sec. 3.1 item 4: keep the cells whose estimate
// passes a threshold) on gfx950: the Bloom filter and exact hot-item set of the heavy
// (row, bucket, sign) items, built from the counters; the collect kernels, which drop a
// particle whose rows miss the filter and test the rest exactly before inserting its key
// into the candidate set; and their batched forms for many sketches in one set of launches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csk_kernel_util.h"

namespace csk {

// est(key) >= theta  <=>  at least need = d - floor((d-1)/2) of the d signed row
// estimates are >= theta (Count-Min: all d).  Rows are read until the answer is known.
template <bool TAB_LDS>
__global__ __launch_bounds__(256) void collect_kernel(const float* __restrict__ pos, uint64_t n, Mesh mesh, Tables t,
                                                      const int32_t* __restrict__ M, int32_t theta,
                                                      uint64_t* set, uint32_t slot_mask, uint32_t* set_count,
                                                      uint32_t max_cand, uint32_t* err) {
  __shared__ uint32_t tabs_lds[TAB_LDS ? kTabLdsRows * kTableWords : 1];
  const uint32_t* tabs = t.tab;
  if (TAB_LDS) {
    load_tables(tabs_lds, t.tab, t.d);
    __syncthreads();
    tabs = tabs_lds;
  }
  const uint32_t need = t.cm ? t.d : t.d - ((t.d - 1) >> 1);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    uint64_t key;
    if (!particle_key(pos, i, mesh, key)) {
      atomicOr(err, kErrDomain);
      continue;
    }
    uint32_t pass = 0;
    for (uint32_t r = 0; r < t.d; ++r) {
      if (pass >= need || pass + (t.d - r) < need) break;
      if (row_estimate(tabs + r * kTableWords, M + (uint64_t)r * t.w, t.w, t.cm, key) >= theta) ++pass;
    }
    if (pass >= need) set_insert(set, slot_mask, key, set_count, max_cand, err);
  }
}

// Row-interleaved collect for d <= 8 on an ungrouped mesh.  When a Bloom filter of the hot (row, bucket,
// sign) items is supplied, a particle whose rows pass the filter fewer than `need`
// times cannot have est >= theta (the filter has no false negatives) and is dropped
// without touching the counters; the rest take the exact test.  Each thread loads
// kCollectPPT particles before working on any of them, so that enough position loads
// are in flight to cover HBM latency at one workgroup per CU.
// FP: the field-probe filter (d = 5, w <= 2^24; packed or multiply-high buckets).  Its probe
// tables take the place of the hash tables in LDS and its filter is 2^15 words; the exact
// test of the particles that pass reads the packed or row-interleaved hash tables from
// device memory (all six key bytes).
// Workgroup g of nwg runs the chunks g, g + nwg, ... of the stream.  The sketch's
// arguments are read in place through cp (argument segment or descriptor array).
template <int D, uint32_t MODE, int HM, bool FP, int KB>
__device__ __forceinline__ void collect2_body(const CollectDesc* __restrict__ cp, const float* __restrict__ pos,
                                              uint64_t n, int32_t theta, uint32_t use_filter, uint32_t g,
                                              uint32_t nwg) {
  const CollectDesc& c = *cp;
  const Mesh& mesh = c.mesh;
  const Tables& t = c.t;
  const int32_t* __restrict__ M = c.M;
  const uint32_t* __restrict__ filter = c.filter;
  const uint32_t* __restrict__ hot = c.hot;
  const uint32_t* __restrict__ hot_table = c.hot_table;
  uint64_t* set = c.set;
  const uint32_t slot_mask = c.slot_mask;
  uint32_t* set_count = c.set_count;
  const uint32_t max_cand = c.max_cand;
  uint32_t* err = c.err;
  constexpr int DP = FP ? 4 : HashWords<D, HM>::value;
  constexpr int PPT = kCollectPPT;
  constexpr uint32_t FW = FP ? kFieldFilterWords : (uint32_t)kFilterWords;
  static_assert(!FP || (D <= 5 && (HM == kHashPacked || HM == kHashMulHi)),
                "field probes: d <= 5 rows of 25 bits, packed or multiply-high buckets");
  extern __shared__ __align__(16) uint32_t lds3[];
  uint32_t* ti = lds3;
  uint64_t* cache = (uint64_t*)(ti + kTableWords * DP);   // kCollectCache keys
  uint32_t* filt = (uint32_t*)(cache + kCollectCache);
  const uint32_t nhot = use_filter ? *hot : 0xFFFFFFFFu;
  // a hot item takes up to fspan entries of the field-probe filter (1 for w = 2^P)
  const bool uf = use_filter && (FP ? (uint64_t)nhot * t.fspan <= kFieldFilterMaxItems : nhot <= kFilterMaxItems);
  // the exact hot-item set replaces the counter reads when it holds every hot item
  const bool uh = use_filter && hot_table != nullptr && nhot <= kHotMaxItems;
  if (uf)
    for (uint32_t i = threadIdx.x; i < FW; i += blockDim.x) filt[i] = filter[i];
  for (uint32_t i = threadIdx.x; i < (uint32_t)kCollectCache; i += blockDim.x) cache[i] = kEmptyKey;
  stage_tables<DP>(ti, FP ? t.tabq : (HM == kHashPacked ? t.tabp : t.tabi), (uint32_t)KB);
  // (bucket, sign) of every row for the exact test: from the staged tables, or (FP) from
  // the packed or row-interleaved tables in device memory over all six key bytes
  auto exact_rows = [&](uint64_t key, uint32_t (&bk)[D], uint32_t (&ng)[D]) {
    if constexpr (FP) rows_bucket_sign_kb<D, HM, kChars>(HM == kHashPacked ? t.tabp : t.tabi, key, t.w, t.wshift, bk, ng);
    else rows_bucket_sign_kb<D, HM, KB>(ti, key, t.w, t.wshift, bk, ng);
  };
  constexpr uint32_t kNeedCS = D - ((D - 1) >> 1);
  const uint32_t need = t.cm ? (uint32_t)D : kNeedCS;
  constexpr uint32_t NT = kCollectThreads;
  const uint64_t chunk = (uint64_t)NT * PPT;
  bool bad = false;
  for (uint64_t first = (uint64_t)g * chunk; first < n; first += (uint64_t)nwg * chunk) {
    const bool full = first + chunk <= n;
    // all PPT position loads are issued before any is used; float records come through a
    // buffer resource over the rest of the stream (loads past it return 0), packed words
    // with a clamped index; particles beyond the stream are masked below
    float px[PPT], py[PPT], pz[PPT];
    uint64_t pw[PPT];
    if constexpr (MODE == kMeshPacked) {
      const uint64_t last = n - 1;
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        uint64_t i = first + (uint64_t)j * NT + threadIdx.x;
        i = i < last ? i : last;
        pw[j] = __builtin_nontemporal_load((const uint64_t*)pos + i);
      }
    } else {
      const __amdgpu_buffer_rsrc_t span = byte_span(pos + 3 * first, (n - first) * 12);
#pragma unroll
      for (int j = 0; j < PPT; ++j) load_xyz(span, 12u * threadIdx.x, 12u * (uint32_t)j * NT, px[j], py[j], pz[j]);
    }
    // keys and the filter verdict of all PPT particles, without branches
    uint64_t keys[PPT];
    uint32_t cand = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const bool in = full || (first + (uint64_t)j * NT + threadIdx.x) < n;
      bool ok;
      if constexpr (MODE == kMeshPacked) ok = packed_key<false>(pw[j], mesh, keys[j]);
      else ok = cell_key_m<MODE, false>(px[j], py[j], pz[j], mesh, keys[j]);
      bad |= in && !ok;
      bool go = in && ok;
      if (uf) {
        uint32_t fp = 0;
        if constexpr (FP) {
          uint32_t q[4];
          row_hashes_kb<4, KB>(ti, keys[j], q);
#pragma unroll
          for (int r = 0; r < D; ++r) fp += field_hit(filt, field_bits<kFieldBits>(q, r));
        } else {
          uint32_t bk[D], sg[D];
          rows_bucket_sign_kb<D, HM, KB>(ti, keys[j], t.w, t.wshift, bk, sg);
#pragma unroll
          for (int r = 0; r < D; ++r) {
            const uint32_t ng = sg[r] & (t.cm ^ 1u);
            const FilterProbe pr = filter_probe((uint32_t)r, bk[r], ng, t.bnorm);
            fp += ((filt[pr.word] & pr.mask) == pr.mask) ? 1u : 0u;
          }
        }
        go = go && fp >= need;
      }
      cand |= (uint32_t)go << j;
    }
    // The particles that may pass.  A key seen recently by this workgroup, or already in the
    // set, needs no exact test: heavy cells repeat thousands of times, and the set only ever
    // gains keys.  The first set slot of every candidate is loaded before any is compared,
    // so that the thread waits on one round trip for all its keys rather than one per key.
    auto cache_slot = [](uint64_t key) { return (uint32_t)(key ^ (key >> 21)) & (kCollectCache - 1); };
    uint32_t todo = cand;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      if ((todo >> j) & 1u)
        if (__hip_atomic_load(&cache[cache_slot(keys[j])], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == keys[j])
          todo &= ~(1u << j);
    }
    // the first slot of each key's probe sequence in the set
    uint64_t s0[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      s0[j] = kEmptyKey;
      if ((todo >> j) & 1u) s0[j] = set[(uint32_t)slot_mix(keys[j]) & slot_mask];
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      if (!((todo >> j) & 1u)) continue;
      bool in = s0[j] == keys[j];
      if (!in && s0[j] != kEmptyKey) in = set_contains(set, slot_mask, keys[j]);   // a longer probe run
      if (in) {
        __hip_atomic_store(&cache[cache_slot(keys[j])], keys[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        todo &= ~(1u << j);
      }
    }
    // Other threads of the workgroup may have inserted a key since the first cache check;
    // looking again before the exact test spares it (one LDS read).
    auto recheck = [&](uint64_t key) {
      return __hip_atomic_load(&cache[cache_slot(key)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == key;
    };
    // The exact test of the rest.  With the hot-item set (2 MiB, resident in L2) the first
    // slot of every row of a group of keys (four for d <= 5, else two) is loaded before any
    // is compared.  Without it the counters are read row by row until the answer is known;
    // in a large table those reads go to HBM, and reading all d rows at once was no faster.
    if (uh) {
      constexpr int GQ = D <= 5 ? 4 : 2;
      static_assert(PPT % GQ == 0, "whole groups of keys");
#pragma unroll
      for (int j0 = 0; j0 < PPT; j0 += GQ) {
        if (!((todo >> j0) & ((1u << GQ) - 1u))) continue;
        uint32_t item[GQ][D], v[GQ][D];
#pragma unroll
        for (int q = 0; q < GQ; ++q) {
          if (!((todo >> (j0 + q)) & 1u)) continue;
          if (recheck(keys[j0 + q])) {
            todo &= ~(1u << (j0 + q));
            continue;
          }
          uint32_t bk[D], ng[D];
          exact_rows(keys[j0 + q], bk, ng);
#pragma unroll
          for (int r = 0; r < D; ++r) {
            item[q][r] = hot_item((uint32_t)r, bk[r], ng[r] & (t.cm ^ 1u));
            v[q][r] = hot_table[hot_slot(item[q][r])];
          }
        }
#pragma unroll
        for (int q = 0; q < GQ; ++q) {
          const int j = j0 + q;
          if (!((todo >> j) & 1u)) continue;
          // row r passes (sign * M >= theta) exactly when its item is in the hot set
          uint32_t pass = 0;
#pragma unroll
          for (int r = 0; r < D; ++r) {
            bool hit = v[q][r] == item[q][r];
            if (!hit && v[q][r] != kHotEmpty) {
              uint32_t sl = (hot_slot(item[q][r]) + 1) & (kHotSlots - 1);
              for (uint32_t probe = 1; probe < kHotSlots; ++probe) {
                const uint32_t x = hot_table[sl];
                if (x == item[q][r]) {
                  hit = true;
                  break;
                }
                if (x == kHotEmpty) break;
                sl = (sl + 1) & (kHotSlots - 1);
              }
            }
            pass += hit ? 1u : 0u;
          }
          if (pass >= need) {
            set_insert(set, slot_mask, keys[j], set_count, max_cand, err);
            __hip_atomic_store(&cache[cache_slot(keys[j])], keys[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        if (!((todo >> j) & 1u) || recheck(keys[j])) continue;
        uint32_t bk[D], ng[D];
        exact_rows(keys[j], bk, ng);
        uint32_t pass = 0;
#pragma unroll
        for (int r = 0; r < D; ++r) {
          if (pass >= need || pass + (uint32_t)(D - r) < need) break;
          const uint32_t c = (uint32_t)M[(uint64_t)r * t.w + bk[r]];
          if ((int32_t)((ng[r] & (t.cm ^ 1u)) ? 0u - c : c) >= theta) ++pass;
        }
        if (pass >= need) {
          set_insert(set, slot_mask, keys[j], set_count, max_cand, err);
          __hip_atomic_store(&cache[cache_slot(keys[j])], keys[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }
  }
  if (bad) atomicOr(err, kErrDomain);
}

template <int D, uint32_t MODE, int HM, bool FP, int KB>
__global__ __launch_bounds__(kCollectThreads) void collect2_kernel(CollectDesc c, const float* __restrict__ pos,
                                                                   uint64_t n, int32_t theta, uint32_t use_filter) {
  collect2_body<D, MODE, HM, FP, KB>(&c, pos, n, theta, use_filter, blockIdx.x, gridDim.x);
}

// Many sketches' candidate passes in one launch: workgroup blockIdx.x serves sketch
// wg_sketch[blockIdx.x] as its workgroup blockIdx.x - wg_first[sketch] of wg_count[sketch].
template <int D, uint32_t MODE, int HM, bool FP, int KB>
__global__ __launch_bounds__(kCollectThreads) void collect2_batch_kernel(const CollectDesc* __restrict__ descs,
                                                                         const uint16_t* __restrict__ wg_sketch,
                                                                         const uint32_t* __restrict__ wg_first,
                                                                         const uint32_t* __restrict__ wg_count,
                                                                         CollectCall call) {
  const uint32_t i = wg_sketch[blockIdx.x];
  collect2_body<D, MODE, HM, FP, KB>(descs + i, call.pos[i], call.n[i], call.theta[i], call.use_filter[i],
                                     blockIdx.x - wg_first[i], wg_count[i]);
}

// Items (r, b, sign) with sign * M[r][b] >= theta (Count-Min: M[r][b] >= theta) go into
// the Bloom filter and, when all of them fit, into the exact hot-item set; theta > 0, so
// empty buckets never do.  *hot counts the items.
// Is the signed counter of (r, b, sign) >= theta?  The signed estimate is -M modulo 2^32
// for a negative sign (Count-Min: M itself), exactly as the collect test reads it.
__device__ __forceinline__ void hot_pair(int32_t c, uint32_t cm, int32_t theta, bool valid, bool& hp, bool& hn) {
  hp = valid && c >= theta;
  hn = valid && !cm && ((int32_t)(0u - (uint32_t)c) >= theta);
}

// Loads kFilterVec groups of 4 counters of row r for this thread (16-byte loads when rows
// are 16-byte aligned) before any is tested.
constexpr int kFilterVec = 2;
__device__ __forceinline__ void load_counters(const int32_t* __restrict__ Mr, uint32_t w, uint64_t b0,
                                              int32_t (&c)[kFilterVec][4]) {
  const bool vec = (w & 3u) == 0;
#pragma unroll
  for (int v = 0; v < kFilterVec; ++v) {
    const uint64_t b = b0 + ((uint64_t)v * blockDim.x + threadIdx.x) * 4;
    if (vec && b < w) {
      const int4 q = *(const int4*)(Mr + b);
      c[v][0] = q.x;
      c[v][1] = q.y;
      c[v][2] = q.z;
      c[v][3] = q.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) c[v][e] = (b + e < w) ? Mr[b + e] : 0;
    }
  }
}

// Pass 1: sets the Bloom filter bits of every hot item and counts the items into *hot
// (per-workgroup count in LDS, one global add per workgroup).
// fcols != NULL: the field-probe filter (item fields from the row maps' columns, P prefix
// bits); else the hashed probe of filter_probe().
// Block bx of nbx scans its share of every row.

// The field-probe filter entries of item (row r, bucket b, sign sg): x = (sg << P) | p for
// every P-bit prefix p of a bucket input h' = h << 1 with umulhi(h', w) = b, i.e.
// h' in [ceil(b 2^32 / w), ceil((b + 1) 2^32 / w) - 1].  For w = 2^P that prefix is b.
__device__ __forceinline__ void field_insert(const uint32_t* __restrict__ cols_r, uint32_t w, uint32_t P, uint32_t b,
                                             uint32_t sg, uint32_t* __restrict__ filter) {
  uint32_t p_lo = b, p_hi = b;
  if ((1u << P) != w) {
    const uint64_t lo = (((uint64_t)b << 32) + w - 1) / w;
    const uint64_t hi = ((((uint64_t)b + 1) << 32) + w - 1) / w - 1;
    p_lo = (uint32_t)(lo >> (32 - P));
    p_hi = (uint32_t)(hi >> (32 - P));
  }
  for (uint32_t p = p_lo; p <= p_hi; ++p) {
    const FilterProbe pr = field_probe(item_field(cols_r, (sg << P) | p));
    atomicOr(&filter[pr.word], pr.mask);
  }
}

__device__ __forceinline__ void filter_build_body(const int32_t* __restrict__ M, uint32_t d, uint32_t w, uint32_t cm,
                                                  uint32_t bnorm, int32_t theta, const uint32_t* __restrict__ fcols,
                                                  uint32_t P, uint32_t* __restrict__ filter,
                                                  uint32_t* __restrict__ hot, uint32_t bx, uint32_t nbx) {
  __shared__ uint32_t count;
  if (threadIdx.x == 0) count = 0;
  __syncthreads();
  uint32_t mine = 0;
  const uint64_t span = (uint64_t)nbx * blockDim.x * 4 * kFilterVec;
  for (uint32_t r = 0; r < d; ++r) {
    const int32_t* __restrict__ Mr = M + (uint64_t)r * w;
    for (uint64_t b0 = (uint64_t)bx * blockDim.x * 4 * kFilterVec; b0 < w; b0 += span) {
      int32_t c[kFilterVec][4];
      load_counters(Mr, w, b0, c);
#pragma unroll
      for (int v = 0; v < kFilterVec; ++v) {
        const uint64_t b = b0 + ((uint64_t)v * blockDim.x + threadIdx.x) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          bool hp, hn;
          hot_pair(c[v][e], cm, theta, b + e < w, hp, hn);
          if (hp) {
            if (fcols) {
              field_insert(fcols + r * kFieldCols, w, P, (uint32_t)(b + e), 0u, filter);
            } else {
              const FilterProbe pr = filter_probe(r, (uint32_t)(b + e), 0u, bnorm);
              atomicOr(&filter[pr.word], pr.mask);
            }
          }
          if (hn) {
            if (fcols) {
              field_insert(fcols + r * kFieldCols, w, P, (uint32_t)(b + e), 1u, filter);
            } else {
              const FilterProbe pr = filter_probe(r, (uint32_t)(b + e), 1u, bnorm);
              atomicOr(&filter[pr.word], pr.mask);
            }
          }
          mine += (uint32_t)hp + (uint32_t)hn;
        }
      }
    }
  }
  if (mine) atomicAdd(&count, mine);
  __syncthreads();
  if (threadIdx.x == 0 && count) atomicAdd(hot, count);
}

__global__ __launch_bounds__(256) void filter_build_kernel(const int32_t* __restrict__ M, uint32_t d, uint32_t w,
                                                           uint32_t cm, uint32_t bnorm, int32_t theta,
                                                           const uint32_t* __restrict__ fcols, uint32_t P,
                                                           uint32_t* __restrict__ filter, uint32_t* __restrict__ hot) {
  filter_build_body(M, d, w, cm, bnorm, theta, fcols, P, filter, hot, blockIdx.x, gridDim.x);
}

__device__ __forceinline__ void hot_insert(uint32_t* table, uint32_t item) {
  uint32_t sl = hot_slot(item);
  for (uint32_t probe = 0; probe < kHotSlots; ++probe) {
    const uint32_t old = atomicCAS(&table[sl], kHotEmpty, item);
    if (old == kHotEmpty || old == item) return;
    sl = (sl + 1) & (kHotSlots - 1);
  }
}

// Pass 2: when every hot item fits (*hot <= kHotMaxItems, so the table stays at most half
// full), inserts them all into the exact hot-item set; otherwise does nothing.
__device__ __forceinline__ void hot_build_body(const int32_t* __restrict__ M, uint32_t d, uint32_t w, uint32_t cm,
                                               int32_t theta, const uint32_t* __restrict__ hot,
                                               uint32_t* __restrict__ hot_table, uint32_t bx, uint32_t nbx) {
  if (*hot > kHotMaxItems) return;
  const uint64_t span = (uint64_t)nbx * blockDim.x * 4 * kFilterVec;
  for (uint32_t r = 0; r < d; ++r) {
    const int32_t* __restrict__ Mr = M + (uint64_t)r * w;
    for (uint64_t b0 = (uint64_t)bx * blockDim.x * 4 * kFilterVec; b0 < w; b0 += span) {
      int32_t c[kFilterVec][4];
      load_counters(Mr, w, b0, c);
#pragma unroll
      for (int v = 0; v < kFilterVec; ++v) {
        const uint64_t b = b0 + ((uint64_t)v * blockDim.x + threadIdx.x) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          bool hp, hn;
          hot_pair(c[v][e], cm, theta, b + e < w, hp, hn);
          if (hp) hot_insert(hot_table, hot_item(r, (uint32_t)(b + e), 0u));
          if (hn) hot_insert(hot_table, hot_item(r, (uint32_t)(b + e), 1u));
        }
      }
    }
  }
}

__global__ __launch_bounds__(256) void hot_build_kernel(const int32_t* __restrict__ M, uint32_t d, uint32_t w,
                                                        uint32_t cm, int32_t theta, const uint32_t* __restrict__ hot,
                                                        uint32_t* __restrict__ hot_table) {
  hot_build_body(M, d, w, cm, theta, hot, hot_table, blockIdx.x, gridDim.x);
}

// Batched forms: blockIdx.y = sketch; a sketch whose call does not use its filter is skipped.
__global__ __launch_bounds__(256) void collect_clear_batch_kernel(const CollectDesc* __restrict__ descs,
                                                                  CollectCall call, uint32_t fw) {
  const uint32_t i = blockIdx.y;
  if (!call.use_filter[i]) return;
  const CollectDesc& c = descs[i];
  const uint64_t nh = c.hot_table != nullptr ? kHotSlots : 0u;
  const uint64_t total = (uint64_t)fw + 1u + nh;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += stride) {
    if (j < fw) c.filter[j] = 0u;
    else if (j == fw) *c.hot = 0u;
    else c.hot_table[j - fw - 1u] = kHotEmpty;
  }
}

__global__ __launch_bounds__(256) void filter_build_batch_kernel(const CollectDesc* __restrict__ descs,
                                                                 CollectCall call, uint32_t field) {
  const uint32_t i = blockIdx.y;
  if (!call.use_filter[i]) return;
  const CollectDesc& c = descs[i];
  filter_build_body(c.M, c.t.d, c.t.w, c.t.cm, c.t.bnorm, call.theta[i], field ? c.t.fcols : nullptr, c.t.fp,
                    c.filter, c.hot, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void hot_build_batch_kernel(const CollectDesc* __restrict__ descs,
                                                              CollectCall call) {
  const uint32_t i = blockIdx.y;
  if (!call.use_filter[i] || descs[i].hot_table == nullptr) return;
  const CollectDesc& c = descs[i];
  hot_build_body(c.M, c.t.d, c.t.w, c.t.cm, call.theta[i], c.hot, c.hot_table, blockIdx.x, gridDim.x);
}

hipError_t launch_filter_build(const Tables& t, const int32_t* M, int32_t theta, uint32_t* filter, uint32_t* hot,
                               uint32_t* hot_table, bool field, hipStream_t s) {
  field = field && t.fcols != nullptr;
  FillSpans f{};   // the three clears in one launch
  f.p[0] = filter;
  f.n[0] = field ? kFieldFilterWords : kFilterWords;
  f.p[1] = hot;
  f.n[1] = 1;
  f.p[2] = hot_table;
  f.n[2] = hot_table != nullptr ? kHotSlots : 0;
  f.v[2] = kHotEmpty;
  hipError_t e = launch_fill_spans(f, s);
  if (e != hipSuccess) return e;
  const dim3 grid(grid_for((t.w + 4 * kFilterVec - 1) / (4 * kFilterVec), 256, 8192));
  hipLaunchKernelGGL(filter_build_kernel, grid, dim3(256), 0, s, M, t.d, t.w, t.cm, t.bnorm, theta,
                     field ? t.fcols : nullptr, t.fp, filter, hot);
  if (hot_table != nullptr)
    hipLaunchKernelGGL(hot_build_kernel, grid, dim3(256), 0, s, M, t.d, t.w, t.cm, theta, hot, hot_table);
  return hipGetLastError();
}

// One collect launch (or a batch of them): the sketch's descriptor and the per-call stream.
struct CollectLaunch {
  const CollectDesc* c;        // one sketch (kernel argument copy), or NULL for a batch
  const float* pos;
  uint64_t n;
  int32_t theta;
  uint32_t use_filter;
  bool field;
  // batch
  const CollectDesc* descs;
  const uint16_t* wg_sketch;
  const uint32_t* wg_first;
  const uint32_t* wg_count;
  const CollectCall* call;
  uint32_t kb;   // key bytes to look up (d = 5): 5 or 6
};

template <int D, uint32_t MM, int HM, bool FP, int KB>
static void launch_collect2_kb(dim3 grid, dim3 block, size_t lds, hipStream_t s, const CollectLaunch& c) {
  if (c.c != nullptr)
    hipLaunchKernelGGL((collect2_kernel<D, MM, HM, FP, KB>), grid, block, lds, s, *c.c, c.pos, c.n, c.theta,
                       c.use_filter);
  else
    hipLaunchKernelGGL((collect2_batch_kernel<D, MM, HM, FP, KB>), grid, block, lds, s, c.descs, c.wg_sketch,
                       c.wg_first, c.wg_count, *c.call);
}

// d = 5 hashes exactly the key bytes its mesh needs (5 below 2^40, else 6); other d all six.
template <int D, uint32_t MM, int HM, bool FP = false>
static void launch_collect2_one(dim3 grid, dim3 block, size_t lds, hipStream_t s, const CollectLaunch& c) {
  if constexpr (D == 5) {
    if (c.kb == 5) {
      launch_collect2_kb<D, MM, HM, FP, 5>(grid, block, lds, s, c);
      return;
    }
  }
  launch_collect2_kb<D, MM, HM, FP, kChars>(grid, block, lds, s, c);
}

template <int D, uint32_t MM>
static void launch_collect2_m(int hm, dim3 grid, dim3 block, size_t lds, hipStream_t s, const CollectLaunch& c) {
  if constexpr (D == 5) {
    if (hm == kHashPacked && c.field) {
      launch_collect2_one<D, MM, kHashPacked, true>(grid, block, lds, s, c);
      return;
    }
    if constexpr (MM != kMeshPacked) {
      if (hm == kHashMulHi && c.field) {
        launch_collect2_one<D, MM, kHashMulHi, true>(grid, block, lds, s, c);
        return;
      }
    }
  }
  if constexpr (D >= 5) {
    if (hm == kHashPacked) {
      launch_collect2_one<D, MM, kHashPacked>(grid, block, lds, s, c);
      return;
    }
  }
  if (hm == kHashMulHi) launch_collect2_one<D, MM, kHashMulHi>(grid, block, lds, s, c);
  else launch_collect2_one<D, MM, kHashShift>(grid, block, lds, s, c);
}

template <int D>
static void launch_collect2_dm(uint32_t mode, int hm, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                               const CollectLaunch& c) {
  if (mode == kMeshPacked) launch_collect2_m<D, kMeshPacked>(hm, grid, block, lds, s, c);
  else if (mode == kMeshPow2Ratio) launch_collect2_m<D, kMeshPow2Ratio>(hm, grid, block, lds, s, c);
  else if (mode == kMeshExactRatio) launch_collect2_m<D, kMeshExactRatio>(hm, grid, block, lds, s, c);
  else launch_collect2_m<D, kMeshGeneral>(hm, grid, block, lds, s, c);
}

static void launch_collect2_d(uint32_t d, uint32_t mode, int hm, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                              const CollectLaunch& c) {
  switch (d) {
    case 1: launch_collect2_dm<1>(mode, hm, grid, block, lds, s, c); break;
    case 2: launch_collect2_dm<2>(mode, hm, grid, block, lds, s, c); break;
    case 3: launch_collect2_dm<3>(mode, hm, grid, block, lds, s, c); break;
    case 4: launch_collect2_dm<4>(mode, hm, grid, block, lds, s, c); break;
    case 5: launch_collect2_dm<5>(mode, hm, grid, block, lds, s, c); break;
    case 6: launch_collect2_dm<6>(mode, hm, grid, block, lds, s, c); break;
    case 7: launch_collect2_dm<7>(mode, hm, grid, block, lds, s, c); break;
    default: launch_collect2_dm<8>(mode, hm, grid, block, lds, s, c); break;
  }
}

size_t collect2_lds_bytes(const Tables& t, bool use_filter, bool field) {
  return field ? ((size_t)kTableWords * 4 + 2 * kCollectCache + kFieldFilterWords) * sizeof(uint32_t)
               : ((size_t)kTableWords * t.dp + 2 * kCollectCache + (use_filter ? kFilterWords : 0)) * sizeof(uint32_t);
}

bool collect_field_form(const Tables& t) {
  return t.d == 5 && t.tabq != nullptr && (t.hash_mode() == kHashPacked || t.hash_mode() == kHashMulHi);
}

hipError_t launch_collect(const float* pos, uint64_t n, const Mesh& mesh, const Tables& t, const int32_t* M,
                          int32_t theta, const uint32_t* filter, const uint32_t* hot, const uint32_t* hot_table,
                          uint64_t* set, uint32_t slot_mask, uint32_t* set_count, uint32_t max_cand, uint32_t* err,
                          bool field, hipStream_t s) {
  if (t.d <= (uint32_t)kTabLdsRows && mesh.group == 1u) {   // collect2_kernel takes ungrouped keys
    const uint32_t use_filter = (filter != nullptr && hot != nullptr) ? 1u : 0u;
    field = field && use_filter && collect_field_form(t);
    const size_t lds = collect2_lds_bytes(t, use_filter != 0, field);
    const dim3 grid(grid_for((n + kCollectPPT - 1) / kCollectPPT, kCollectThreads, 256)), block(kCollectThreads);
    const CollectDesc cd{mesh, t, M, const_cast<uint32_t*>(filter), const_cast<uint32_t*>(hot),
                         const_cast<uint32_t*>(hot_table), set, slot_mask, set_count, max_cand, err};
    const CollectLaunch ca{&cd, pos, n, theta, use_filter, field, nullptr, nullptr, nullptr, nullptr, nullptr,
                           key_bytes_kb(mesh.nch)};
    launch_collect2_d(t.d, mesh.mode, t.hash_mode(), grid, block, lds, s, ca);
  } else {
    hipLaunchKernelGGL(collect_kernel<false>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, pos, n, mesh, t, M, theta,
                       set, slot_mask, set_count, max_cand, err);
  }
  return hipGetLastError();
}

hipError_t launch_collect_batch(const CollectDesc* descs, const CollectDesc* host_descs, uint32_t count,
                                const uint16_t* wg_sketch, const uint32_t* wg_first, const uint32_t* wg_count,
                                uint32_t nwg_total, uint32_t d, uint32_t mesh_mode, int hm, bool field,
                                uint32_t w_max, const CollectCall& call, hipStream_t s) {
  if (count == 0 || nwg_total == 0) return hipSuccess;
  bool any_filter = false;
  size_t lds = 0;
  for (uint32_t i = 0; i < count; ++i) {
    any_filter = any_filter || call.use_filter[i] != 0;
    const size_t b = collect2_lds_bytes(host_descs[i].t, true, field);
    lds = b > lds ? b : lds;
  }
  if (any_filter) {
    const uint32_t fw = field ? kFieldFilterWords : (uint32_t)kFilterWords;
    hipLaunchKernelGGL(collect_clear_batch_kernel, dim3(grid_for((uint64_t)fw + 1 + kHotSlots, 256, 256), count),
                       dim3(256), 0, s, descs, call, fw);
    const dim3 grid(grid_for((w_max + 4 * kFilterVec - 1) / (4 * kFilterVec), 256, 8192), count);
    hipLaunchKernelGGL(filter_build_batch_kernel, grid, dim3(256), 0, s, descs, call, field ? 1u : 0u);
    hipLaunchKernelGGL(hot_build_batch_kernel, grid, dim3(256), 0, s, descs, call);
  }
  uint32_t kb = 5;
  for (uint32_t i = 0; i < count; ++i) kb = key_bytes_kb(host_descs[i].mesh.nch) > kb ? key_bytes_kb(host_descs[i].mesh.nch) : kb;
  const CollectLaunch ca{nullptr, nullptr, 0, 0, 0, field, descs, wg_sketch, wg_first, wg_count, &call, kb};
  launch_collect2_d(d, mesh_mode, hm, dim3(nwg_total), dim3(kCollectThreads), lds, s, ca);
  return hipGetLastError();
}

}  // namespace csk
