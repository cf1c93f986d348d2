// csk_kernels.hip — gfx950 kernels of the streaming Count-Sketch hot path after the
// update (which lives in csk_update.hip):
// query   (Sec. 2.2 Estimate; Alg. 4 Estimate): lower median of the d signed counters.
// collect (Sec. 3.1 item 4): threshold test per particle, distinct keys into a hash set.
// topk    (Sec. 2.2 UpdateHeap; Alg. 1 query): two-stage radix select on
//         (estimate desc, key asc), then an exact rank placement of the k winners.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csk_kernel_util.h"

namespace csk {

// ------------------------------------------------------------------ keys

__global__ __launch_bounds__(256) void keys_kernel(const float* __restrict__ pos, uint64_t n, Mesh mesh,
                                                   uint64_t* __restrict__ keys) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    uint64_t key;
    keys[i] = particle_key(pos, i, mesh, key) ? key : kEmptyKey;
  }
}

hipError_t launch_keys(const float* pos, uint64_t n, const Mesh& mesh, uint64_t* keys, hipStream_t s) {
  hipLaunchKernelGGL(keys_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, pos, n, mesh, keys);
  return hipGetLastError();
}

// Packing: word = qx | qy << 21 | qz << 42 with q = floor(p * 2^21 / L) exactly (the cell
// index of a mesh of 2^21 cells, wrapped), or all ones outside the domain (bit 0 of *err).
__global__ __launch_bounds__(256) void pack_kernel(const float* __restrict__ pos, uint64_t n, Mesh pm,
                                                   uint64_t* __restrict__ out, uint32_t* __restrict__ err) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    int32_t qx, qy, qz;
    const bool ok = (int)cell_index(pos[3 * i], pm, qx) & (int)cell_index(pos[3 * i + 1], pm, qy) &
                    (int)cell_index(pos[3 * i + 2], pm, qz);
    out[i] = ok ? ((uint64_t)(uint32_t)qx | (uint64_t)(uint32_t)qy << kPackBits |
                   (uint64_t)(uint32_t)qz << (2 * kPackBits))
                : kPackedOutside;
    bad |= !ok;
  }
  if (bad) atomicOr(err, 1u);
}

hipError_t launch_pack(const float* pos, uint64_t n, const Mesh& pm, uint64_t* out, uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, pos, n, pm, out, err);
  return hipGetLastError();
}

// ------------------------------------------------------------------ query

template <int MAXD, bool TAB_LDS>
__global__ __launch_bounds__(256) void query_kernel(const uint64_t* __restrict__ keys, uint64_t m, Tables t,
                                                    const int32_t* __restrict__ M, int32_t* __restrict__ est) {
  __shared__ uint32_t tabs_lds[TAB_LDS ? kTabLdsRows * kTableWords : 1];
  const uint32_t* tabs = t.tab;
  if (TAB_LDS) {
    load_tables(tabs_lds, t.tab, t.d);
    __syncthreads();
    tabs = tabs_lds;
  }
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    est[i] = estimate_key<MAXD>(tabs, M, t.d, t.w, t.cm, keys[i] & 0xFFFFFFFFFFFFull);
  }
}

hipError_t launch_query(const uint64_t* keys, uint64_t m, const Tables& t, const int32_t* M, int32_t* est,
                        hipStream_t s) {
  const dim3 grid(grid_for(m, 256, 8192));
  if (t.d <= (uint32_t)kTabLdsRows)
    hipLaunchKernelGGL((query_kernel<kTabLdsRows, true>), grid, dim3(256), 0, s, keys, m, t, M, est);
  else
    hipLaunchKernelGGL((query_kernel<32, false>), grid, dim3(256), 0, s, keys, m, t, M, est);
  return hipGetLastError();
}

// ------------------------------------------------------------------ collect

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
// FP: the field-probe filter (d = 5, packed hash).  Its probe tables take the place of the
// hash tables in LDS and its filter is 2^15 words; the exact test of the particles that
// pass reads the packed hash tables from device memory (all six key bytes).
template <int D, uint32_t MODE, int HM, bool FP>
__global__ __launch_bounds__(kCollectThreads) void collect2_kernel(const float* __restrict__ pos, uint64_t n, Mesh mesh,
                                                                   Tables t, const int32_t* __restrict__ M,
                                                                   int32_t theta, const uint32_t* __restrict__ filter,
                                                                   const uint32_t* __restrict__ hot, uint32_t use_filter,
                                                                   const uint32_t* __restrict__ hot_table,
                                                                   uint64_t* set, uint32_t slot_mask,
                                                                   uint32_t* set_count, uint32_t max_cand,
                                                                   uint32_t* err) {
  constexpr int DP = FP ? 4 : HashWords<D, HM>::value;
  constexpr int PPT = kCollectPPT;
  constexpr uint32_t FW = FP ? kFieldFilterWords : (uint32_t)kFilterWords;
  static_assert(!FP || (D <= 5 && HM == kHashPacked), "field probes: d <= 5 rows of 25 bits, packed hash");
  extern __shared__ __align__(16) uint32_t lds3[];
  uint32_t* ti = lds3;
  uint64_t* cache = (uint64_t*)(ti + kTableWords * DP);   // kCollectCache keys
  uint32_t* filt = (uint32_t*)(cache + kCollectCache);
  const uint32_t nhot = use_filter ? *hot : 0xFFFFFFFFu;
  const bool uf = use_filter && nhot <= (FP ? kFieldFilterMaxItems : kFilterMaxItems);
  // the tables the exact test hashes with: staged in LDS, or (FP) read from device memory
  const uint32_t* tx = FP ? t.tabp : ti;
  const uint32_t nchx = FP ? (uint32_t)kChars : mesh.nch;
  // the exact hot-item set replaces the counter reads when it holds every hot item
  const bool uh = use_filter && hot_table != nullptr && nhot <= kHotMaxItems;
  if (uf)
    for (uint32_t i = threadIdx.x; i < FW; i += blockDim.x) filt[i] = filter[i];
  for (uint32_t i = threadIdx.x; i < (uint32_t)kCollectCache; i += blockDim.x) cache[i] = kEmptyKey;
  stage_tables<DP>(ti, FP ? t.tabq : (HM == kHashPacked ? t.tabp : t.tabi), mesh.nch);
  constexpr uint32_t kNeedCS = D - ((D - 1) >> 1);
  const uint32_t need = t.cm ? (uint32_t)D : kNeedCS;
  constexpr uint32_t NT = kCollectThreads;
  const uint64_t chunk = (uint64_t)NT * PPT;
  bool bad = false;
  for (uint64_t first = (uint64_t)blockIdx.x * chunk; first < n; first += (uint64_t)gridDim.x * chunk) {
    const bool full = first + chunk <= n;
    // all PPT position loads are issued before any is used (a clamped index keeps the
    // loads unconditional; particles beyond the stream are masked below)
    float px[PPT], py[PPT], pz[PPT];
    uint64_t pw[PPT];
    const uint64_t last = n - 1;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      uint64_t i = first + (uint64_t)j * NT + threadIdx.x;
      i = i < last ? i : last;
      if constexpr (MODE == kMeshPacked) {
        pw[j] = __builtin_nontemporal_load((const uint64_t*)pos + i);
      } else {
        px[j] = __builtin_nontemporal_load(pos + 3 * i);
        py[j] = __builtin_nontemporal_load(pos + 3 * i + 1);
        pz[j] = __builtin_nontemporal_load(pos + 3 * i + 2);
      }
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
          row_hashes<4>(ti, keys[j], mesh.nch, q);
#pragma unroll
          for (int r = 0; r < D; ++r) {
            const FilterProbe pr = field_probe(field_bits<kFieldBits>(q, r));
            fp += ((filt[pr.word] & pr.mask) == pr.mask) ? 1u : 0u;
          }
        } else {
          uint32_t bk[D], sg[D];
          rows_bucket_sign<D, HM>(ti, keys[j], mesh.nch, t.w, t.wshift, bk, sg);
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
          rows_bucket_sign<D, HM>(tx, keys[j0 + q], nchx, t.w, t.wshift, bk, ng);
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
        rows_bucket_sign<D, HM>(tx, keys[j], nchx, t.w, t.wshift, bk, ng);
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

// Candidate pass over the whole dictionary (Count Sketch with Full Search, Sec. 2.2
// item 1; Alg. 1): every key in [0, nkeys) is estimated once, so no key cache or set
// lookup is needed.  Keys whose rows pass the Bloom filter fewer than `need` times are
// dropped; the rest take the exact test (hot-item set or counter reads) and, if they
// pass, go into the set.  d <= 8, tables in LDS.
template <int D, int HM>
__global__ __launch_bounds__(kCollectThreads) void dict_collect_kernel(uint64_t nkeys, Mesh mesh, Tables t,
                                                                       const int32_t* __restrict__ M, int32_t theta,
                                                                       const uint32_t* __restrict__ filter,
                                                                       const uint32_t* __restrict__ hot,
                                                                       uint32_t use_filter,
                                                                       const uint32_t* __restrict__ hot_table,
                                                                       uint64_t* set, uint32_t slot_mask,
                                                                       uint32_t* set_count, uint32_t max_cand,
                                                                       uint32_t* err) {
  constexpr int DP = HashWords<D, HM>::value;
  extern __shared__ __align__(16) uint32_t lds4[];
  uint32_t* ti = lds4;
  uint32_t* filt = ti + kTableWords * DP;
  const uint32_t nhot = use_filter ? *hot : 0xFFFFFFFFu;
  const bool uf = use_filter && nhot <= kFilterMaxItems;
  const bool uh = use_filter && hot_table != nullptr && nhot <= kHotMaxItems;
  if (uf)
    for (uint32_t i = threadIdx.x; i < (uint32_t)kFilterWords; i += blockDim.x) filt[i] = filter[i];
  stage_tables<DP>(ti, HM == kHashPacked ? t.tabp : t.tabi, mesh.nch);
  constexpr uint32_t kNeedCS = D - ((D - 1) >> 1);
  const uint32_t need = t.cm ? (uint32_t)D : kNeedCS;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t key = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; key < nkeys; key += stride) {
    uint32_t bk[D], ng[D];
    rows_bucket_sign<D, HM>(ti, key, mesh.nch, t.w, t.wshift, bk, ng);
#pragma unroll
    for (int r = 0; r < D; ++r) ng[r] &= t.cm ^ 1u;
    if (uf) {
      uint32_t fp = 0;
#pragma unroll
      for (int r = 0; r < D; ++r) {
        const FilterProbe pr = filter_probe((uint32_t)r, bk[r], ng[r], t.bnorm);
        fp += ((filt[pr.word] & pr.mask) == pr.mask) ? 1u : 0u;
      }
      if (fp < need) continue;
    }
    uint32_t pass = 0;
    if (uh) {
#pragma unroll
      for (int r = 0; r < D; ++r) {
        if (pass >= need || pass + (uint32_t)(D - r) < need) break;
        const uint32_t item = hot_item((uint32_t)r, bk[r], ng[r]);
        uint32_t sl = hot_slot(item);
        for (uint32_t probe = 0; probe < kHotSlots; ++probe) {
          const uint32_t v = hot_table[sl];
          if (v == item) {
            ++pass;
            break;
          }
          if (v == kHotEmpty) break;
          sl = (sl + 1) & (kHotSlots - 1);
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < D; ++r) {
        if (pass >= need || pass + (uint32_t)(D - r) < need) break;
        const uint32_t c = (uint32_t)M[(uint64_t)r * t.w + bk[r]];
        if ((int32_t)(ng[r] ? 0u - c : c) >= theta) ++pass;
      }
    }
    if (pass >= need) set_insert(set, slot_mask, key, set_count, max_cand, err);
  }
}

// The same for any d, with row-major tables read from global memory (d > 8).
__global__ __launch_bounds__(256) void dict_collect_generic_kernel(uint64_t nkeys, Tables t,
                                                                   const int32_t* __restrict__ M, int32_t theta,
                                                                   uint64_t* set, uint32_t slot_mask,
                                                                   uint32_t* set_count, uint32_t max_cand,
                                                                   uint32_t* err) {
  const uint32_t need = t.cm ? t.d : t.d - ((t.d - 1) >> 1);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t key = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; key < nkeys; key += stride) {
    uint32_t pass = 0;
    for (uint32_t r = 0; r < t.d; ++r) {
      if (pass >= need || pass + (t.d - r) < need) break;
      if (row_estimate(t.tab + r * kTableWords, M + (uint64_t)r * t.w, t.w, t.cm, key) >= theta) ++pass;
    }
    if (pass >= need) set_insert(set, slot_mask, key, set_count, max_cand, err);
  }
}

// The keys of a candidate set as a list (order unspecified): out[0 .. *count).  At most
// `cap` are written; more keys than that latches the capacity error in *err.
__global__ __launch_bounds__(256) void set_list_kernel(const uint64_t* __restrict__ set, uint32_t slots,
                                                       uint64_t* __restrict__ out, uint32_t* count, uint32_t cap,
                                                       uint32_t* err) {
  for (uint32_t i0 = blockIdx.x * blockDim.x; i0 < slots; i0 += gridDim.x * blockDim.x) {
    const uint32_t i = i0 + threadIdx.x;
    const uint64_t key = (i < slots) ? set[i] : kEmptyKey;
    const bool have = key != kEmptyKey;
    const uint32_t slot = wave_append(count, have);
    if (have) {
      if (slot < cap) out[slot] = key;
      else atomicOr(err, kErrCapacity);
    }
  }
}

// Every key of the router's exact table joins a candidate set.
__global__ __launch_bounds__(256) void table_to_set_kernel(const uint64_t* __restrict__ tk, uint32_t tslots, uint64_t* set,
                                                           uint32_t slot_mask, uint32_t* set_count, uint32_t max_cand,
                                                           uint32_t* err) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < tslots; i += gridDim.x * blockDim.x) {
    const uint64_t key = tk[i];
    if (key != kEmptyKey) set_insert(set, slot_mask, key, set_count, max_cand, err);
  }
}

hipError_t launch_table_to_set(const uint64_t* tk, uint32_t tslots, uint64_t* set, uint32_t slot_mask,
                               uint32_t* set_count, uint32_t max_cand, uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(table_to_set_kernel, dim3(grid_for(tslots, 256, 1024)), dim3(256), 0, s, tk, tslots, set,
                     slot_mask, set_count, max_cand, err);
  return hipGetLastError();
}

// Second layer of the hierarchical query (Alg. 3): for each super-item j of the list,
// every child key of [j R, min((j + 1) R, ncells)) is estimated from the fine counters
// and goes into the fine set if its estimate is >= theta.  One workgroup per super-item
// at a time, children spread over the threads.
template <int MAXD, bool TAB_LDS>
__global__ __launch_bounds__(256) void children_kernel(const uint64_t* __restrict__ list,
                                                       const uint32_t* __restrict__ count, uint32_t cap,
                                                       uint32_t group, uint64_t ncells, Tables t,
                                                       const int32_t* __restrict__ M, int32_t theta, uint64_t* set,
                                                       uint32_t slot_mask, uint32_t* set_count, uint32_t max_cand,
                                                       uint32_t* err) {
  __shared__ uint32_t tabs_lds[TAB_LDS ? kTabLdsRows * kTableWords : 1];
  const uint32_t* tabs = t.tab;
  if (TAB_LDS) {
    load_tables(tabs_lds, t.tab, t.d);
    __syncthreads();
    tabs = tabs_lds;
  }
  const uint32_t m = min(*count, cap);
  for (uint32_t i = blockIdx.x; i < m; i += gridDim.x) {
    const uint64_t lo = list[i] * group;
    const uint64_t hi = (lo + group < ncells) ? lo + group : ncells;
    for (uint64_t c = lo + threadIdx.x; c < hi; c += blockDim.x)
      if (estimate_key<MAXD>(tabs, M, t.d, t.w, t.cm, c) >= theta) set_insert(set, slot_mask, c, set_count, max_cand, err);
  }
}

hipError_t launch_collect_children(const uint64_t* coarse_set, uint32_t coarse_slots, uint64_t* list,
                                   uint32_t* list_count, uint32_t list_cap, uint32_t group, uint64_t ncells,
                                   const Tables& t, const int32_t* M, int32_t theta, uint64_t* set,
                                   uint32_t slot_mask, uint32_t* set_count, uint32_t max_cand, uint32_t* err,
                                   hipStream_t s) {
  hipError_t e = launch_fill_u32(list_count, 1, 0u, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(set_list_kernel, dim3(grid_for(coarse_slots, 256, 4096)), dim3(256), 0, s, coarse_set,
                     coarse_slots, list, list_count, list_cap, err);
  const dim3 grid(2048), block(256);
  if (t.d <= (uint32_t)kTabLdsRows)
    hipLaunchKernelGGL((children_kernel<kTabLdsRows, true>), grid, block, 0, s, list, list_count, list_cap, group,
                       ncells, t, M, theta, set, slot_mask, set_count, max_cand, err);
  else
    hipLaunchKernelGGL((children_kernel<32, false>), grid, block, 0, s, list, list_count, list_cap, group, ncells, t,
                       M, theta, set, slot_mask, set_count, max_cand, err);
  return hipGetLastError();
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
// fcols != NULL: the field-probe filter (item fields from the row maps' columns, w = 2^lw);
// else the hashed probe of filter_probe().
__global__ __launch_bounds__(256) void filter_build_kernel(const int32_t* __restrict__ M, uint32_t d, uint32_t w,
                                                           uint32_t cm, uint32_t bnorm, int32_t theta,
                                                           const uint32_t* __restrict__ fcols, uint32_t lw,
                                                           uint32_t* __restrict__ filter, uint32_t* __restrict__ hot) {
  __shared__ uint32_t count;
  if (threadIdx.x == 0) count = 0;
  __syncthreads();
  uint32_t mine = 0;
  const uint64_t span = (uint64_t)gridDim.x * blockDim.x * 4 * kFilterVec;
  for (uint32_t r = 0; r < d; ++r) {
    const int32_t* __restrict__ Mr = M + (uint64_t)r * w;
    for (uint64_t b0 = (uint64_t)blockIdx.x * blockDim.x * 4 * kFilterVec; b0 < w; b0 += span) {
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
            const FilterProbe pr = fcols ? field_probe(item_field(fcols + r * kFieldCols, (uint32_t)(b + e)))
                                         : filter_probe(r, (uint32_t)(b + e), 0u, bnorm);
            atomicOr(&filter[pr.word], pr.mask);
          }
          if (hn) {
            const FilterProbe pr = fcols ? field_probe(item_field(fcols + r * kFieldCols, (1u << lw) | (uint32_t)(b + e)))
                                         : filter_probe(r, (uint32_t)(b + e), 1u, bnorm);
            atomicOr(&filter[pr.word], pr.mask);
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
__global__ __launch_bounds__(256) void hot_build_kernel(const int32_t* __restrict__ M, uint32_t d, uint32_t w,
                                                        uint32_t cm, int32_t theta, const uint32_t* __restrict__ hot,
                                                        uint32_t* __restrict__ hot_table) {
  if (*hot > kHotMaxItems) return;
  const uint64_t span = (uint64_t)gridDim.x * blockDim.x * 4 * kFilterVec;
  for (uint32_t r = 0; r < d; ++r) {
    const int32_t* __restrict__ Mr = M + (uint64_t)r * w;
    for (uint64_t b0 = (uint64_t)blockIdx.x * blockDim.x * 4 * kFilterVec; b0 < w; b0 += span) {
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
                     field ? t.fcols : nullptr, t.lw, filter, hot);
  if (hot_table != nullptr)
    hipLaunchKernelGGL(hot_build_kernel, grid, dim3(256), 0, s, M, t.d, t.w, t.cm, theta, hot, hot_table);
  return hipGetLastError();
}

struct CollectArgs {
  const float* pos;
  uint64_t n;
  Mesh mesh;
  Tables t;
  const int32_t* M;
  int32_t theta;
  const uint32_t* filter;
  const uint32_t* hot;
  uint32_t use_filter;
  const uint32_t* hot_table;
  uint64_t* set;
  uint32_t slot_mask;
  uint32_t* set_count;
  uint32_t max_cand;
  uint32_t* err;
  bool field;   // the filter is a field-probe filter (collect2_kernel<..., FP = true>)
};

template <int D, uint32_t MM, int HM, bool FP = false>
static void launch_collect2_one(dim3 grid, dim3 block, size_t lds, hipStream_t s, const CollectArgs& c) {
  hipLaunchKernelGGL((collect2_kernel<D, MM, HM, FP>), grid, block, lds, s, c.pos, c.n, c.mesh, c.t, c.M, c.theta,
                     c.filter, c.hot, c.use_filter, c.hot_table, c.set, c.slot_mask, c.set_count, c.max_cand, c.err);
}

template <int D, uint32_t MM>
static void launch_collect2_m(int hm, dim3 grid, dim3 block, size_t lds, hipStream_t s, const CollectArgs& c) {
  if constexpr (D == 5) {
    if (hm == kHashPacked && c.field) {
      launch_collect2_one<D, MM, kHashPacked, true>(grid, block, lds, s, c);
      return;
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
                               const CollectArgs& c) {
  if (mode == kMeshPacked) launch_collect2_m<D, kMeshPacked>(hm, grid, block, lds, s, c);
  else if (mode == kMeshPow2Ratio) launch_collect2_m<D, kMeshPow2Ratio>(hm, grid, block, lds, s, c);
  else if (mode == kMeshExactRatio) launch_collect2_m<D, kMeshExactRatio>(hm, grid, block, lds, s, c);
  else launch_collect2_m<D, kMeshGeneral>(hm, grid, block, lds, s, c);
}

static void launch_collect2_d(uint32_t d, uint32_t mode, int hm, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                              const CollectArgs& c) {
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

template <int D, int HM>
static void launch_dict_one(dim3 grid, dim3 block, size_t lds, hipStream_t s, uint64_t nkeys, const Mesh& mesh,
                            const Tables& t, const int32_t* M, int32_t theta, const uint32_t* filter,
                            const uint32_t* hot, uint32_t use_filter, const uint32_t* hot_table, uint64_t* set,
                            uint32_t slot_mask, uint32_t* set_count, uint32_t max_cand, uint32_t* err) {
  hipLaunchKernelGGL((dict_collect_kernel<D, HM>), grid, block, lds, s, nkeys, mesh, t, M, theta, filter, hot,
                     use_filter, hot_table, set, slot_mask, set_count, max_cand, err);
}

template <int D>
static void launch_dict_d(int hm, dim3 grid, dim3 block, size_t lds, hipStream_t s, uint64_t nkeys, const Mesh& mesh,
                          const Tables& t, const int32_t* M, int32_t theta, const uint32_t* filter,
                          const uint32_t* hot, uint32_t use_filter, const uint32_t* hot_table, uint64_t* set,
                          uint32_t slot_mask, uint32_t* set_count, uint32_t max_cand, uint32_t* err) {
  if constexpr (D >= 5) {
    if (hm == kHashPacked) {
      launch_dict_one<D, kHashPacked>(grid, block, lds, s, nkeys, mesh, t, M, theta, filter, hot, use_filter,
                                      hot_table, set, slot_mask, set_count, max_cand, err);
      return;
    }
  }
  if (hm == kHashMulHi)
    launch_dict_one<D, kHashMulHi>(grid, block, lds, s, nkeys, mesh, t, M, theta, filter, hot, use_filter, hot_table,
                                   set, slot_mask, set_count, max_cand, err);
  else
    launch_dict_one<D, kHashShift>(grid, block, lds, s, nkeys, mesh, t, M, theta, filter, hot, use_filter, hot_table,
                                   set, slot_mask, set_count, max_cand, err);
}

hipError_t launch_collect_dictionary(uint64_t nkeys, const Mesh& mesh, const Tables& t, const int32_t* M,
                                     int32_t theta, const uint32_t* filter, const uint32_t* hot,
                                     const uint32_t* hot_table, uint64_t* set, uint32_t slot_mask,
                                     uint32_t* set_count, uint32_t max_cand, uint32_t* err, hipStream_t s) {
  if (t.d <= (uint32_t)kTabLdsRows) {
    const uint32_t use_filter = (filter != nullptr && hot != nullptr) ? 1u : 0u;
    const size_t lds = ((size_t)kTableWords * t.dp + (use_filter ? kFilterWords : 0)) * sizeof(uint32_t);
    const dim3 grid(grid_for(nkeys, kCollectThreads, 1024)), block(kCollectThreads);
    const int hm = t.hash_mode();
#define CSK_DICT(DD)                                                                                    \
  launch_dict_d<DD>(hm, grid, block, lds, s, nkeys, mesh, t, M, theta, filter, hot, use_filter, hot_table, set, \
                    slot_mask, set_count, max_cand, err)
    switch (t.d) {
      case 1: CSK_DICT(1); break;
      case 2: CSK_DICT(2); break;
      case 3: CSK_DICT(3); break;
      case 4: CSK_DICT(4); break;
      case 5: CSK_DICT(5); break;
      case 6: CSK_DICT(6); break;
      case 7: CSK_DICT(7); break;
      default: CSK_DICT(8); break;
    }
#undef CSK_DICT
  } else {
    hipLaunchKernelGGL(dict_collect_generic_kernel, dim3(grid_for(nkeys, 256, 8192)), dim3(256), 0, s, nkeys, t, M,
                       theta, set, slot_mask, set_count, max_cand, err);
  }
  return hipGetLastError();
}

hipError_t launch_collect(const float* pos, uint64_t n, const Mesh& mesh, const Tables& t, const int32_t* M,
                          int32_t theta, const uint32_t* filter, const uint32_t* hot, const uint32_t* hot_table,
                          uint64_t* set, uint32_t slot_mask, uint32_t* set_count, uint32_t max_cand, uint32_t* err,
                          bool field, hipStream_t s) {
  if (t.d <= (uint32_t)kTabLdsRows && mesh.group == 1u) {   // collect2_kernel takes ungrouped keys
    const uint32_t use_filter = (filter != nullptr && hot != nullptr) ? 1u : 0u;
    field = field && use_filter && t.d == 5 && t.hash_mode() == kHashPacked && t.tabq != nullptr;
    const size_t lds = field ? ((size_t)kTableWords * 4 + 2 * kCollectCache + kFieldFilterWords) * sizeof(uint32_t)
                             : ((size_t)kTableWords * t.dp + 2 * kCollectCache + (use_filter ? kFilterWords : 0)) *
                                   sizeof(uint32_t);
    const dim3 grid(grid_for((n + kCollectPPT - 1) / kCollectPPT, kCollectThreads, 256)), block(kCollectThreads);
    const CollectArgs ca{pos, n, mesh, t, M, theta, filter, hot, use_filter, hot_table, set, slot_mask, set_count,
                         max_cand, err, field};
    launch_collect2_d(t.d, mesh.mode, t.hash_mode(), grid, block, lds, s, ca);
  } else {
    hipLaunchKernelGGL(collect_kernel<false>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, pos, n, mesh, t, M, theta,
                       set, slot_mask, set_count, max_cand, err);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ fills

__global__ void fill_u64_kernel(uint64_t* p, uint64_t n, uint64_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}
__global__ void fill_u32_kernel(uint32_t* p, uint64_t n, uint32_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}
hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// Word i of the concatenated spans goes to the span it falls in (spans of length 0 are skipped).
__global__ void fill_spans_kernel(FillSpans f) {
  const uint64_t total = f.n[0] + f.n[1] + f.n[2] + f.n[3];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    uint64_t j = i;
    int r = 0;
    while (r < kFillSpans - 1 && j >= f.n[r]) {
      j -= f.n[r];
      ++r;
    }
    f.p[r][j] = f.v[r];
  }
}
hipError_t launch_fill_spans(const FillSpans& f, hipStream_t s) {
  uint64_t total = 0;
  for (int r = 0; r < kFillSpans; ++r) total += f.n[r];
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_spans_kernel, dim3(grid_for(total, 256, 4096)), dim3(256), 0, s, f);
  return hipGetLastError();
}

// ------------------------------------------------------------------ top-k

__device__ __forceinline__ void sel_init_body(SelState* st) {
  uint32_t* w = (uint32_t*)st;
  for (uint32_t i = threadIdx.x; i < sizeof(SelState) / 4; i += blockDim.x) w[i] = 0;
}
__global__ void sel_init_kernel(SelState* st) { sel_init_body(st); }

// Distinct keys of the set -> (key, estimate from the current counters).
// Exact count of key in the router's table (linear probing from table_slot), or -1.
__device__ __forceinline__ int64_t table_count(const uint64_t* __restrict__ tk, const uint32_t* __restrict__ tc,
                                               uint32_t tmask, uint64_t key) {
  uint32_t sl = table_slot(key, tmask);
  for (uint32_t probe = 0; probe <= tmask; ++probe) {
    const uint64_t k = tk[sl];
    if (k == key) return (int64_t)tc[sl];
    if (k == kEmptyKey) return -1;
    sl = (sl + 1) & tmask;
  }
  return -1;
}

// With an exact table (ov_keys != NULL), a candidate found in it takes its exact count
// as its estimate (the learned router's table; counts of up to 2^31 - 1).
template <int MAXD, bool TAB_LDS>
__device__ __forceinline__ void compact_body(const uint64_t* __restrict__ set, uint32_t slots, Tables t,
                                                      const int32_t* __restrict__ M, uint32_t max_cand,
                                                      SelState* st, uint64_t* __restrict__ ck,
                                                      int32_t* __restrict__ ce, const uint64_t* __restrict__ ov_keys,
                                                      const uint32_t* __restrict__ ov_counts, uint32_t ov_mask) {
  __shared__ uint32_t tabs_lds[TAB_LDS ? kTabLdsRows * kTableWords : 1];
  const uint32_t* tabs = t.tab;
  if (TAB_LDS) {
    load_tables(tabs_lds, t.tab, t.d);
    __syncthreads();
    tabs = tabs_lds;
  }
  for (uint32_t i0 = blockIdx.x * blockDim.x; i0 < slots; i0 += gridDim.x * blockDim.x) {
    const uint32_t i = i0 + threadIdx.x;
    const uint64_t key = (i < slots) ? set[i] : kEmptyKey;
    const bool have = key != kEmptyKey;
    const uint32_t slot = wave_append(&st->m, have);
    if (have && slot < max_cand) {
      ck[slot] = key;
      const int64_t exact = ov_keys ? table_count(ov_keys, ov_counts, ov_mask, key) : -1;
      ce[slot] = exact >= 0 ? (int32_t)exact : estimate_key<MAXD>(tabs, M, t.d, t.w, t.cm, key);
    }
  }
}
template <int MAXD, bool TAB_LDS>
__global__ __launch_bounds__(256) void compact_kernel(const uint64_t* __restrict__ set, uint32_t slots, Tables t,
                                                      const int32_t* __restrict__ M, uint32_t max_cand,
                                                      SelState* st, uint64_t* __restrict__ ck,
                                                      int32_t* __restrict__ ce, const uint64_t* __restrict__ ov_keys,
                                                      const uint32_t* __restrict__ ov_counts, uint32_t ov_mask) {
  compact_body<MAXD, TAB_LDS>(set, slots, t, M, max_cand, st, ck, ce, ov_keys, ov_counts, ov_mask);
}

__device__ __forceinline__ void clamp_m_body(SelState* st, uint32_t max_cand) {
  if (threadIdx.x == 0 && st->m > max_cand) st->m = max_cand;
}
__global__ void clamp_m_kernel(SelState* st, uint32_t max_cand) { clamp_m_body(st, max_cand); }

// Histogram of one 8-bit digit over the current class (stage 1: est; stage 2: key
// among est == T).
template <bool KEYS>
__device__ __forceinline__ void sel_hist_body(const uint64_t* __restrict__ ck, const int32_t* __restrict__ ce,
                                                       SelState* st, int shift) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t m = st->m;
  const uint32_t epre = st->est_prefix, emask = st->est_mask;
  const uint64_t kpre = st->key_prefix, kmask = st->key_mask;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const uint32_t u = (uint32_t)ce[i] ^ 0x80000000u;
    if (!KEYS) {
      if ((u & emask) == epre) atomicAdd(&h[(u >> shift) & 255u], 1u);
    } else {
      const uint64_t k = ck[i];
      if (u == epre && (k & kmask) == kpre) atomicAdd(&h[(uint32_t)(k >> shift) & 255u], 1u);
    }
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&st->hist[threadIdx.x], h[threadIdx.x]);
}
template <bool KEYS>
__global__ __launch_bounds__(256) void sel_hist_kernel(const uint64_t* __restrict__ ck, const int32_t* __restrict__ ce,
                                                       SelState* st, int shift) {
  sel_hist_body<KEYS>(ck, ce, st, shift);
}

// Pick the digit holding the k_rem-th item: descending for estimates, ascending for keys.
// One wave: position q of the scan order is digit 255 - q (estimates) or q (keys); lane l
// holds positions 4l .. 4l + 3.  The chosen position is the first whose inclusive prefix
// count reaches k_rem, or the last one (255) when none does; k_rem becomes k_rem minus the
// count before it.  The histogram is cleared for the next pass.
template <bool KEYS>
__device__ __forceinline__ void sel_pick_body(SelState* st, uint32_t k, int shift) {
  const uint32_t lane = threadIdx.x;
  if (!KEYS && shift == 24 && lane == 0) st->k_rem = min(k, st->m);
  __syncthreads();
  const uint32_t need = st->k_rem;
  uint32_t h[4], sum = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t q = lane * 4 + (uint32_t)e;
    h[e] = st->hist[KEYS ? q : 255u - q];
    sum += h[e];
  }
  const uint32_t incl = wave_incl_scan(sum);
  if (need > 0) {
    const uint64_t hit = __ballot(incl >= need);
    const uint32_t lead = hit ? (uint32_t)__ffsll((unsigned long long)hit) - 1u : 63u;
    if (lane == lead) {
      uint32_t cum = incl - sum, q = lane * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        q = lane * 4 + (uint32_t)e;
        if (q == 255u || cum + h[e] >= need) break;
        cum += h[e];
      }
      const uint32_t dg = KEYS ? q : 255u - q;
      if (!KEYS) {
        st->est_prefix |= dg << shift;
        st->est_mask |= 255u << shift;
      } else {
        st->key_prefix |= (uint64_t)dg << shift;
        st->key_mask |= 255ull << shift;
      }
      st->k_rem = need - cum;
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 4; ++e) st->hist[lane * 4 + (uint32_t)e] = 0;
}
template <bool KEYS>
__global__ __launch_bounds__(64) void sel_pick_kernel(SelState* st, uint32_t k, int shift) {
  sel_pick_body<KEYS>(st, k, shift);
}

// Winners: est > T, or est == T and key <= K (T, K from the two stages).
__device__ __forceinline__ void sel_gather_body(const uint64_t* __restrict__ ck, const int32_t* __restrict__ ce,
                                                         SelState* st, uint32_t k, uint64_t* __restrict__ sk,
                                                         int32_t* __restrict__ se) {
  const uint32_t m = st->m;
  const uint32_t T = st->est_prefix;
  const uint64_t K = st->key_prefix;
  const bool any = min(k, m) > 0;
  for (uint32_t i0 = blockIdx.x * blockDim.x; i0 < m; i0 += gridDim.x * blockDim.x) {
    const uint32_t i = i0 + threadIdx.x;
    bool take = false;
    uint64_t key = 0;
    int32_t e = 0;
    if (i < m && any) {
      key = ck[i];
      e = ce[i];
      const uint32_t u = (uint32_t)e ^ 0x80000000u;
      take = (u > T) || (u == T && key <= K);
    }
    const uint32_t slot = wave_append(&st->n_sel, take);
    if (take && slot < k) {
      sk[slot] = key;
      se[slot] = e;
    }
  }
}
__global__ __launch_bounds__(256) void sel_gather_kernel(const uint64_t* __restrict__ ck, const int32_t* __restrict__ ce,
                                                         SelState* st, uint32_t k, uint64_t* __restrict__ sk,
                                                         int32_t* __restrict__ se) {
  sel_gather_body(ck, ce, st, k, sk, se);
}

// Place each winner at its rank in (est desc, key asc); keys are distinct.
// Rank of winner i = number of winners ahead of it in (estimate desc, key asc) order.
// Block (x, y) counts, for the 256 winners of tile x, those ahead of them among the
// `chunk` winners of chunk y, and adds the partial counts to rank[].  Keys are distinct,
// so the ranks are a permutation of [0, n).
constexpr uint32_t kRankChunk = 1024;      // smallest chunk
constexpr uint32_t kMaxGridY = 65535;
__device__ __forceinline__ void rank_count_body(const uint64_t* __restrict__ sk, const int32_t* __restrict__ se,
                                                const SelState* st, uint32_t k, uint32_t chunk,
                                                uint32_t* __restrict__ rank, uint32_t cy = blockIdx.y) {
  __shared__ uint64_t tk[256];
  __shared__ int32_t te[256];
  const uint32_t n = min(st->n_sel, k);
  const uint32_t i0 = blockIdx.x * 256;
  const uint64_t j_lo64 = (uint64_t)cy * chunk;
  if (i0 >= n || j_lo64 >= n) return;   // uniform over the block
  const uint32_t j_lo = (uint32_t)j_lo64;
  const uint32_t j_hi = (uint32_t)min((uint64_t)n, j_lo64 + chunk);
  const uint32_t i = i0 + threadIdx.x;
  const bool act = i < n;
  const uint64_t ki = act ? sk[i] : 0;
  const int32_t ei = act ? se[i] : 0;
  uint32_t cnt = 0;
  for (uint32_t j0 = j_lo; j0 < j_hi; j0 += 256) {
    __syncthreads();
    if (j0 + threadIdx.x < j_hi) {
      tk[threadIdx.x] = sk[j0 + threadIdx.x];
      te[threadIdx.x] = se[j0 + threadIdx.x];
    }
    __syncthreads();
    const uint32_t lim = min(256u, j_hi - j0);
    for (uint32_t t = 0; t < lim; ++t) cnt += (te[t] > ei) || (te[t] == ei && tk[t] < ki);
  }
  if (act && cnt) atomicAdd(&rank[i], cnt);
}
__global__ __launch_bounds__(256) void rank_count_kernel(const uint64_t* __restrict__ sk, const int32_t* __restrict__ se,
                                                         const SelState* st, uint32_t k, uint32_t chunk,
                                                         uint32_t* __restrict__ rank) {
  rank_count_body(sk, se, st, k, chunk, rank);
}

__device__ __forceinline__ void rank_place_body(const uint64_t* __restrict__ sk, const int32_t* __restrict__ se,
                                                         const SelState* st, uint32_t k,
                                                         const uint32_t* __restrict__ rank, uint64_t* __restrict__ ok,
                                                         int32_t* __restrict__ oe) {
  const uint32_t n = min(st->n_sel, k);
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const uint32_t r = rank[i];
    ok[r] = sk[i];
    oe[r] = se[i];
  }
}
__global__ __launch_bounds__(256) void rank_place_kernel(const uint64_t* __restrict__ sk, const int32_t* __restrict__ se,
                                                         const SelState* st, uint32_t k,
                                                         const uint32_t* __restrict__ rank, uint64_t* __restrict__ ok,
                                                         int32_t* __restrict__ oe) {
  rank_place_body(sk, se, st, k, rank, ok, oe);
}

// Number written and status of a top-k, for callers that do not synchronize: out[0] =
// min(k, m); out[1] = 1 (incomplete) when fewer than k were found from a partial set.
__device__ __forceinline__ void topk_out_body(const SelState* st, uint32_t k, uint32_t partial, uint32_t* out) {
  if (threadIdx.x == 0) {
    const uint32_t got = min(k, st->m);
    out[0] = got;
    out[1] = (got < k && partial) ? 1u : 0u;
  }
}
__global__ void topk_out_kernel(const SelState* st, uint32_t k, uint32_t partial, uint32_t* out) {
  topk_out_body(st, k, partial, out);
}

hipError_t launch_topk_out(const SelState* st, uint32_t k, uint32_t partial, uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(topk_out_kernel, dim3(1), dim3(64), 0, s, st, k, partial, out);
  return hipGetLastError();
}

__device__ __forceinline__ void sel_finish_body(SelState* st, const uint32_t* err) {
  if (threadIdx.x == 0) st->err = *err;
}
__global__ void sel_finish_kernel(SelState* st, const uint32_t* err) { sel_finish_body(st, err); }

__global__ void sel_set_m_kernel(SelState* st, uint32_t m) {
  if (threadIdx.x == 0) st->m = m;
}

// Radix select of the top k of the st->m pairs (ck, ce) in (ce desc, ck asc) order (ck
// below 2^48), then the winners placed at their ranks in ok / oe.  rank: k words.
static hipError_t select_stages(const uint64_t* ck, const int32_t* ce, uint32_t m_max, uint32_t k, SelState* st,
                                uint64_t* sk, int32_t* se, uint32_t* rank, uint64_t* ok, int32_t* oe,
                                const uint32_t* err, hipStream_t s) {
  const dim3 hgrid(grid_for(m_max, 256, 1024));
  for (int shift = 24; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(sel_hist_kernel<false>, hgrid, dim3(256), 0, s, ck, ce, st, shift);
    hipLaunchKernelGGL(sel_pick_kernel<false>, dim3(1), dim3(64), 0, s, st, k, shift);
  }
  for (int shift = 40; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(sel_hist_kernel<true>, hgrid, dim3(256), 0, s, ck, ce, st, shift);
    hipLaunchKernelGGL(sel_pick_kernel<true>, dim3(1), dim3(64), 0, s, st, k, shift);
  }
  hipLaunchKernelGGL(sel_gather_kernel, hgrid, dim3(256), 0, s, ck, ce, st, k, sk, se);
  hipError_t e = launch_fill_u32(rank, k, 0u, s);
  if (e != hipSuccess) return e;
  uint64_t chunk = kRankChunk;
  while ((k + chunk - 1) / chunk > kMaxGridY) chunk *= 2;
  hipLaunchKernelGGL(rank_count_kernel, dim3((k + 255) / 256, (uint32_t)((k + chunk - 1) / chunk)), dim3(256), 0, s,
                     sk, se, st, k, (uint32_t)chunk, rank);
  hipLaunchKernelGGL(rank_place_kernel, dim3(grid_for(k, 256, 1024)), dim3(256), 0, s, sk, se, st, k, rank, ok, oe);
  hipLaunchKernelGGL(sel_finish_kernel, dim3(1), dim3(64), 0, s, st, err);
  return hipGetLastError();
}

// ---- the top-k of many sketches at once: block row blockIdx.y (blockIdx.z for the rank
// count) serves sketch y of the descriptors; per-call k and outputs come by value.
__global__ void sel_init_batch_kernel(const TopkDesc* __restrict__ D) { sel_init_body(D[blockIdx.y].st); }

template <int MAXD, bool TAB_LDS>
__global__ __launch_bounds__(256) void compact_batch_kernel(const TopkDesc* __restrict__ D) {
  const TopkDesc& d = D[blockIdx.y];
  compact_body<MAXD, TAB_LDS>(d.set, d.slots, d.t, d.M, d.max_cand, d.st, d.ck, d.ce, nullptr, nullptr, 0u);
}

__global__ void clamp_m_batch_kernel(const TopkDesc* __restrict__ D) {
  clamp_m_body(D[blockIdx.y].st, D[blockIdx.y].max_cand);
}

template <bool KEYS>
__global__ __launch_bounds__(256) void sel_hist_batch_kernel(const TopkDesc* __restrict__ D, int shift) {
  const TopkDesc& d = D[blockIdx.y];
  sel_hist_body<KEYS>(d.ck, d.ce, d.st, shift);
}

template <bool KEYS>
__global__ __launch_bounds__(64) void sel_pick_batch_kernel(const TopkDesc* __restrict__ D, TopkCall call, int shift) {
  sel_pick_body<KEYS>(D[blockIdx.y].st, call.k[blockIdx.y], shift);
}

__global__ __launch_bounds__(256) void sel_gather_batch_kernel(const TopkDesc* __restrict__ D, TopkCall call) {
  const TopkDesc& d = D[blockIdx.y];
  sel_gather_body(d.ck, d.ce, d.st, call.k[blockIdx.y], d.sk, d.se);
}

// ranks live in the first k words of each sketch's candidate estimates (no longer needed)
__global__ __launch_bounds__(256) void rank_clear_batch_kernel(const TopkDesc* __restrict__ D, TopkCall call) {
  uint32_t* r = (uint32_t*)D[blockIdx.y].ce;
  const uint32_t k = call.k[blockIdx.y];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) r[i] = 0;
}

__global__ __launch_bounds__(256) void rank_count_batch_kernel(const TopkDesc* __restrict__ D, TopkCall call,
                                                               uint32_t chunk) {
  const TopkDesc& d = D[blockIdx.z];
  rank_count_body(d.sk, d.se, d.st, call.k[blockIdx.z], chunk, (uint32_t*)d.ce, blockIdx.y);
}

__global__ __launch_bounds__(256) void rank_place_batch_kernel(const TopkDesc* __restrict__ D, TopkCall call) {
  const TopkDesc& d = D[blockIdx.y];
  rank_place_body(d.sk, d.se, d.st, call.k[blockIdx.y], (const uint32_t*)d.ce, call.keys[blockIdx.y],
                  call.est[blockIdx.y]);
}

__global__ void sel_finish_out_batch_kernel(const TopkDesc* __restrict__ D, TopkCall call) {
  const TopkDesc& d = D[blockIdx.y];
  sel_finish_body(d.st, d.err);
  topk_out_body(d.st, call.k[blockIdx.y], call.partial[blockIdx.y], call.out[blockIdx.y]);
}

hipError_t launch_topk_batch(const TopkDesc* D, uint32_t count, uint32_t d, uint32_t slots_max,
                             uint32_t max_cand_max, uint32_t k_max, const TopkCall& call, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(sel_init_batch_kernel, dim3(1, count), dim3(256), 0, s, D);
  const dim3 cgrid(grid_for(slots_max, 256, 4096), count);
  if (d <= (uint32_t)kTabLdsRows)
    hipLaunchKernelGGL((compact_batch_kernel<kTabLdsRows, true>), cgrid, dim3(256), 0, s, D);
  else
    hipLaunchKernelGGL((compact_batch_kernel<32, false>), cgrid, dim3(256), 0, s, D);
  hipLaunchKernelGGL(clamp_m_batch_kernel, dim3(1, count), dim3(64), 0, s, D);
  const dim3 hgrid(grid_for(max_cand_max, 256, 1024), count);
  for (int shift = 24; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(sel_hist_batch_kernel<false>, hgrid, dim3(256), 0, s, D, shift);
    hipLaunchKernelGGL(sel_pick_batch_kernel<false>, dim3(1, count), dim3(64), 0, s, D, call, shift);
  }
  for (int shift = 40; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(sel_hist_batch_kernel<true>, hgrid, dim3(256), 0, s, D, shift);
    hipLaunchKernelGGL(sel_pick_batch_kernel<true>, dim3(1, count), dim3(64), 0, s, D, call, shift);
  }
  hipLaunchKernelGGL(sel_gather_batch_kernel, hgrid, dim3(256), 0, s, D, call);
  if (k_max > 0) {
    hipLaunchKernelGGL(rank_clear_batch_kernel, dim3(grid_for(k_max, 256, 1024), count), dim3(256), 0, s, D, call);
    uint64_t chunk = kRankChunk;
    while ((k_max + chunk - 1) / chunk > kMaxGridY) chunk *= 2;
    hipLaunchKernelGGL(rank_count_batch_kernel, dim3((k_max + 255) / 256, (uint32_t)((k_max + chunk - 1) / chunk), count),
                       dim3(256), 0, s, D, call, (uint32_t)chunk);
    hipLaunchKernelGGL(rank_place_batch_kernel, dim3(grid_for(k_max, 256, 1024), count), dim3(256), 0, s, D, call);
  }
  hipLaunchKernelGGL(sel_finish_out_batch_kernel, dim3(1, count), dim3(64), 0, s, D, call);
  return hipGetLastError();
}

hipError_t launch_topk(const uint64_t* set, uint32_t slots, const Tables& t, const int32_t* M,
                       uint32_t max_cand, uint32_t k, SelState* st, uint64_t* ck, int32_t* ce,
                       uint64_t* sk, int32_t* se, uint64_t* ok, int32_t* oe, const uint32_t* err,
                       hipStream_t s, const uint64_t* ov_keys, const uint32_t* ov_counts, uint32_t ov_mask) {
  hipLaunchKernelGGL(sel_init_kernel, dim3(1), dim3(256), 0, s, st);
  const dim3 cgrid(grid_for(slots, 256, 4096));
  if (t.d <= (uint32_t)kTabLdsRows)
    hipLaunchKernelGGL((compact_kernel<kTabLdsRows, true>), cgrid, dim3(256), 0, s, set, slots, t, M, max_cand, st,
                       ck, ce, ov_keys, ov_counts, ov_mask);
  else
    hipLaunchKernelGGL((compact_kernel<32, false>), cgrid, dim3(256), 0, s, set, slots, t, M, max_cand, st, ck,
                       ce, ov_keys, ov_counts, ov_mask);
  hipLaunchKernelGGL(clamp_m_kernel, dim3(1), dim3(64), 0, s, st, max_cand);
  // the candidate estimates are no longer needed once gathered: their first k words hold the ranks
  return select_stages(ck, ce, max_cand, k, st, sk, se, (uint32_t*)ce, ok, oe, err, s);
}

hipError_t launch_select_pairs(const uint64_t* ck, const int32_t* ce, uint32_t m, uint32_t k, SelState* st,
                               uint64_t* sk, int32_t* se, uint32_t* rank, uint64_t* ok, int32_t* oe,
                               const uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(sel_init_kernel, dim3(1), dim3(256), 0, s, st);
  hipLaunchKernelGGL(sel_set_m_kernel, dim3(1), dim3(64), 0, s, st, m);
  return select_stages(ck, ce, m, k, st, sk, se, rank, ok, oe, err, s);
}

}  // namespace csk
