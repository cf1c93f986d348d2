// csk_kernels.hip — gfx950 kernels of the streaming Count-Sketch hot path after the
// update (which lives in csk_update.hip):
// query   (Sec. 2.2 Estimate; Alg. 4 Estimate): lower median of the d signed counters.
// dictionary and hierarchy (Sec. 2.2 items 1 and 3): candidates without positions.
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

// ------------------------------------------------------------------ dictionary and hierarchy

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
__global__ void fill_spans_batch_kernel(const ResetSpans* __restrict__ sp) {
  const uint32_t y = blockIdx.y;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (int r = 0; r < kFillSpans; ++r) {
    uint32_t* __restrict__ p = sp->p[y][r];
    const uint64_t n = sp->n[y][r];
    const uint32_t v = sp->v[y][r];
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) p[j] = v;
  }
}
hipError_t launch_fill_spans_batch(const ResetSpans* spans, uint32_t count, uint64_t max_words, hipStream_t s) {
  if (count == 0 || max_words == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_spans_batch_kernel, dim3(grid_for(max_words, 256, 1024), count), dim3(256), 0, s, spans);
  return hipGetLastError();
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

// Distinct keys of the set -> (key, estimate from the current counters).  Each block stages
// the d hash tables (up to 30 KiB) in LDS and then walks kCompactSlots slots per thread, so
// that the staging is paid once per 4096 slots rather than per 256 (with 2048 blocks per
// sketch of 2^19 slots, a batch of 64 read 3.9 GB of tables from L2 for its compaction).
constexpr uint32_t kCompactSlots = 16;
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
  if (blockIdx.x * blockDim.x >= slots) return;   // no slot here (uniform): skip the table staging
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
// (est, key) as one 64-bit word for keys below 2^32: j comes before i in the output order
// (higher estimate, then lower key) exactly when its word is the larger.
__device__ __forceinline__ uint64_t rank_word(int32_t e, uint64_t k) {
  return ((uint64_t)((uint32_t)e ^ 0x80000000u) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)k);
}

__device__ __forceinline__ void rank_count_body(const uint64_t* __restrict__ sk, const int32_t* __restrict__ se,
                                                const SelState* st, uint32_t k, uint32_t chunk,
                                                uint32_t* __restrict__ rank, uint32_t cy = blockIdx.y,
                                                bool key32 = false) {
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
  if (key32) {   // one 64-bit comparison per pair
    const uint64_t wi = rank_word(ei, ki);
    for (uint32_t j0 = j_lo; j0 < j_hi; j0 += 256) {
      __syncthreads();
      if (j0 + threadIdx.x < j_hi) tk[threadIdx.x] = rank_word(se[j0 + threadIdx.x], sk[j0 + threadIdx.x]);
      __syncthreads();
      const uint32_t lim = min(256u, j_hi - j0);
      for (uint32_t t = 0; t < lim; ++t) cnt += tk[t] > wi;
    }
  } else {
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

__global__ void sel_set_m_dev_kernel(SelState* st, const uint64_t* m_dev, uint32_t cap) {
  if (threadIdx.x == 0) st->m = (uint32_t)(*m_dev < cap ? *m_dev : cap);
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
  rank_count_body(d.sk, d.se, d.st, call.k[blockIdx.z], chunk, (uint32_t*)d.ce, blockIdx.y, call.key32[blockIdx.z] != 0u);
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
  const dim3 cgrid(grid_for(slots_max, 256 * kCompactSlots, 4096), count);
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
  const dim3 cgrid(grid_for(slots, 256 * kCompactSlots, 4096));
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

hipError_t launch_select_pairs_dev(const uint64_t* ck, const int32_t* ce, const uint64_t* m_dev, uint32_t cap,
                                   uint32_t k, SelState* st, uint64_t* sk, int32_t* se, uint32_t* rank, uint64_t* ok,
                                   int32_t* oe, const uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(sel_init_kernel, dim3(1), dim3(256), 0, s, st);
  hipLaunchKernelGGL(sel_set_m_dev_kernel, dim3(1), dim3(64), 0, s, st, m_dev, cap);
  return select_stages(ck, ce, cap, k, st, sk, se, rank, ok, oe, err, s);
}

hipError_t launch_select_pairs(const uint64_t* ck, const int32_t* ce, uint32_t m, uint32_t k, SelState* st,
                               uint64_t* sk, int32_t* se, uint32_t* rank, uint64_t* ok, int32_t* oe,
                               const uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(sel_init_kernel, dim3(1), dim3(256), 0, s, st);
  hipLaunchKernelGGL(sel_set_m_kernel, dim3(1), dim3(64), 0, s, st, m);
  return select_stages(ck, ce, m, k, st, sk, se, rank, ok, oe, err, s);
}

}  // namespace csk
