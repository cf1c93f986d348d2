// csk_internal.h — kernel launch interface between the C ABI (csk_api.hip) and the
// kernels (csk_kernels.hip).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csk_device.h"

namespace csk {

// Candidate selection state (one per handle, device memory).
struct SelState {
  uint32_t m;           // candidates compacted from the set
  uint32_t k_rem;       // items still to take inside the current class
  uint32_t est_prefix;  // chosen high bits of (est ^ 0x80000000)
  uint32_t est_mask;
  uint64_t key_prefix;  // chosen high bits of the key among est == T
  uint64_t key_mask;
  uint32_t n_sel;       // items gathered
  uint32_t err;         // snapshot of the error latch, read back by the host
  uint32_t hist[256];
};

struct Tables {
  const uint32_t* tab;  // [d][6][256] uint32, device
  const uint32_t* tabi; // row-interleaved [6][256][dp] uint32 (d <= 8), device
  const uint32_t* tabp; // packed top-F-bit fields [6][256][4] uint32 (d = 5..8), device, or NULL
  const uint32_t* tabs; // the packed fields permuted into sort words (see csk_sortbin.hip), or NULL
  const uint32_t* tabq; // probe tables of the field-probe filter (d <= 5, w = 2^lw <= 2^24), or NULL
  const uint32_t* fcols; // the columns and salts of its row maps (d x kFieldCols), or NULL
  uint32_t lw;          // log2(w) when w is a power of two, else 0
  uint32_t fp;          // the field-probe filter's prefix bits P (w <= 2^P < 2w), 0 without tabq
  uint32_t fspan;       // at most this many P-bit prefixes per bucket (1 when w = 2^P)
  uint32_t dp;          // 4 (d <= 4), 6 (d <= 6) or 8 (d <= 8); 0 when d > 8
  uint32_t d;
  uint32_t w;
  uint32_t wshift;      // 32 - log2(w) when w is a power of two >= 2, else 0
  uint32_t bnorm;       // 32 - bits(w - 1): shifts a bucket to the top of a word
  uint32_t cm;          // 1: Count-Min (no sign, minimum), 0: Count Sketch
  // kHashPacked when the packed tables serve this w, else kHashShift (w = 2^lw) or kHashMulHi
  int hash_mode() const {
    if (tabp != nullptr && wshift != 0 && d >= 5 && d <= 8 && (32u - wshift) + 1u <= (uint32_t)packed_bits((int)d))
      return kHashPacked;
    return wshift ? kHashShift : kHashMulHi;
  }
};

// Binned update: sizes chosen by the host.
struct BinPlan {
  uint32_t Pr;          // slices per row: ceil(w / 2^15)
  uint32_t P;           // d * Pr
  uint32_t nwg;         // workgroups of the bin kernel
  uint64_t ntiles;      // ceil(n / tile)
  uint32_t cap;         // tokens per (slice, workgroup) region, multiple of 8
  uint32_t tile;        // particles per tile
  uint32_t tab_rows_lds;
  uint32_t lds_bytes;
  uint32_t fast;        // 1: row-interleaved kernel (d <= 8)
  uint32_t sort;        // the sort-word bin kernel: kSortPacked or kSortRows, 0: not
  uint32_t rp;          // its rows per LDS pass (2 or 3)
  uint32_t pf;          // 1: it loads the next tile's positions while sorting the current one
  uint32_t nt;          // its threads per workgroup (512 or 1024)
};

constexpr int kBin2Threads = 1024;                 // row-interleaved bin kernel
// particles per thread per tile: all d tokens of each stay in registers
constexpr int bin2_ppt(int d) { return d == 1 ? 16 : (d == 2 ? 12 : (d <= 5 ? 8 : 4)); }
constexpr int kBin2Rows = 2;                       // rows sorted per LDS pass
constexpr int kCollectThreads = 1024;
constexpr int kCollectCache = 1024;               // per-workgroup cache of inserted keys
constexpr int kCollectPPT = 8;                    // particles per thread per round (loads in flight)
constexpr int kBinThreads = 512;
constexpr int kBinPPT = 16;                       // particles per thread per tile
constexpr int kBinTile = kBinThreads * kBinPPT;   // 8192
constexpr int kAccThreads = 1024;
constexpr uint32_t kMaxSlicesPerRow = 4096;
constexpr uint32_t kMaxLds = 160 * 1024;

// Returns false if the binned path does not fit (then use the direct path).
bool plan_bin(uint64_t n, uint32_t d, uint32_t w, BinPlan& plan);
// The same with at most max_wg workgroups (>= 1) for the bin kernel.
bool plan_bin_wg(uint64_t n, uint32_t d, uint32_t w, uint64_t max_wg, BinPlan& plan);
uint32_t bin_wg_cap(uint32_t d, uint32_t requested);
// Bin kernel forms (csk_set_update_tiling): automatic, the general row-interleaved
// kernel, or the sort-word kernel.
constexpr uint32_t kFormAuto = 0;
constexpr uint32_t kFormGeneral = 1;
constexpr uint32_t kFormSortWord = 2;
// Sort-word bin kernel forms: on the packed sort-word table (w = 2^lw within the packed
// fields), or on the row-interleaved tables with multiply-high buckets (any w <= 2^24).
constexpr uint32_t kSortPacked = 1;
constexpr uint32_t kSortRows = 2;
// Turn a fast bin plan into a sort-word plan when the form asks for it (or leaves it
// to us) and the sketch, the mesh (ungrouped, not packed) and LDS allow: want_nt 0 (auto),
// 512 or 1024 threads; want_rp 0 (auto), 2 or 3 rows per pass; want_pf 0 (auto), 1 (off)
// or 2 (on; 512 threads only).  The packed table is used when the sketch has it; else,
// with rows_ok, the row tables (1024 threads, no prefetch).  Returns true if the plan now
// uses the sort-word kernel.
bool plan_sortbin(BinPlan& p, uint32_t d, const Mesh& mesh, const Tables& t, uint32_t form, uint32_t want_nt,
                  uint32_t want_rp, uint32_t want_pf, bool rows_ok);

// The learned router's exclusion (csk_sketch_update_routed): a particle whose coarse parent
// (its fine index divided by `factor` on each axis, on the mesh of G / factor cells a side)
// is one of the admitted coarse cells is counted exactly, in child[position of the parent
// in the admitted list * factor^3 + position of the fine cell inside it], and is not added
// to the sketch.  admitted == NULL: no exclusion.
struct RouteExclude {
  const uint64_t* admitted;   // admitted coarse keys (device)
  const uint32_t* na;         // how many (device); at most na_max are used
  uint32_t na_max;            // min(kMaxAdmitted, floor(2^15 / factor^3))
  uint32_t factor;
  uint32_t fmagic;            // ceil(2^32 / factor): i / factor = umulhi(i, fmagic) for i < 2^16
  uint32_t f3;                // factor^3
  uint32_t gc;                // G / factor
  uint32_t* child;            // na_max * f3 counters (device)
  uint32_t* err;              // bit 2: *na was above na_max (device)
};
// The routing split's LDS hash of the admitted keys: 1024 slots (load <= 1/2).
constexpr uint32_t kAdmHashSlots = 1024;
// The exclusion's LDS table inside the update kernels: 2048 64-bit key slots (load <= 1/4),
// their 16-bit positions, and a 2^16-bit prefilter that most particles stop at.
constexpr uint32_t kExSlots = 2048;
constexpr uint32_t kExBitWords = 2048;
constexpr uint32_t kExLdsWords = kExSlots * 2 + kExSlots / 2 + kExBitWords;

// Everything the bin kernel needs for one sketch and one stream.
struct BinArgs {
  const float* __restrict__ pos;
  uint64_t n;
  Mesh mesh;
  const uint32_t* __restrict__ tab;
  const uint32_t* __restrict__ tabi;
  const uint32_t* __restrict__ tabp;
  const uint32_t* __restrict__ tabs;
  uint32_t d, w, wshift, cm;
  BinPlan plan;
  uint16_t* __restrict__ tok;
  uint32_t* __restrict__ cnt;
  int32_t* __restrict__ M;
  uint32_t* __restrict__ err;
  RouteExclude ex;
};

// Everything the accumulate kernel needs for one sketch.
struct AccArgs {
  const uint16_t* __restrict__ tok;
  const uint32_t* __restrict__ cnt;
  BinPlan plan;
  uint32_t w;
  int32_t* __restrict__ M;
};

// Per-call streams of a batched update: sketch i reads n[i] particles at pos[i].
constexpr uint32_t kMaxBatch = 64;
struct BatchCall {
  const float* pos[kMaxBatch];
  uint64_t n[kMaxBatch];
};

// LDS of the sort-word bin kernel: rows false for the packed sort-word table, true for the
// row-interleaved tables over the mesh's nch key bytes; ex: with the router's exclusion table.
uint32_t sortbin_lds_bytes(uint32_t d, uint32_t rp, uint32_t Pr, uint32_t P, bool rows, uint32_t nch, bool ex);
hipError_t launch_sortbin(const BinArgs& a, uint32_t mesh_mode, hipStream_t s);
// The row-table form (plan.sort == kSortRows), and its d = 5 form with the exclusion in a.ex
// (two rows per pass; plan.lds_bytes from sortbin_lds_bytes(5, 2, ..., true, nch, true)).
hipError_t launch_sortbin_rows(const BinArgs& a, uint32_t mesh_mode, hipStream_t s);
hipError_t launch_sortbin_routed(const BinArgs& a, uint32_t mesh_mode, hipStream_t s);
hipError_t launch_sortbin_batch(const BinArgs* descs, const uint16_t* wg_sketch, const uint32_t* wg_first,
                                uint32_t nwg_total, uint32_t lds_bytes, uint32_t d, uint32_t mode, const BinPlan& form,
                                uint32_t kb, const BatchCall& call, hipStream_t s);
BinArgs make_bin_args(const float* pos, uint64_t n, const Mesh& mesh, const Tables& t, const BinPlan& plan,
                      uint16_t* tok, uint32_t* cnt, int32_t* M, uint32_t* err);
// One bin launch for many sketches of the same d, mesh mode and hash mode (fast path,
// d <= 8): workgroup g serves sketch wg_sketch[g] as its workgroup g - wg_first[sketch].
hipError_t launch_bin_batch(const BinArgs* descs, const uint16_t* wg_sketch, const uint32_t* wg_first,
                            uint32_t nwg_total, uint32_t lds_bytes, uint32_t d, uint32_t mode, int hm,
                            const BatchCall& call, hipStream_t s);
// One accumulate launch for many sketches: block b sums slice b - acc_first[sketch] of
// sketch acc_sketch[b].
hipError_t launch_accumulate_batch(const AccArgs* descs, const uint16_t* acc_sketch, const uint32_t* acc_first,
                                   uint32_t nblocks, hipStream_t s);

hipError_t launch_bin(const float* pos, uint64_t n, const Mesh& mesh, const Tables& t, const BinPlan& plan,
                      uint16_t* tok, uint32_t* cnt, int32_t* M, uint32_t* err, hipStream_t s);
hipError_t launch_accumulate(const uint16_t* tok, const uint32_t* cnt, const BinPlan& plan, uint32_t w,
                             int32_t* M, hipStream_t s);
hipError_t launch_update_direct(const float* pos, uint64_t n, const Mesh& mesh, const Tables& t, int32_t* M,
                                uint32_t* err, hipStream_t s);
// The update with the learned router's exclusion: the general bin kernel (d = 5, a fast
// general plan with plan.rp 2 or 3 rows per pass and lds_bytes = bin3_lds_bytes(.., true))
// or the direct update (any d); both need float positions on an ungrouped mesh.
hipError_t launch_bin_routed(const float* pos, uint64_t n, const Mesh& mesh, const Tables& t, const BinPlan& plan,
                             uint16_t* tok, uint32_t* cnt, int32_t* M, uint32_t* err, const RouteExclude& ex,
                             hipStream_t s);
// LDS bytes of the general bin kernel for a plan with rp rows per pass (with the exclusion's
// hash when ex).
uint32_t bin3_lds_bytes(const BinPlan& p, uint32_t d, uint32_t rp, bool ex);
hipError_t launch_update_direct_routed(const float* pos, uint64_t n, const Mesh& mesh, const Tables& t, int32_t* M,
                                       uint32_t* err, const RouteExclude& ex, hipStream_t s);
hipError_t launch_keys(const float* pos, uint64_t n, const Mesh& mesh, uint64_t* keys, hipStream_t s);
hipError_t launch_pack(const float* pos, uint64_t n, const Mesh& pm, uint64_t* out, uint32_t* err, hipStream_t s);
hipError_t launch_query(const uint64_t* keys, uint64_t m, const Tables& t, const int32_t* M, int32_t* est,
                        hipStream_t s);
// Bloom filter of the (row, bucket, sign) items whose signed counter is >= theta
// (theta > 0); filter: kFilterWords words, hot: item count (both zeroed here).
// hot_table (kHotSlots words, may be NULL) receives every item when the count is at most
// kHotMaxItems, and stays empty otherwise.
hipError_t launch_filter_build(const Tables& t, const int32_t* M, int32_t theta, uint32_t* filter, uint32_t* hot,
                               uint32_t* hot_table, bool field, hipStream_t s);
// A sketch's candidate-pass arguments (kernel argument, or one entry of a batch's
// descriptor array).
struct CollectDesc {
  Mesh mesh;
  Tables t;
  const int32_t* M;
  uint32_t* filter;           // Bloom filter (device) or NULL
  uint32_t* hot;              // its hot-item count
  uint32_t* hot_table;        // exact hot-item set or NULL
  uint64_t* set;
  uint32_t slot_mask;
  uint32_t* set_count;
  uint32_t max_cand;
  uint32_t* err;
};
// Per-call arguments of a batched candidate pass (kernel argument).
struct CollectCall {
  const float* pos[kMaxBatch];
  uint64_t n[kMaxBatch];
  int32_t theta[kMaxBatch];
  uint32_t use_filter[kMaxBatch];   // theta > 0 and the sketch has a filter
};
size_t collect2_lds_bytes(const Tables& t, bool use_filter, bool field);
// The field-probe filter serves this sketch (d = 5, packed hash, probe tables).
bool collect_field_form(const Tables& t);
// Batched candidate pass: the clears, the filter and hot-set builds of every sketch whose
// theta is > 0, then one collect launch of nwg_total workgroups (workgroup g serves sketch
// wg_sketch[g] as its workgroup g - wg_first[sketch] of wg_count[sketch]).  All sketches
// share d, the mesh mode and the hash mode; field: every one uses the field-probe filter.
hipError_t launch_collect_batch(const CollectDesc* descs, const CollectDesc* host_descs, uint32_t count,
                                const uint16_t* wg_sketch, const uint32_t* wg_first, const uint32_t* wg_count,
                                uint32_t nwg_total, uint32_t d, uint32_t mesh_mode, int hm, bool field,
                                uint32_t w_max, const CollectCall& call, hipStream_t s);

// field: the filter is a field-probe filter (built with field = true; used only when the
// sketch has probe tables, d = 5 and the packed hash).
hipError_t launch_collect(const float* pos, uint64_t n, const Mesh& mesh, const Tables& t, const int32_t* M,
                          int32_t theta, const uint32_t* filter, const uint32_t* hot, const uint32_t* hot_table,
                          uint64_t* set, uint32_t slot_mask, uint32_t* set_count, uint32_t max_cand, uint32_t* err,
                          bool field, hipStream_t s);
// Candidate pass over every key in [0, nkeys) (the whole G^3 dictionary); arguments as
// launch_collect without the positions.
hipError_t launch_collect_dictionary(uint64_t nkeys, const Mesh& mesh, const Tables& t, const int32_t* M,
                                     int32_t theta, const uint32_t* filter, const uint32_t* hot,
                                     const uint32_t* hot_table, uint64_t* set, uint32_t slot_mask,
                                     uint32_t* set_count, uint32_t max_cand, uint32_t* err, hipStream_t s);
// Hierarchical query, second layer: list the coarse set's super-items (list_count is
// zeroed here; more than list_cap latches the capacity error in err), then insert every
// child key of theirs whose fine estimate is >= theta into the fine set.
hipError_t launch_collect_children(const uint64_t* coarse_set, uint32_t coarse_slots, uint64_t* list,
                                   uint32_t* list_count, uint32_t list_cap, uint32_t group, uint64_t ncells,
                                   const Tables& t, const int32_t* M, int32_t theta, uint64_t* set,
                                   uint32_t slot_mask, uint32_t* set_count, uint32_t max_cand, uint32_t* err,
                                   hipStream_t s);
// out[0] = min(k, candidates), out[1] = 1 if that is below k and `partial`, else 0.
hipError_t launch_topk_out(const SelState* st, uint32_t k, uint32_t partial, uint32_t* out, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
// Up to kFillSpans spans of 32-bit words, span r set to v[r], in one launch (the clears of a
// handle's state).  A span with n[r] = 0 is skipped and its pointer is not used.
constexpr int kFillSpans = 4;
struct FillSpans {
  uint32_t* p[kFillSpans];
  uint64_t n[kFillSpans];
  uint32_t v[kFillSpans];
};
hipError_t launch_fill_spans(const FillSpans& f, hipStream_t s);
// The clears of up to kMaxBatch handles in one launch: spans (device) holds, for sketch y,
// kFillSpans spans of 32-bit words, span r set to v[y][r]; blockIdx.y = sketch.
struct ResetSpans {
  uint32_t* p[kMaxBatch][kFillSpans];
  uint64_t n[kMaxBatch][kFillSpans];
  uint32_t v[kMaxBatch][kFillSpans];
};
hipError_t launch_fill_spans_batch(const ResetSpans* spans, uint32_t count, uint64_t max_words, hipStream_t s);
// ov_keys / ov_counts / ov_mask: an exact table whose counts replace the estimates of the
// candidates found in it (NULL: none).
hipError_t launch_topk(const uint64_t* set, uint32_t slots, const Tables& t, const int32_t* M,
                       uint32_t max_cand, uint32_t k, SelState* st, uint64_t* cand_key, int32_t* cand_est,
                       uint64_t* sel_key, int32_t* sel_est, uint64_t* out_key, int32_t* out_est,
                       const uint32_t* err, hipStream_t s, const uint64_t* ov_keys = nullptr,
                       const uint32_t* ov_counts = nullptr, uint32_t ov_mask = 0);
// Top k of the m pairs (ck[i], ce[i]) in (ce desc, ck asc) order, keys distinct and below
// 2^48 (equal keys only where they cannot reach the top k): winners in ok / oe, ranks in
// `rank` (k words), sk / se (k) scratch.
// One sketch of a batched top-k (device array, built once per batch).
struct TopkDesc {
  const uint64_t* set;
  uint32_t slots;
  uint32_t max_cand;
  Tables t;
  const int32_t* M;
  SelState* st;
  uint64_t* ck;
  int32_t* ce;
  uint64_t* sk;
  int32_t* se;
  const uint32_t* err;
};
// Per-call arguments of a batched top-k (kernel arguments): k, outputs and the partial-set
// flag of each sketch.
struct TopkCall {
  uint64_t* keys[kMaxBatch];
  int32_t* est[kMaxBatch];
  uint32_t* out[kMaxBatch];
  uint32_t k[kMaxBatch];
  uint32_t partial[kMaxBatch];
  uint32_t key32[kMaxBatch];   // 1: the sketch's keys are below 2^32 (G^3 <= 2^32)
};
hipError_t launch_topk_batch(const TopkDesc* D, uint32_t count, uint32_t d, uint32_t slots_max,
                             uint32_t max_cand_max, uint32_t k_max, const TopkCall& call, hipStream_t s);

hipError_t launch_select_pairs(const uint64_t* ck, const int32_t* ce, uint32_t m, uint32_t k, SelState* st,
                               uint64_t* sk, int32_t* se, uint32_t* rank, uint64_t* ok, int32_t* oe,
                               const uint32_t* err, hipStream_t s);
// The same over the first min(*m_dev, cap) pairs of a device count.
hipError_t launch_select_pairs_dev(const uint64_t* ck, const int32_t* ce, const uint64_t* m_dev, uint32_t cap,
                                   uint32_t k, SelState* st, uint64_t* sk, int32_t* se, uint32_t* rank, uint64_t* ok,
                                   int32_t* oe, const uint32_t* err, hipStream_t s);
// Insert every non-empty key of an exact table (tslots slots) into a candidate set.
hipError_t launch_table_to_set(const uint64_t* tk, uint32_t tslots, uint64_t* set, uint32_t slot_mask,
                               uint32_t* set_count, uint32_t max_cand, uint32_t* err, hipStream_t s);

}  // namespace csk
