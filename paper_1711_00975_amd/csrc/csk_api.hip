// csk_api.hip — the C ABI declared in include/csk.h: argument checks, device memory of a
// handle, hash-table seeding, and the kernel sequences of each call.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "csk.h"
#include "csk_internal.h"
#include "csk_router.h"

using namespace csk;

namespace {

thread_local char g_last_error[512] = "";

csk_status fail(csk_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return code;
}

csk_status hip_fail(hipError_t e, const char* where) {
  if (e == hipErrorOutOfMemory) return fail(CSK_E_NOMEM, "%s: out of device memory", where);
  return fail(CSK_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define CSK_HIP(expr, where)                       \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

// SplitMix64 (Steele, Lea & Flood 2014): Weyl increment, then the variant-13 mixer.
uint64_t splitmix64(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Tabulation tables T[r][c][v], filled row by row, character by character, value by
// value from one SplitMix64 stream: two 32-bit entries per draw, low half first.
std::vector<uint32_t> make_tables(uint64_t seed, uint32_t d) {
  std::vector<uint32_t> T((size_t)d * kTableWords);
  uint64_t st = seed;
  for (size_t i = 0; i < T.size(); i += 2) {
    const uint64_t z = splitmix64(st);
    T[i] = (uint32_t)z;
    if (i + 1 < T.size()) T[i + 1] = (uint32_t)(z >> 32);
  }
  return T;
}

// The same tables with the rows of each (character, value) entry side by side,
// padded to dp = 4, 6 or 8 words, for kernels that hash every row in one pass.
std::vector<uint32_t> interleave_tables(const std::vector<uint32_t>& T, uint32_t d, uint32_t dp) {
  std::vector<uint32_t> Ti((size_t)kTableWords * dp, 0u);
  for (uint32_t r = 0; r < d; ++r)
    for (uint32_t e = 0; e < (uint32_t)kTableWords; ++e) Ti[(size_t)e * dp + r] = T[(size_t)r * kTableWords + e];
  return Ti;
}

// The top F = floor(128 / d) bits of every row's entry, packed into four words per
// (character, value) entry with row r at bit r * F (d = 5..8).  Hashing is XOR, so the
// packed XOR over a key's characters holds the top F bits of every row's word.
std::vector<uint32_t> pack_tables(const std::vector<uint32_t>& T, uint32_t d) {
  const uint32_t F = (uint32_t)packed_bits((int)d);
  std::vector<uint32_t> P((size_t)kTableWords * 4, 0u);
  for (uint32_t e = 0; e < (uint32_t)kTableWords; ++e) {
    for (uint32_t r = 0; r < d; ++r) {
      const uint32_t f = T[(size_t)r * kTableWords + e] >> (32u - F);
      const uint32_t o = r * F, wi = o / 32u, sh = o % 32u;
      P[(size_t)e * 4 + wi] |= f << sh;
      if (sh + F > 32u) P[(size_t)e * 4 + wi + 1] |= f >> (32u - sh);
    }
  }
  return P;
}

// The packed fields of pack_tables() with each row's bits rearranged into the sort word
// of the update kernel for w = 2^lw: (slice << 16) | (sign << 15) | (offset in the
// 2^15-counter slice).  Bits below the bucket are dropped; Count-Min drops the sign.  A
// fixed rearrangement of every entry's bits commutes with the XOR of the tabulation, so
// the XOR of these entries is the rearranged field of the full row word.
std::vector<uint32_t> sort_tables(const std::vector<uint32_t>& T, uint32_t d, uint32_t lw, bool count_min) {
  const uint32_t F = (uint32_t)packed_bits((int)d);
  std::vector<uint32_t> S((size_t)kTableWords * 4, 0u);
  for (uint32_t e = 0; e < (uint32_t)kTableWords; ++e) {
    for (uint32_t r = 0; r < d; ++r) {
      const uint32_t f = T[(size_t)r * kTableWords + e] >> (32u - F);
      const uint32_t sign = count_min ? 0u : (f >> (F - 1u));
      const uint32_t b = (f >> (F - 1u - lw)) & ((1u << lw) - 1u);
      const uint32_t v = ((b >> kSliceBits) << 16) | (sign << 15) | (b & (kSlice - 1u));
      const uint32_t o = r * F, wi = o / 32u, sh = o % 32u;
      S[(size_t)e * 4 + wi] |= v << sh;
      if (sh + F > 32u) S[(size_t)e * 4 + wi + 1] |= v >> (32u - sh);
    }
  }
  return S;
}

// The row maps of the field-probe filter: kFieldCols words per row (25 random 25-bit
// columns, then a 25-bit salt) from a SplitMix64 stream of its own.
std::vector<uint32_t> probe_columns(uint64_t seed, uint32_t d) {
  std::vector<uint32_t> C((size_t)d * kFieldCols);
  uint64_t st = seed ^ 0x243F6A8885A308D3ull;
  for (auto& c : C) c = (uint32_t)splitmix64(st) & ((1u << kFieldBits) - 1u);
  return C;
}

// Probe tables of the field-probe filter with P prefix bits (w <= 2^P < 2w): entry (c, v)
// holds, for every row r at bit 25 r, L_r applied to x = (sign << P) | (top P bits of the
// bucket input h << 1) of T[r][c][v] -- a bit selection, so the XOR over a key's bytes gives
// L_r of the key's own x -- with the salt added to the entries of byte 0 only, so that
// every key's XOR holds it exactly once.  For w = 2^P the prefix is the bucket itself; for
// any other w the bucket, umulhi(h << 1, w), is fixed by one of at most fspan prefixes,
// all of which the filter build inserts.
std::vector<uint32_t> probe_tables(const std::vector<uint32_t>& T, uint32_t d, uint32_t P, bool count_min,
                                   const std::vector<uint32_t>& C) {
  std::vector<uint32_t> Q((size_t)kTableWords * 4, 0u);
  for (uint32_t e = 0; e < (uint32_t)kTableWords; ++e) {
    for (uint32_t r = 0; r < d; ++r) {
      const uint32_t H = T[(size_t)r * kTableWords + e];
      const uint32_t b = (H << 1) >> (32u - P);
      const uint32_t sign = count_min ? 0u : (H >> 31);
      const uint32_t x = (sign << P) | b;
      const uint32_t* col = &C[(size_t)r * kFieldCols];
      uint32_t f = (e < 256u) ? col[kFieldBits] : 0u;
      for (uint32_t i = 0; i < (uint32_t)kFieldBits; ++i)
        if ((x >> i) & 1u) f ^= col[i];
      const uint32_t o = r * (uint32_t)kFieldBits, wi = o / 32u, sh = o % 32u;
      Q[(size_t)e * 4 + wi] |= f << sh;
      if (sh + kFieldBits > 32u) Q[(size_t)e * 4 + wi + 1] |= f >> (32u - sh);
    }
  }
  return Q;
}

// Scratch of csk_sketch_update_noalloc: the token regions of one bin plan, then their
// counts.  Each device holds its own copy for the life of the process; host code never
// uses the array's name as an address, only the per-device pointer that
// hipGetSymbolAddress returns for it (noalloc_scratch()).
constexpr uint64_t kNoAllocScratchBytes = 64ull << 20;
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];
uint8_t* g_scratch_ptr[kNoAllocMaxDevices] = {};
std::mutex g_scratch_mutex;

// Looks up this device's copy of `scratch` once per device (the device is current).
hipError_t noalloc_scratch_setup(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[device] != nullptr) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = (uint8_t*)ptr;
  return hipSuccess;
}

uint8_t* noalloc_scratch(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  return g_scratch_ptr[device];
}

}  // namespace

struct csk_sketch {
  int device = 0;
  uint32_t d = 0, w = 0;
  uint32_t group = 1;        // items are cell keys / group (hierarchical coarse layer)
  int32_t upd_mode = CSK_UPDATE_AUTO;  // how csk_sketch_update adds (csk_set_update_plan)
  uint32_t upd_max_wg = 0;             // most bin workgroups (0: the default)
  uint32_t upd_form = kFormAuto;       // bin kernel form, threads, rows per pass, prefetch
  uint32_t upd_nt = 0, upd_rp = 0, upd_pf = 0;   // (csk_set_update_tiling; 0: automatic)
  uint64_t seed = 0;
  int32_t variant = CSK_VARIANT_COUNT_SKETCH;
  int32_t* M = nullptr;
  uint32_t* tab = nullptr;
  uint32_t* tabi = nullptr;  // row-interleaved tables (d <= 8)
  uint32_t* tabp = nullptr;  // packed top-bit tables (d = 5..8)
  uint32_t* tabs = nullptr;  // the packed fields as sort words (d = 5..8, w = 2^lw <= 2^24)
  uint32_t* tabq = nullptr;  // probe tables of the field-probe filter (d = 5, w <= 2^24)
  uint32_t fp = 0, fspan = 0; // its prefix bits and prefixes per bucket
  uint32_t* fcols = nullptr; // the columns and salts of its row maps
  uint32_t dp = 0;
  uint32_t* filter = nullptr; // Bloom filter of hot items + [kFilterAllocWords] item count
  uint32_t* hot_table = nullptr; // exact set of hot items (kHotSlots words)
  uint64_t* set = nullptr;
  uint32_t slots = 0;
  uint32_t max_cand = 0;
  uint32_t* ctl = nullptr;   // [0] error latch, [1] set count
  SelState* sel = nullptr;
  uint64_t* cand_key = nullptr;
  int32_t* cand_est = nullptr;
  uint64_t* sel_key = nullptr;
  int32_t* sel_est = nullptr;
  uint32_t sel_cap = 0;
  uint16_t* tok = nullptr;
  uint64_t tok_bytes = 0;
  uint32_t* cnt = nullptr;
  uint64_t cnt_bytes = 0;
  SelState* host_sel = nullptr;   // pinned
  uint32_t* host_ctl = nullptr;   // pinned
  bool mesh_set = false;
  double delta = 0, L = 0;
  Mesh mesh{};
  bool partial_set = false;   // some collect since the last clear used theta > INT32_MIN
  uint64_t bytes = 0;

  uint32_t* err() const { return ctl; }
  uint32_t* set_count() const { return ctl + 1; }
  Tables tables() const {
    Tables t;
    t.tab = tab;
    t.tabi = tabi;
    t.tabp = tabp;
    t.tabs = tabs;
    t.tabq = tabq;
    t.fcols = fcols;
    t.fp = tabq ? fp : 0u;
    t.fspan = tabq ? fspan : 0u;
    t.lw = (w >= 2 && (w & (w - 1)) == 0) ? (uint32_t)__builtin_ctz(w) : 0u;
    t.dp = dp;
    t.d = d;
    t.w = w;
    t.wshift = 0;
    if (w >= 2 && (w & (w - 1)) == 0) t.wshift = 32u - (uint32_t)__builtin_ctz(w);
    t.bnorm = (w >= 2) ? (uint32_t)__builtin_clz(w - 1) : 31u;
    t.cm = (variant == CSK_VARIANT_COUNT_MIN) ? 1u : 0u;
    return t;
  }
};

namespace {

template <typename T>
hipError_t dmalloc(csk_sketch* s, T** p, uint64_t count) {
  const uint64_t b = count * sizeof(T);
  hipError_t e = hipMalloc((void**)p, b ? b : 1);
  if (e == hipSuccess) s->bytes += b;
  return e;
}

void free_all(csk_sketch* s) {
  void* ptrs[] = {s->M, s->tab, s->tabi, s->tabp, s->tabs, s->tabq, s->fcols, s->filter, s->hot_table, s->set, s->ctl, s->sel, s->cand_key, s->cand_est, s->sel_key, s->sel_est,
                  s->tok, s->cnt};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (s->host_sel) (void)hipHostFree(s->host_sel);
  if (s->host_ctl) (void)hipHostFree(s->host_ctl);
}

// The mesh of G cells per side over [0, L) and its floor path.
void classify_mesh(Mesh* out, long long G, double L) {
  out->L = L;
  out->invL = 1.0 / L;
  out->twoL = 2.0 * L;
  out->Gd = (double)G;
  out->G = (int32_t)G;
  out->nch = key_chars((int32_t)(G < 65535 ? G : 65535));
  out->group = 1u;
  out->ginv = 1.0;
  // exact-ratio modes: R = G/L exactly representable with <= 29 significant bits
  out->mode = kMeshGeneral;
  out->R = (double)G / L;
  out->Rf = (float)out->R;
  out->twoLf = (float)(2.0 * L);
  if (std::fma(out->R, L, -(double)G) == 0.0 && std::isfinite(out->R) && out->R > 0.0) {
    int ex;
    const double mant = std::frexp(out->R, &ex);       // R = mant * 2^ex, mant in [0.5, 1)
    const double scaled = std::ldexp(mant, 29);         // integer iff <= 29 significant bits
    if (scaled == std::floor(scaled)) out->mode = kMeshExactRatio;
    if (mant == 0.5 && ex >= 1 && (double)out->twoLf == 2.0 * L) out->mode = kMeshPow2Ratio;
  }
}

csk_status check_mesh(csk_sketch* s, double delta, double L, Mesh* out) {
  if (!(delta > 0.0) || !(L > 0.0) || !std::isfinite(delta) || !std::isfinite(L))
    return fail(CSK_E_INVALID, "mesh: delta and L must be finite and positive (delta=%g, L=%g)", delta, L);
  const double q = L / delta;
  if (!(q >= 0.5) || !(q < 65535.5))
    return fail(CSK_E_INVALID, "mesh: L/delta = %g outside [1, 65535]", q);
  const long long G = std::llround(q);
  if (G < 1 || G > 65535 || std::fabs(q - (double)G) > 1e-6 * (double)G)
    return fail(CSK_E_INVALID, "mesh: L/delta = %.17g is not within 1e-6 of an integer in [1, 65535]", q);
  if (s != nullptr && s->mesh_set && (s->delta != delta || s->L != L))
    return fail(CSK_E_STATE, "mesh (delta=%g, L=%g) differs from the one latched on this handle (%g, %g)", delta,
                L, s->delta, s->L);
  classify_mesh(out, G, L);
  out->group = (s != nullptr) ? s->group : 1u;
  out->ginv = 1.0 / (double)out->group;
  return CSK_OK;
}

void latch_mesh(csk_sketch* s, double delta, double L, const Mesh& m) {
  s->mesh_set = true;
  s->delta = delta;
  s->L = L;
  s->mesh = m;
}

csk_status clear_candidates(csk_sketch* s, hipStream_t st) {
  CSK_HIP(launch_fill_u64(s->set, s->slots, kEmptyKey, st), "clear candidates");
  CSK_HIP(launch_fill_u32(s->set_count(), 1, 0u, st), "clear candidates");
  s->partial_set = false;
  return CSK_OK;
}

// Read the latch (synchronizing) and clear it.
csk_status take_latch(csk_sketch* s, hipStream_t st, uint32_t* bits) {
  CSK_HIP(hipMemcpyAsync(s->host_ctl, s->ctl, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st), "read latch");
  CSK_HIP(hipStreamSynchronize(st), "synchronize");
  *bits = s->host_ctl[0];
  if (*bits) CSK_HIP(launch_fill_u32(s->err(), 1, 0u, st), "clear latch");
  return CSK_OK;
}

csk_status latch_status(uint32_t bits) {
  if (bits & kErrCapacity)
    return fail(CSK_E_CAPACITY, "candidate set overflowed its capacity: raise theta or max_candidates");
  if (bits & kErrDomain)
    return fail(CSK_E_DOMAIN, "some particle had a non-finite coordinate or |p| >= 2L and was skipped");
  return CSK_OK;
}

}  // namespace

extern "C" {

csk_status csk_sketch_init_ex(csk_sketch** out, uint32_t d, uint32_t w, uint64_t seed, int32_t variant,
                              uint64_t max_candidates) {
  return csk_sketch_init_group(out, d, w, seed, variant, max_candidates, 1);
}

csk_status csk_sketch_init_group(csk_sketch** out, uint32_t d, uint32_t w, uint64_t seed, int32_t variant,
                                 uint64_t max_candidates, uint32_t group) {
  if (out == nullptr) return fail(CSK_E_INVALID, "init: out is NULL");
  *out = nullptr;
  if (group < 1 || group > (1u << 30)) return fail(CSK_E_INVALID, "init: group=%u outside [1, 2^30]", group);
  if (d < 1 || d > CSK_MAX_ROWS) return fail(CSK_E_INVALID, "init: d=%u outside [1, %u]", d, CSK_MAX_ROWS);
  if (w < 1 || w > CSK_MAX_WIDTH) return fail(CSK_E_INVALID, "init: w=%u outside [1, 2^30]", w);
  if (variant != CSK_VARIANT_COUNT_SKETCH && variant != CSK_VARIANT_COUNT_MIN)
    return fail(CSK_E_INVALID, "init: unknown variant %d", variant);
  if (max_candidates == 0) max_candidates = CSK_DEFAULT_CANDIDATES;
  if (max_candidates > (1ull << 30)) return fail(CSK_E_INVALID, "init: max_candidates above 2^30");
  csk_sketch* s = new (std::nothrow) csk_sketch();
  if (!s) return fail(CSK_E_NOMEM, "init: host allocation failed");
  s->d = d;
  s->w = w;
  s->group = group;
  s->seed = seed;
  s->variant = variant;
  s->max_cand = (uint32_t)max_candidates;
  uint64_t slots = 1024;
  while (slots < 2 * max_candidates) slots <<= 1;
  s->slots = (uint32_t)slots;
  hipError_t e = hipGetDevice(&s->device);
  if (e == hipSuccess) e = noalloc_scratch_setup(s->device);
  const auto T = make_tables(seed, d);
  s->dp = (d <= 4) ? 4u : (d <= 6 ? 6u : (d <= (uint32_t)kTabLdsRows ? 8u : 0u));
  std::vector<uint32_t> Ti;
  if (s->dp) Ti = interleave_tables(T, d, s->dp);
  std::vector<uint32_t> Tp;
  if (d >= 5 && d <= (uint32_t)kTabLdsRows) Tp = pack_tables(T, d);
  std::vector<uint32_t> Ts;
  if (!Tp.empty() && w >= 2 && (w & (w - 1)) == 0) {
    const uint32_t lw = (uint32_t)__builtin_ctz(w);
    if (lw <= 24 && lw + 1 <= (uint32_t)packed_bits((int)d))
      Ts = sort_tables(T, d, lw, variant == CSK_VARIANT_COUNT_MIN);
  }
  std::vector<uint32_t> Fc, Tq;
  if (d == 5 && !Tp.empty() && w >= 2 && w <= (1u << 24)) {   // the field-probe filter: P + 1 <= 25 bits
    uint32_t P = 1;
    while ((1u << P) < w) ++P;
    s->fp = P;
    s->fspan = ((1u << P) == w) ? 1u : (uint32_t)(((1ull << P) + w - 1) / w) + 1u;
    Fc = probe_columns(seed, d);
    Tq = probe_tables(T, d, P, variant == CSK_VARIANT_COUNT_MIN, Fc);
  }
  if (e == hipSuccess) e = dmalloc(s, &s->M, (uint64_t)d * w);
  if (e == hipSuccess) e = dmalloc(s, &s->tab, T.size());
  if (e == hipSuccess && s->dp) e = dmalloc(s, &s->tabi, Ti.size());
  if (e == hipSuccess && !Tp.empty()) e = dmalloc(s, &s->tabp, Tp.size());
  if (e == hipSuccess && !Ts.empty()) e = dmalloc(s, &s->tabs, Ts.size());
  if (e == hipSuccess && !Tq.empty()) e = dmalloc(s, &s->tabq, Tq.size());
  if (e == hipSuccess && !Fc.empty()) e = dmalloc(s, &s->fcols, Fc.size());
  if (e == hipSuccess && s->dp) e = dmalloc(s, &s->filter, (uint64_t)kFilterAllocWords + 1);
  // items pack the bucket in 28 bits, so the exact hot set needs w < 2^28
  if (e == hipSuccess && s->dp && w < (1u << 28)) e = dmalloc(s, &s->hot_table, (uint64_t)kHotSlots);
  if (e == hipSuccess) e = dmalloc(s, &s->set, slots);
  if (e == hipSuccess) e = dmalloc(s, &s->ctl, 4);
  if (e == hipSuccess) e = dmalloc(s, &s->sel, 1);
  if (e == hipSuccess) e = dmalloc(s, &s->cand_key, max_candidates);
  if (e == hipSuccess) e = dmalloc(s, &s->cand_est, max_candidates);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->host_sel, sizeof(SelState), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->host_ctl, 4 * sizeof(uint32_t), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemcpy(s->tab, T.data(), T.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && s->dp)
    e = hipMemcpy(s->tabi, Ti.data(), Ti.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && !Tp.empty())
    e = hipMemcpy(s->tabp, Tp.data(), Tp.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && !Ts.empty())
    e = hipMemcpy(s->tabs, Ts.data(), Ts.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && !Tq.empty())
    e = hipMemcpy(s->tabq, Tq.data(), Tq.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && !Fc.empty())
    e = hipMemcpy(s->fcols, Fc.data(), Fc.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_fill_u32((uint32_t*)s->M, (uint64_t)d * w, 0u, nullptr);
  if (e == hipSuccess) e = launch_fill_u32(s->ctl, 4, 0u, nullptr);
  if (e == hipSuccess) e = launch_fill_u64(s->set, slots, kEmptyKey, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_all(s);
    delete s;
    return hip_fail(e, "init");
  }
  *out = s;
  return CSK_OK;
}

csk_status csk_sketch_init(csk_sketch** out, uint32_t d, uint32_t w, uint64_t seed) {
  return csk_sketch_init_ex(out, d, w, seed, CSK_VARIANT_COUNT_SKETCH, 0);
}

csk_status csk_sketch_destroy(csk_sketch* s) {
  if (s == nullptr) return CSK_OK;
  (void)hipDeviceSynchronize();
  free_all(s);
  delete s;
  return CSK_OK;
}

csk_status csk_set_update_plan(csk_sketch* s, int32_t mode, uint32_t max_wg) {
  if (s == nullptr) return fail(CSK_E_INVALID, "set_update_plan: NULL handle");
  if (mode != CSK_UPDATE_AUTO && mode != CSK_UPDATE_BINNED && mode != CSK_UPDATE_DIRECT)
    return fail(CSK_E_INVALID, "set_update_plan: unknown mode %d", mode);
  if (max_wg > 65535) return fail(CSK_E_INVALID, "set_update_plan: max_wg=%u above 65535", max_wg);
  s->upd_mode = mode;
  s->upd_max_wg = max_wg;
  return CSK_OK;
}

csk_status csk_set_update_tiling(csk_sketch* s, int32_t form, uint32_t threads, uint32_t rows_per_pass,
                                 int32_t prefetch) {
  if (s == nullptr) return fail(CSK_E_INVALID, "set_update_tiling: NULL handle");
  if (form != CSK_BIN_AUTO && form != CSK_BIN_GENERAL && form != CSK_BIN_SORT_WORD)
    return fail(CSK_E_INVALID, "set_update_tiling: unknown form %d", form);
  if (threads != 0 && threads != 512 && threads != 1024)
    return fail(CSK_E_INVALID, "set_update_tiling: threads=%u not 0, 512 or 1024", threads);
  if (rows_per_pass != 0 && rows_per_pass != 2 && rows_per_pass != 3)
    return fail(CSK_E_INVALID, "set_update_tiling: rows_per_pass=%u not 0, 2 or 3", rows_per_pass);
  if (prefetch < 0 || prefetch > 2) return fail(CSK_E_INVALID, "set_update_tiling: prefetch=%d not 0, 1 or 2", prefetch);
  if (prefetch == 2 && threads == 1024)
    return fail(CSK_E_INVALID, "set_update_tiling: the 1024-thread form has no registers for a prefetched tile");
  s->upd_form = (uint32_t)form;
  s->upd_nt = threads;
  s->upd_rp = rows_per_pass;
  s->upd_pf = (uint32_t)prefetch;
  return CSK_OK;
}

namespace {

// The update of a float (x, y, z) stream, or of a packed stream (src = 64-bit words).
// noalloc: tokens go to the device's static scratch, never to memory allocated here;
// a stream whose bin plan does not fit it is refused before anything runs.
// The handle's token and count scratch grown to what the plan needs (a growth synchronizes
// the stream first: earlier work may still read the old buffers).
hipError_t ensure_update_scratch(csk_sketch* s, const BinPlan& plan, hipStream_t st) {
  const uint64_t tok_need = (uint64_t)plan.P * plan.nwg * plan.cap * sizeof(uint16_t);
  const uint64_t cnt_need = (uint64_t)plan.P * plan.nwg * sizeof(uint32_t);
  if (tok_need <= s->tok_bytes && cnt_need <= s->cnt_bytes) return hipSuccess;
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  if (tok_need > s->tok_bytes) {
    if (s->tok) (void)hipFree(s->tok);
    s->bytes -= s->tok_bytes;
    s->tok = nullptr;
    s->tok_bytes = 0;
    e = dmalloc(s, &s->tok, tok_need / sizeof(uint16_t));
    if (e != hipSuccess) return e;
    s->tok_bytes = tok_need;
  }
  if (cnt_need > s->cnt_bytes) {
    if (s->cnt) (void)hipFree(s->cnt);
    s->bytes -= s->cnt_bytes;
    s->cnt = nullptr;
    s->cnt_bytes = 0;
    e = dmalloc(s, &s->cnt, cnt_need / sizeof(uint32_t));
    if (e != hipSuccess) return e;
    s->cnt_bytes = cnt_need;
  }
  return hipSuccess;
}

csk_status update_impl(csk_sketch* s, const void* src, bool packed, uint64_t n, double delta, double L,
                       void* stream, bool noalloc = false) {
  if (s == nullptr) return fail(CSK_E_INVALID, "update: NULL handle");
  Mesh mesh;
  csk_status rc = check_mesh(s, delta, L, &mesh);
  if (rc != CSK_OK) return rc;
  if (n > 0 && src == nullptr) return fail(CSK_E_INVALID, "update: NULL positions");
  if (n > (1ull << 40)) return fail(CSK_E_INVALID, "update: n above 2^40");
  hipStream_t st = (hipStream_t)stream;
  const Tables t = s->tables();
  if (noalloc) {
    uint8_t* base = noalloc_scratch(s->device);
    if (base == nullptr) return fail(CSK_E_STATE, "update_noalloc: no scratch for device %d", s->device);
    if (n > (1ull << 30)) return fail(CSK_E_CAPACITY, "update_noalloc: n=%llu above 2^30", (unsigned long long)n);
    BinPlan plan;
    bool binned = false;
    uint64_t tok_need = 0, need = 0;
    if (s->upd_mode != CSK_UPDATE_DIRECT) {
      // the usual plan, else fewer workgroups (shorter regions), until the regions fit
      for (uint64_t max_wg = bin_wg_cap(s->d, s->upd_max_wg); max_wg >= 1; max_wg /= 2) {
        if (!plan_bin_wg(n, s->d, s->w, max_wg, plan)) break;
        binned = true;
        tok_need = ((uint64_t)plan.P * plan.nwg * plan.cap * sizeof(uint16_t) + 255) & ~255ull;
        need = tok_need + (uint64_t)plan.P * plan.nwg * sizeof(uint32_t);
        if (need <= kNoAllocScratchBytes || max_wg == 1) break;
      }
    }
    if (binned && need > kNoAllocScratchBytes)
      return fail(CSK_E_CAPACITY,
                  "update_noalloc: %llu particles at d=%u, w=%u need %llu bytes of token scratch; the "
                  "no-allocation update holds %llu: split the stream",
                  (unsigned long long)n, s->d, s->w, (unsigned long long)need,
                  (unsigned long long)kNoAllocScratchBytes);
    latch_mesh(s, delta, L, mesh);
    if (n == 0) return CSK_OK;
    if (packed) mesh.mode = kMeshPacked;
    if (binned) (void)plan_sortbin(plan, s->d, mesh, t, s->upd_form, s->upd_nt, s->upd_rp, s->upd_pf, true);
    if (!binned) {
      CSK_HIP(launch_update_direct((const float*)src, n, mesh, t, s->M, s->err(), st), "update_noalloc (direct)");
      return CSK_OK;
    }
    uint16_t* tok = (uint16_t*)base;
    uint32_t* cnt = (uint32_t*)(base + tok_need);
    CSK_HIP(launch_bin((const float*)src, n, mesh, t, plan, tok, cnt, s->M, s->err(), st), "update_noalloc (bin)");
    CSK_HIP(launch_accumulate(tok, cnt, plan, s->w, s->M, st), "update_noalloc (accumulate)");
    return CSK_OK;
  }
  latch_mesh(s, delta, L, mesh);
  if (n == 0) return CSK_OK;
  if (packed) mesh.mode = kMeshPacked;
  const uint64_t piece_max = 1ull << 30;
  for (uint64_t off = 0; off < n; off += piece_max) {
    const uint64_t m = (n - off < piece_max) ? n - off : piece_max;
    const float* p = packed ? (const float*)((const uint64_t*)src + off) : (const float*)src + 3 * off;
    BinPlan plan;
    const uint64_t max_wg = bin_wg_cap(s->d, s->upd_max_wg);
    if (s->upd_mode == CSK_UPDATE_DIRECT || !plan_bin_wg(m, s->d, s->w, max_wg, plan)) {
      CSK_HIP(launch_update_direct(p, m, mesh, t, s->M, s->err(), st), "update (direct)");
      continue;
    }
    (void)plan_sortbin(plan, s->d, mesh, t, s->upd_form, s->upd_nt, s->upd_rp, s->upd_pf, true);
    CSK_HIP(ensure_update_scratch(s, plan, st), "update: token scratch");
    CSK_HIP(launch_bin(p, m, mesh, t, plan, s->tok, s->cnt, s->M, s->err(), st), "update (bin)");
    CSK_HIP(launch_accumulate(s->tok, s->cnt, plan, s->w, s->M, st), "update (accumulate)");
  }
  return CSK_OK;
}

}  // namespace

csk_status csk_sketch_update(csk_sketch* s, const float* pos, uint64_t n, double delta, double L, void* stream) {
  return update_impl(s, pos, false, n, delta, L, stream);
}

csk_status csk_sketch_update_packed(csk_sketch* s, const uint64_t* packed, uint64_t n, double delta, double L,
                                   void* stream) {
  return update_impl(s, packed, true, n, delta, L, stream);
}

csk_status csk_sketch_update_noalloc(csk_sketch* s, const float* pos, uint64_t n, double delta, double L,
                                     void* stream) {
  return update_impl(s, pos, false, n, delta, L, stream, true);
}

csk_status csk_sketch_query(csk_sketch* s, const uint64_t* keys, uint64_t m, int32_t* est, void* stream) {
  if (s == nullptr) return fail(CSK_E_INVALID, "query: NULL handle");
  if (m > 0 && (keys == nullptr || est == nullptr)) return fail(CSK_E_INVALID, "query: NULL keys or est");
  if (m == 0) return CSK_OK;
  CSK_HIP(launch_query(keys, m, s->tables(), s->M, est, (hipStream_t)stream), "query");
  return CSK_OK;
}

csk_status csk_cell_keys(const float* pos, uint64_t n, double delta, double L, uint64_t* keys, void* stream) {
  Mesh mesh;
  csk_status rc = check_mesh(nullptr, delta, L, &mesh);
  if (rc != CSK_OK) return rc;
  if (n > 0 && (pos == nullptr || keys == nullptr)) return fail(CSK_E_INVALID, "cell_keys: NULL pointer");
  if (n == 0) return CSK_OK;
  CSK_HIP(launch_keys(pos, n, mesh, keys, (hipStream_t)stream), "cell_keys");
  return CSK_OK;
}

csk_status csk_cell_keys_packed(const uint64_t* packed, uint64_t n, double delta, double L, uint64_t* keys,
                                void* stream) {
  Mesh mesh;
  csk_status rc = check_mesh(nullptr, delta, L, &mesh);
  if (rc != CSK_OK) return rc;
  if (n > 0 && (packed == nullptr || keys == nullptr)) return fail(CSK_E_INVALID, "cell_keys_packed: NULL pointer");
  if (n == 0) return CSK_OK;
  mesh.mode = kMeshPacked;
  CSK_HIP(launch_keys((const float*)packed, n, mesh, keys, (hipStream_t)stream), "cell_keys_packed");
  return CSK_OK;
}

csk_status csk_pack_positions(const float* pos, uint64_t n, double L, uint64_t* packed, uint32_t* err, void* stream) {
  if (!(L > 0.0) || !std::isfinite(L)) return fail(CSK_E_INVALID, "pack: L=%g must be finite and positive", L);
  if (n > 0 && (pos == nullptr || packed == nullptr || err == nullptr)) return fail(CSK_E_INVALID, "pack: NULL pointer");
  if (n == 0) return CSK_OK;
  Mesh pm;
  classify_mesh(&pm, 1ll << kPackBits, L);
  CSK_HIP(launch_pack(pos, n, pm, packed, err, (hipStream_t)stream), "pack");
  return CSK_OK;
}

namespace {

csk_status collect_impl(csk_sketch* s, const void* src, bool packed, uint64_t n, double delta, double L,
                        int32_t theta, void* stream) {
  if (s == nullptr) return fail(CSK_E_INVALID, "collect: NULL handle");
  Mesh mesh;
  csk_status rc = check_mesh(s, delta, L, &mesh);
  if (rc != CSK_OK) return rc;
  if (n > 0 && src == nullptr) return fail(CSK_E_INVALID, "collect: NULL positions");
  latch_mesh(s, delta, L, mesh);
  if (theta != INT32_MIN) s->partial_set = true;
  if (n == 0) return CSK_OK;
  if (packed) mesh.mode = kMeshPacked;
  hipStream_t st = (hipStream_t)stream;
  const Tables t = s->tables();
  const uint32_t* filter = nullptr;
  const uint32_t* hot = nullptr;
  if (s->filter != nullptr && theta > 0) {
    CSK_HIP(launch_filter_build(t, s->M, theta, s->filter, s->filter + kFilterAllocWords, s->hot_table, true, st),
            "collect (filter)");
    filter = s->filter;
    hot = s->filter + kFilterAllocWords;
  }
  CSK_HIP(launch_collect((const float*)src, n, mesh, t, s->M, theta, filter, hot, filter ? s->hot_table : nullptr, s->set,
                         s->slots - 1, s->set_count(), s->max_cand, s->err(), true, st),
          "collect");
  return CSK_OK;
}

}  // namespace

csk_status csk_collect(csk_sketch* s, const float* pos, uint64_t n, double delta, double L, int32_t theta,
                       void* stream) {
  return collect_impl(s, pos, false, n, delta, L, theta, stream);
}

csk_status csk_collect_packed(csk_sketch* s, const uint64_t* packed, uint64_t n, double delta, double L, int32_t theta,
                              void* stream) {
  return collect_impl(s, packed, true, n, delta, L, theta, stream);
}

csk_status csk_collect_dictionary(csk_sketch* s, double delta, double L, int32_t theta, void* stream) {
  if (s == nullptr) return fail(CSK_E_INVALID, "collect_dictionary: NULL handle");
  Mesh mesh;
  csk_status rc = check_mesh(s, delta, L, &mesh);
  if (rc != CSK_OK) return rc;
  latch_mesh(s, delta, L, mesh);
  if (theta != INT32_MIN) s->partial_set = true;
  hipStream_t st = (hipStream_t)stream;
  const Tables t = s->tables();
  const uint32_t* filter = nullptr;
  const uint32_t* hot = nullptr;
  if (s->filter != nullptr && theta > 0) {
    CSK_HIP(launch_filter_build(t, s->M, theta, s->filter, s->filter + kFilterAllocWords, s->hot_table, false, st),
            "collect_dictionary (filter)");
    filter = s->filter;
    hot = s->filter + kFilterAllocWords;
  }
  const uint64_t ncells = (uint64_t)mesh.G * mesh.G * mesh.G;
  const uint64_t nkeys = (ncells + s->group - 1) / s->group;   // the items: cell keys / group
  CSK_HIP(launch_collect_dictionary(nkeys, mesh, t, s->M, theta, filter, hot, filter ? s->hot_table : nullptr, s->set,
                                    s->slots - 1, s->set_count(), s->max_cand, s->err(), st),
          "collect_dictionary");
  return CSK_OK;
}

csk_status csk_collect_children(csk_sketch* fine, csk_sketch* coarse, int32_t theta, void* stream) {
  if (fine == nullptr || coarse == nullptr) return fail(CSK_E_INVALID, "collect_children: NULL handle");
  if (fine == coarse) return fail(CSK_E_INVALID, "collect_children: fine and coarse are the same handle");
  if (fine->group != 1) return fail(CSK_E_INVALID, "collect_children: the fine handle has group %u", fine->group);
  if (!fine->mesh_set || !coarse->mesh_set)
    return fail(CSK_E_STATE, "collect_children: both handles need a latched mesh (update or collect first)");
  if (fine->delta != coarse->delta || fine->L != coarse->L)
    return fail(CSK_E_STATE, "collect_children: the handles latched different meshes");
  if (fine->device != coarse->device) return fail(CSK_E_INVALID, "collect_children: handles on different devices");
  hipStream_t st = (hipStream_t)stream;
  const uint64_t ncells = (uint64_t)fine->mesh.G * fine->mesh.G * fine->mesh.G;
  // the coarse handle's candidate list array and a spare control word serve as scratch
  CSK_HIP(launch_collect_children(coarse->set, coarse->slots, coarse->cand_key, coarse->ctl + 2, coarse->max_cand,
                                  coarse->group, ncells, fine->tables(), fine->M, theta, fine->set, fine->slots - 1,
                                  fine->set_count(), fine->max_cand, fine->err(), st),
          "collect_children");
  if (theta != INT32_MIN || coarse->partial_set) fine->partial_set = true;
  return CSK_OK;
}

csk_status csk_candidates_clear(csk_sketch* s, void* stream) {
  if (s == nullptr) return fail(CSK_E_INVALID, "candidates_clear: NULL handle");
  return clear_candidates(s, (hipStream_t)stream);
}

csk_status csk_topk(csk_sketch* s, uint32_t k, uint64_t* keys, int32_t* est, uint32_t* k_out, void* stream) {
  if (s == nullptr || k_out == nullptr) return fail(CSK_E_INVALID, "topk: NULL handle or k_out");
  *k_out = 0;
  if (k > 0 && (keys == nullptr || est == nullptr)) return fail(CSK_E_INVALID, "topk: NULL output");
  if (k > s->max_cand) return fail(CSK_E_INVALID, "topk: k=%u above max_candidates=%u", k, s->max_cand);
  hipStream_t st = (hipStream_t)stream;
  if (k > s->sel_cap) {
    CSK_HIP(hipStreamSynchronize(st), "topk: grow scratch");
    if (s->sel_key) (void)hipFree(s->sel_key);
    if (s->sel_est) (void)hipFree(s->sel_est);
    s->bytes -= (uint64_t)s->sel_cap * (sizeof(uint64_t) + sizeof(int32_t));
    s->sel_key = nullptr;
    s->sel_est = nullptr;
    s->sel_cap = 0;
    CSK_HIP(dmalloc(s, &s->sel_key, k), "topk: scratch");
    CSK_HIP(dmalloc(s, &s->sel_est, k), "topk: scratch");
    s->sel_cap = k;
  }
  if (k > 0) {
    CSK_HIP(launch_topk(s->set, s->slots, s->tables(), s->M, s->max_cand, k, s->sel, s->cand_key, s->cand_est,
                        s->sel_key, s->sel_est, keys, est, s->err(), st),
            "topk");
  } else {
    CSK_HIP(launch_fill_u32((uint32_t*)s->sel, sizeof(SelState) / 4, 0u, st), "topk");
  }
  CSK_HIP(hipMemcpyAsync(s->host_sel, s->sel, sizeof(SelState), hipMemcpyDeviceToHost, st), "topk: read back");
  uint32_t bits = 0;
  csk_status rc = take_latch(s, st, &bits);
  if (rc != CSK_OK) return rc;
  rc = latch_status(bits);
  if (rc != CSK_OK) return rc;
  const uint32_t m = s->host_sel->m;
  const uint32_t got = (k < m) ? k : m;
  *k_out = got;
  if (got < k && s->partial_set)
    return fail(CSK_W_INCOMPLETE, "topk: only %u of %u candidates passed theta", got, k);
  return CSK_OK;
}

csk_status csk_topk_async(csk_sketch* s, uint32_t k, uint64_t* keys, int32_t* est, uint32_t* out, void* stream) {
  if (s == nullptr || out == nullptr) return fail(CSK_E_INVALID, "topk_async: NULL handle or out");
  if (k > 0 && (keys == nullptr || est == nullptr)) return fail(CSK_E_INVALID, "topk_async: NULL output");
  if (k > s->max_cand) return fail(CSK_E_INVALID, "topk_async: k=%u above max_candidates=%u", k, s->max_cand);
  hipStream_t st = (hipStream_t)stream;
  if (k > s->sel_cap) {   // first call with a larger k: grow the scratch (synchronizes)
    CSK_HIP(hipStreamSynchronize(st), "topk_async: grow scratch");
    if (s->sel_key) (void)hipFree(s->sel_key);
    if (s->sel_est) (void)hipFree(s->sel_est);
    s->bytes -= (uint64_t)s->sel_cap * (sizeof(uint64_t) + sizeof(int32_t));
    s->sel_key = nullptr;
    s->sel_est = nullptr;
    s->sel_cap = 0;
    CSK_HIP(dmalloc(s, &s->sel_key, k), "topk_async: scratch");
    CSK_HIP(dmalloc(s, &s->sel_est, k), "topk_async: scratch");
    s->sel_cap = k;
  }
  if (k > 0) {
    CSK_HIP(launch_topk(s->set, s->slots, s->tables(), s->M, s->max_cand, k, s->sel, s->cand_key, s->cand_est,
                        s->sel_key, s->sel_est, keys, est, s->err(), st),
            "topk_async");
  } else {
    CSK_HIP(launch_fill_u32((uint32_t*)s->sel, sizeof(SelState) / 4, 0u, st), "topk_async");
  }
  CSK_HIP(launch_topk_out(s->sel, k, s->partial_set ? 1u : 0u, out, st), "topk_async");
  return CSK_OK;
}

csk_status csk_get_counters(const csk_sketch* cs, int32_t* out, void* stream) {
  csk_sketch* s = const_cast<csk_sketch*>(cs);
  if (s == nullptr || out == nullptr) return fail(CSK_E_INVALID, "get_counters: NULL argument");
  hipStream_t st = (hipStream_t)stream;
  CSK_HIP(hipMemcpyAsync(out, s->M, (uint64_t)s->d * s->w * sizeof(int32_t), hipMemcpyDeviceToDevice, st),
          "get_counters");
  uint32_t bits = 0;
  csk_status rc = take_latch(s, st, &bits);
  if (rc != CSK_OK) return rc;
  return latch_status(bits);
}

csk_status csk_set_counters(csk_sketch* s, const int32_t* in, void* stream) {
  if (s == nullptr || in == nullptr) return fail(CSK_E_INVALID, "set_counters: NULL argument");
  hipStream_t st = (hipStream_t)stream;
  CSK_HIP(hipMemcpyAsync(s->M, in, (uint64_t)s->d * s->w * sizeof(int32_t), hipMemcpyDeviceToDevice, st),
          "set_counters");
  return clear_candidates(s, st);
}

csk_status csk_reset(csk_sketch* s, void* stream) {
  if (s == nullptr) return fail(CSK_E_INVALID, "reset: NULL handle");
  hipStream_t st = (hipStream_t)stream;
  // counters, latch, candidate set (empty slots are all-ones words) and its count in one launch
  FillSpans f{};
  f.p[0] = (uint32_t*)s->M;
  f.n[0] = (uint64_t)s->d * s->w;
  f.p[1] = s->err();
  f.n[1] = 1;
  f.p[2] = (uint32_t*)s->set;
  f.n[2] = 2ull * s->slots;
  f.v[2] = 0xFFFFFFFFu;
  f.p[3] = s->set_count();
  f.n[3] = 1;
  static_assert(kEmptyKey == ~0ull, "an empty slot is two all-ones words");
  CSK_HIP(launch_fill_spans(f, st), "reset");
  s->mesh_set = false;
  s->partial_set = false;
  return CSK_OK;
}

csk_status csk_check(csk_sketch* s, void* stream) {
  if (s == nullptr) return fail(CSK_E_INVALID, "check: NULL handle");
  uint32_t bits = 0;
  csk_status rc = take_latch(s, (hipStream_t)stream, &bits);
  if (rc != CSK_OK) return rc;
  return latch_status(bits);
}

uint64_t csk_device_bytes(const csk_sketch* s) { return s ? s->bytes : 0; }

const char* csk_last_error(void) { return g_last_error; }

}  // extern "C"

// ------------------------------------------------------------------ batched update

struct csk_batch {
  int device = 0;
  uint32_t count = 0, d = 0, mode = 0, nwg_total = 0, nacc_total = 0, lds_bytes = 0;
  int hm = 0;
  BinPlan form{};                // the sort-word kernel's form when form.sort (the same for all)
  uint32_t kb = 6;               // key bytes its hashing looks up (the most any mesh needs)
  std::vector<csk_sketch*> sk;
  std::vector<uint64_t> max_n;
  BinArgs* bin = nullptr;        // per-sketch bin arguments (device)
  AccArgs* acc = nullptr;        // per-sketch accumulate arguments (device)
  uint16_t* wg_sketch = nullptr; // bin workgroup -> sketch (device)
  uint32_t* wg_first = nullptr;  // sketch -> its first bin workgroup (device)
  uint16_t* acc_sketch = nullptr;
  uint32_t* acc_first = nullptr;
  uint16_t* tok = nullptr;       // every sketch's token regions
  uint32_t* cnt = nullptr;
  TopkDesc* topk = nullptr;      // per-sketch top-k descriptors (device), built on first use
  std::vector<TopkDesc> topk_host;
  std::vector<double> delta, L;  // each sketch's mesh (latched again by a collect after a reset)
  // batched candidate pass
  CollectDesc* cdesc = nullptr;  // per-sketch collect descriptors (device)
  std::vector<CollectDesc> cdesc_host;
  uint16_t* cwg_sketch = nullptr; // collect workgroup -> sketch (device)
  uint32_t* cwg_first = nullptr;  // sketch -> its first collect workgroup
  uint32_t* cwg_count = nullptr;  // sketch -> its collect workgroups
  uint32_t ncwg_total = 0;
  bool cfield = false;            // every sketch uses the field-probe filter
  bool cgrouped = false;          // some sketch has grouped items: collects go one by one
  uint32_t w_max = 0;
  ResetSpans* rspans = nullptr;   // the clears of every sketch's reset (device)
  uint64_t rmax = 0;              // the longest span
};

namespace {

void batch_free(csk_batch* b) {
  void* ptrs[] = {b->bin,       b->acc,       b->wg_sketch, b->wg_first,  b->acc_sketch, b->acc_first, b->tok,
                  b->cnt,       b->topk,      b->cdesc,     b->cwg_sketch, b->cwg_first,  b->cwg_count,  b->rspans};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

template <typename T>
hipError_t bmalloc(T** p, uint64_t count) {
  return hipMalloc((void**)p, (count ? count : 1) * sizeof(T));
}

}  // namespace

namespace {

csk_status batch_create_impl(csk_batch** out, csk_sketch* const* sketches, const uint64_t* max_n, uint32_t count,
                             const double* delta, const double* L, uint32_t wg_budget) {
  if (out == nullptr) return fail(CSK_E_INVALID, "batch_create: out is NULL");
  *out = nullptr;
  if (sketches == nullptr || max_n == nullptr) return fail(CSK_E_INVALID, "batch_create: NULL array");
  if (count < 1 || count > kMaxBatch) return fail(CSK_E_INVALID, "batch_create: count=%u outside [1, %u]", count, kMaxBatch);
  for (uint32_t i = 0; i < count; ++i) {
    if (sketches[i] == nullptr) return fail(CSK_E_INVALID, "batch_create: sketch %u is NULL", i);
    for (uint32_t j = 0; j < i; ++j)
      if (sketches[j] == sketches[i]) return fail(CSK_E_INVALID, "batch_create: sketch %u appears twice", i);
  }
  const csk_sketch* s0 = sketches[0];
  if (s0->d > (uint32_t)kTabLdsRows) return fail(CSK_E_INVALID, "batch_create: d=%u above %d", s0->d, kTabLdsRows);
  const int hm = s0->tables().hash_mode();
  Mesh mesh0;
  for (uint32_t i = 0; i < count; ++i) {
    const csk_sketch* s = sketches[i];
    if (s->d != s0->d) return fail(CSK_E_INVALID, "batch_create: sketches of different d (%u, %u)", s0->d, s->d);
    if (s->device != s0->device) return fail(CSK_E_INVALID, "batch_create: sketches on different devices");
    if (s->tables().hash_mode() != hm)
      return fail(CSK_E_INVALID, "batch_create: widths need different hash forms (sketch %u, w=%u)", i, s->w);
    Mesh m;
    csk_status rc = check_mesh(sketches[i], delta[i], L[i], &m);
    if (rc != CSK_OK) return rc;
    if (i == 0) mesh0 = m;
    if (m.mode != mesh0.mode)
      return fail(CSK_E_INVALID, "batch_create: meshes need different cell-index paths (sketch %u)", i);
  }
  for (uint32_t i = 0; i < count; ++i) {
    Mesh m;
    (void)check_mesh(sketches[i], delta[i], L[i], &m);
    latch_mesh(sketches[i], delta[i], L[i], m);
  }
  const uint32_t d = s0->d;
  const uint64_t tile = (uint64_t)kBin2Threads * bin2_ppt((int)d);
  uint64_t total_tiles = 0;
  std::vector<uint64_t> tiles(count);
  for (uint32_t i = 0; i < count; ++i) {
    tiles[i] = (max_n[i] + tile - 1) / tile;
    total_tiles += tiles[i];
  }
  const uint64_t budget = wg_budget ? wg_budget : 512;
  std::vector<BinArgs> hb(count);
  std::vector<AccArgs> ha(count);
  std::vector<uint16_t> wg_map, acc_map;
  std::vector<uint32_t> wg_first(count), acc_first(count);
  uint64_t tok_words = 0, cnt_words = 0, lds = 0;
  std::vector<uint64_t> tok_off(count), cnt_off(count);
  std::vector<BinPlan> plans(count);
  for (uint32_t i = 0; i < count; ++i) {
    uint64_t want = total_tiles ? (budget * tiles[i] + total_tiles / 2) / total_tiles : 1;
    if (want < 1) want = 1;
    BinPlan& p = plans[i];
    if (!plan_bin_wg(max_n[i] ? max_n[i] : 1, d, sketches[i]->w, want, p) || !p.fast)
      return fail(CSK_E_INVALID, "batch_create: sketch %u (w=%u) does not fit the binned path", i, sketches[i]->w);
    tok_off[i] = tok_words;
    cnt_off[i] = cnt_words;
    tok_words += (uint64_t)p.P * p.nwg * p.cap;
    cnt_words += (uint64_t)p.P * p.nwg;
    if (p.lds_bytes > lds) lds = p.lds_bytes;
    wg_first[i] = (uint32_t)wg_map.size();
    for (uint32_t g = 0; g < p.nwg; ++g) wg_map.push_back((uint16_t)i);
    acc_first[i] = (uint32_t)acc_map.size();
    for (uint32_t q = 0; q < p.P; ++q) acc_map.push_back((uint16_t)i);
  }
  // the sort-word kernel serves the batch when it serves every sketch in the same form
  bool sort_all = true;
  for (uint32_t i = 0; i < count && sort_all; ++i) {
    const csk_sketch* s = sketches[i];
    sort_all = plan_sortbin(plans[i], d, mesh0, s->tables(), s0->upd_form, s0->upd_nt, s0->upd_rp, s0->upd_pf,
                            false) &&
               plans[i].nt == plans[0].nt && plans[i].rp == plans[0].rp && plans[i].pf == plans[0].pf;
  }
  BinPlan form{};
  if (sort_all) {
    form = plans[0];
    for (uint32_t i = 0; i < count; ++i)
      if (plans[i].lds_bytes > lds) lds = plans[i].lds_bytes;
  } else {
    lds = 0;
    for (uint32_t i = 0; i < count; ++i) {
      BinPlan p;
      (void)plan_bin_wg(max_n[i] ? max_n[i] : 1, d, sketches[i]->w, plans[i].nwg, p);
      plans[i] = p;   // the general kernel's plan (same tiles, workgroups and regions)
      if (p.lds_bytes > lds) lds = p.lds_bytes;
    }
  }
  if (wg_map.size() > 65535 || acc_map.size() > (1u << 30))
    return fail(CSK_E_INVALID, "batch_create: %zu workgroups exceed the launch limit", wg_map.size());
  csk_batch* b = new (std::nothrow) csk_batch();
  if (!b) return fail(CSK_E_NOMEM, "batch_create: host allocation failed");
  b->device = s0->device;
  b->count = count;
  b->d = d;
  b->mode = mesh0.mode;
  b->hm = hm;
  b->sk.assign(sketches, sketches + count);
  b->max_n.assign(max_n, max_n + count);
  b->nwg_total = (uint32_t)wg_map.size();
  b->nacc_total = (uint32_t)acc_map.size();
  b->lds_bytes = (uint32_t)lds;
  b->form = form;
  b->kb = 5;
  for (uint32_t i = 0; i < count; ++i) {
    Mesh m;
    (void)check_mesh(sketches[i], delta[i], L[i], &m);
    if (key_bytes_kb(m.nch) > b->kb) b->kb = key_bytes_kb(m.nch);
  }
  hipError_t e = bmalloc(&b->bin, count);
  if (e == hipSuccess) e = bmalloc(&b->acc, count);
  if (e == hipSuccess) e = bmalloc(&b->wg_sketch, wg_map.size());
  if (e == hipSuccess) e = bmalloc(&b->wg_first, count);
  if (e == hipSuccess) e = bmalloc(&b->acc_sketch, acc_map.size());
  if (e == hipSuccess) e = bmalloc(&b->acc_first, count);
  if (e == hipSuccess) e = bmalloc(&b->tok, tok_words);
  if (e == hipSuccess) e = bmalloc(&b->cnt, cnt_words);
  if (e == hipSuccess) {
    for (uint32_t i = 0; i < count; ++i) {
      csk_sketch* s = sketches[i];
      Mesh m;
      (void)check_mesh(s, delta[i], L[i], &m);
      hb[i] = make_bin_args(nullptr, 0, m, s->tables(), plans[i], b->tok + tok_off[i], b->cnt + cnt_off[i], s->M,
                            s->err());
      ha[i].tok = b->tok + tok_off[i];
      ha[i].cnt = b->cnt + cnt_off[i];
      ha[i].plan = plans[i];
      ha[i].w = s->w;
      ha[i].M = s->M;
    }
    e = hipMemcpy(b->bin, hb.data(), count * sizeof(BinArgs), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemcpy(b->acc, ha.data(), count * sizeof(AccArgs), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->wg_sketch, wg_map.data(), wg_map.size() * 2, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->wg_first, wg_first.data(), count * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->acc_sketch, acc_map.data(), acc_map.size() * 2, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->acc_first, acc_first.data(), count * 4, hipMemcpyHostToDevice);
  // the batched candidate pass: one descriptor per sketch and a static share of the collect
  // workgroups in proportion to each stream's tiles (at least one each)
  b->delta.assign(delta, delta + count);
  b->L.assign(L, L + count);
  if (e == hipSuccess) {
    const uint64_t ctile = (uint64_t)kCollectThreads * kCollectPPT;
    const uint64_t cbudget = 1024;
    uint64_t ct_total = 0;
    std::vector<uint64_t> ct(count);
    for (uint32_t i = 0; i < count; ++i) {
      ct[i] = (max_n[i] + ctile - 1) / ctile;
      ct_total += ct[i];
    }
    std::vector<uint16_t> cmap;
    std::vector<uint32_t> cfirst(count), ccount(count);
    b->cfield = true;
    b->cdesc_host.resize(count);
    ResetSpans rs{};
    for (uint32_t i = 0; i < count; ++i) {
      csk_sketch* s = sketches[i];
      Mesh m;
      (void)check_mesh(s, delta[i], L[i], &m);
      const Tables t = s->tables();
      b->cfield = b->cfield && collect_field_form(t);
      b->cgrouped = b->cgrouped || s->group != 1u;
      b->w_max = s->w > b->w_max ? s->w : b->w_max;
      b->cdesc_host[i] = CollectDesc{m,           t,           s->M,          s->filter,
                                     s->filter ? s->filter + kFilterAllocWords : nullptr,
                                     s->hot_table, s->set,     s->slots - 1,  s->set_count(),
                                     s->max_cand, s->err()};
      uint64_t want = ct_total ? (cbudget * ct[i] + ct_total / 2) / ct_total : 1;
      if (want > ct[i]) want = ct[i];
      if (want < 1) want = 1;
      cfirst[i] = (uint32_t)cmap.size();
      ccount[i] = (uint32_t)want;
      for (uint64_t g = 0; g < want; ++g) cmap.push_back((uint16_t)i);
      rs.p[i][0] = (uint32_t*)s->M;
      rs.n[i][0] = (uint64_t)s->d * s->w;
      rs.p[i][1] = s->err();
      rs.n[i][1] = 1;
      rs.p[i][2] = (uint32_t*)s->set;
      rs.n[i][2] = 2ull * s->slots;
      rs.v[i][2] = 0xFFFFFFFFu;
      rs.p[i][3] = s->set_count();
      rs.n[i][3] = 1;
      for (int r = 0; r < kFillSpans; ++r) b->rmax = rs.n[i][r] > b->rmax ? rs.n[i][r] : b->rmax;
    }
    b->ncwg_total = (uint32_t)cmap.size();
    if (cmap.size() > 65535) e = hipErrorInvalidValue;
    if (e == hipSuccess) e = bmalloc(&b->cdesc, count);
    if (e == hipSuccess) e = bmalloc(&b->cwg_sketch, cmap.size());
    if (e == hipSuccess) e = bmalloc(&b->cwg_first, count);
    if (e == hipSuccess) e = bmalloc(&b->cwg_count, count);
    if (e == hipSuccess) e = bmalloc(&b->rspans, 1);
    if (e == hipSuccess)
      e = hipMemcpy(b->cdesc, b->cdesc_host.data(), count * sizeof(CollectDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->cwg_sketch, cmap.data(), cmap.size() * 2, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->cwg_first, cfirst.data(), count * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->cwg_count, ccount.data(), count * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->rspans, &rs, sizeof(ResetSpans), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    batch_free(b);
    delete b;
    return hip_fail(e, "batch_create");
  }
  *out = b;
  return CSK_OK;
}

}  // namespace

csk_status csk_batch_create(csk_batch** out, csk_sketch* const* sketches, const uint64_t* max_n, uint32_t count,
                            double delta, double L, uint32_t wg_budget) {
  if (count < 1 || count > kMaxBatch) {
    if (out != nullptr) *out = nullptr;
    return fail(CSK_E_INVALID, "batch_create: count=%u outside [1, %u]", count, kMaxBatch);
  }
  std::vector<double> d(count, delta), l(count, L);
  return batch_create_impl(out, sketches, max_n, count, d.data(), l.data(), wg_budget);
}

csk_status csk_batch_create_meshes(csk_batch** out, csk_sketch* const* sketches, const uint64_t* max_n,
                                   uint32_t count, const double* delta, const double* L, uint32_t wg_budget) {
  if (delta == nullptr || L == nullptr) {
    if (out != nullptr) *out = nullptr;
    return fail(CSK_E_INVALID, "batch_create_meshes: NULL mesh arrays");
  }
  return batch_create_impl(out, sketches, max_n, count, delta, L, wg_budget);
}

csk_status csk_batch_update(csk_batch* b, const float* const* pos, const uint64_t* n, void* stream) {
  if (b == nullptr || pos == nullptr || n == nullptr) return fail(CSK_E_INVALID, "batch_update: NULL argument");
  BatchCall call{};
  for (uint32_t i = 0; i < b->count; ++i) {
    if (n[i] > b->max_n[i])
      return fail(CSK_E_INVALID, "batch_update: n[%u]=%llu above its max_n %llu", i, (unsigned long long)n[i],
                  (unsigned long long)b->max_n[i]);
    if (n[i] > 0 && pos[i] == nullptr) return fail(CSK_E_INVALID, "batch_update: pos[%u] is NULL", i);
    call.pos[i] = pos[i];
    call.n[i] = n[i];
  }
  hipStream_t st = (hipStream_t)stream;
  if (b->form.sort)
    CSK_HIP(launch_sortbin_batch(b->bin, b->wg_sketch, b->wg_first, b->nwg_total, b->lds_bytes, b->d, b->mode, b->form, b->kb,
                                 call, st),
            "batch_update (bin)");
  else
    CSK_HIP(launch_bin_batch(b->bin, b->wg_sketch, b->wg_first, b->nwg_total, b->lds_bytes, b->d, b->mode, b->hm,
                             call, st),
            "batch_update (bin)");
  CSK_HIP(launch_accumulate_batch(b->acc, b->acc_sketch, b->acc_first, b->nacc_total, st), "batch_update (accumulate)");
  return CSK_OK;
}

csk_status csk_batch_topk(csk_batch* b, const uint32_t* k, uint64_t* const* keys, int32_t* const* est,
                          uint32_t* const* out, void* stream) {
  if (b == nullptr || k == nullptr || out == nullptr) return fail(CSK_E_INVALID, "batch_topk: NULL argument");
  hipStream_t st = (hipStream_t)stream;
  uint32_t k_max = 0, slots_max = 0, mc_max = 0;
  for (uint32_t i = 0; i < b->count; ++i) {
    const csk_sketch* s = b->sk[i];
    if (k[i] > s->max_cand)
      return fail(CSK_E_INVALID, "batch_topk: k[%u]=%u above max_candidates=%u", i, k[i], s->max_cand);
    if (k[i] > 0 && (keys == nullptr || est == nullptr || keys[i] == nullptr || est[i] == nullptr))
      return fail(CSK_E_INVALID, "batch_topk: NULL output of sketch %u", i);
    if (out[i] == nullptr) return fail(CSK_E_INVALID, "batch_topk: out[%u] is NULL", i);
    k_max = k[i] > k_max ? k[i] : k_max;
    slots_max = s->slots > slots_max ? s->slots : slots_max;
    mc_max = s->max_cand > mc_max ? s->max_cand : mc_max;
  }
  // the selection scratch of each sketch holds its k (grown here, synchronizing, as by csk_topk_async)
  for (uint32_t i = 0; i < b->count; ++i) {
    csk_sketch* s = b->sk[i];
    if (k[i] <= s->sel_cap) continue;
    CSK_HIP(hipStreamSynchronize(st), "batch_topk: grow scratch");
    if (s->sel_key) (void)hipFree(s->sel_key);
    if (s->sel_est) (void)hipFree(s->sel_est);
    s->bytes -= (uint64_t)s->sel_cap * (sizeof(uint64_t) + sizeof(int32_t));
    s->sel_key = nullptr;
    s->sel_est = nullptr;
    s->sel_cap = 0;
    CSK_HIP(dmalloc(s, &s->sel_key, k[i]), "batch_topk: scratch");
    CSK_HIP(dmalloc(s, &s->sel_est, k[i]), "batch_topk: scratch");
    s->sel_cap = k[i];
  }
  // descriptors: built once, rebuilt when a sketch's selection scratch moved
  bool stale = b->topk == nullptr || b->topk_host.size() != b->count;
  for (uint32_t i = 0; !stale && i < b->count; ++i)
    stale = b->topk_host[i].sk != b->sk[i]->sel_key || b->topk_host[i].se != b->sk[i]->sel_est;
  if (stale) {
    std::vector<TopkDesc> h(b->count);
    for (uint32_t i = 0; i < b->count; ++i) {
      csk_sketch* s = b->sk[i];
      h[i] = TopkDesc{s->set, s->slots, s->max_cand, s->tables(), s->M, s->sel, s->cand_key, s->cand_est,
                      s->sel_key, s->sel_est, s->err()};
    }
    CSK_HIP(hipStreamSynchronize(st), "batch_topk: descriptors");
    if (b->topk == nullptr) CSK_HIP(bmalloc(&b->topk, b->count), "batch_topk: descriptors");
    CSK_HIP(hipMemcpy(b->topk, h.data(), sizeof(TopkDesc) * b->count, hipMemcpyHostToDevice),
            "batch_topk: descriptors");
    b->topk_host = h;
  }
  TopkCall call{};
  for (uint32_t i = 0; i < b->count; ++i) {
    call.keys[i] = k[i] ? keys[i] : nullptr;
    call.est[i] = k[i] ? est[i] : nullptr;
    call.out[i] = out[i];
    call.k[i] = k[i];
    call.partial[i] = b->sk[i]->partial_set ? 1u : 0u;
    // the set holds keys of the latched mesh only (a different mesh needs a reset), all
    // below G^3: the rank count compares (estimate, key) as one word when that is <= 2^32
    const uint64_t G = b->sk[i]->mesh_set ? (uint64_t)b->sk[i]->mesh.G : 0u;
    call.key32[i] = (b->sk[i]->mesh_set && G * G * G <= (1ull << 32)) ? 1u : 0u;
  }
  CSK_HIP(launch_topk_batch(b->topk, b->count, b->d, slots_max, mc_max, k_max, call, st), "batch_topk");
  return CSK_OK;
}

csk_status csk_batch_reset(csk_batch* b, void* stream) {
  if (b == nullptr) return fail(CSK_E_INVALID, "batch_reset: NULL batch");
  CSK_HIP(launch_fill_spans_batch(b->rspans, b->count, b->rmax, (hipStream_t)stream), "batch_reset");
  for (csk_sketch* s : b->sk) {
    s->mesh_set = false;
    s->partial_set = false;
  }
  return CSK_OK;
}

csk_status csk_batch_collect(csk_batch* b, const float* const* pos, const uint64_t* n, const int32_t* theta,
                             void* stream) {
  if (b == nullptr || pos == nullptr || n == nullptr || theta == nullptr)
    return fail(CSK_E_INVALID, "batch_collect: NULL argument");
  for (uint32_t i = 0; i < b->count; ++i) {
    if (n[i] > (1ull << 40)) return fail(CSK_E_INVALID, "batch_collect: n[%u] above 2^40", i);
    if (n[i] > 0 && pos[i] == nullptr) return fail(CSK_E_INVALID, "batch_collect: pos[%u] is NULL", i);
    Mesh m;
    csk_status rc = check_mesh(b->sk[i], b->delta[i], b->L[i], &m);
    if (rc != CSK_OK) return rc;
  }
  hipStream_t st = (hipStream_t)stream;
  if (b->cgrouped) {   // grouped items: the general collect, sketch by sketch
    for (uint32_t i = 0; i < b->count; ++i) {
      csk_status rc = csk_collect(b->sk[i], pos[i], n[i], b->delta[i], b->L[i], theta[i], stream);
      if (rc != CSK_OK) return rc;
    }
    return CSK_OK;
  }
  CollectCall call{};
  for (uint32_t i = 0; i < b->count; ++i) {
    csk_sketch* s = b->sk[i];
    Mesh m;
    (void)check_mesh(s, b->delta[i], b->L[i], &m);
    latch_mesh(s, b->delta[i], b->L[i], m);
    if (theta[i] != INT32_MIN) s->partial_set = true;
    call.pos[i] = n[i] ? pos[i] : nullptr;
    call.n[i] = n[i];
    call.theta[i] = theta[i];
    call.use_filter[i] = (s->filter != nullptr && theta[i] > 0) ? 1u : 0u;
  }
  CSK_HIP(launch_collect_batch(b->cdesc, b->cdesc_host.data(), b->count, b->cwg_sketch, b->cwg_first, b->cwg_count,
                               b->ncwg_total, b->d, b->mode, b->hm, b->cfield, b->w_max, call, st),
          "batch_collect");
  return CSK_OK;
}

csk_status csk_batch_destroy(csk_batch* b) {
  if (b == nullptr) return CSK_OK;
  (void)hipDeviceSynchronize();
  batch_free(b);
  delete b;
  return CSK_OK;
}

// ------------------------------------------------------------------ learned router

struct csk_mlp {
  int device = 0;
  uint32_t max_batch = 0;
  uint64_t step = 0;
  float* p = nullptr;     // fp32 master parameters (kParams)
  float* g = nullptr;     // gradients
  float* m1 = nullptr;    // Adam moments
  float* m2 = nullptr;
  float* H1 = nullptr;    // [max_batch][64]
  float* H2 = nullptr;
  float* dA2 = nullptr;
  float* dA1 = nullptr;
  float* z = nullptr;     // [max_batch]
  float* dz = nullptr;
  float* loss = nullptr;  // [1]
  float* part = nullptr;  // split-k partial products of the weight gradients
  uint64_t part_floats = 0;
};

namespace {

void mlp_free(csk_mlp* m) {
  void* ptrs[] = {m->p, m->g, m->m1, m->m2, m->H1, m->H2, m->dA2, m->dA1, m->z, m->dz, m->loss, m->part};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
}

// forward of rows [0, b) of x into H1, H2 and z (logits)
// The forward pass over b rows.  The training pass (y != NULL) rounds every matrix operand to
// bf16; the scoring pass carries each as a hi + lo bf16 pair (three products per MFMA tile)
// and does not round the output layer, so its logits stay within fp32 roundings of the fp32
// forward pass of the same weights.
hipError_t mlp_forward_rows(csk_mlp* m, const float* x, uint32_t b, float* z, const float* y, hipStream_t st) {
  const float* P = m->p;
  const bool split = (y == nullptr);
  hipError_t e = launch_gemm_bf16(b, kHidden, kFeatPad, x, kFeatPad, 1, P + kOffW1, 1, kFeatPad, m->H1, kHidden, 1,
                                  0.0f, st, nullptr, 0, split);
  if (e == hipSuccess) e = launch_bias_act(m->H1, b, kHidden, P + kOffB1, true, st);
  if (e == hipSuccess)
    e = launch_gemm_bf16(b, kHidden, kHidden, m->H1, kHidden, 1, P + kOffW2, 1, kHidden, m->H2, kHidden, 1, 0.0f, st,
                         nullptr, 0, split);
  if (e == hipSuccess) e = launch_bias_act(m->H2, b, kHidden, P + kOffB2, true, st);
  if (e == hipSuccess) e = launch_head(m->H2, b, P + kOffW3, P + kOffB3, z, y, m->dz, m->loss, !split, st);
  return e;
}

}  // namespace

csk_status csk_mlp_create(csk_mlp** out, uint64_t seed, uint32_t max_batch) {
  if (out == nullptr) return fail(CSK_E_INVALID, "mlp_create: out is NULL");
  *out = nullptr;
  if (max_batch < 1 || max_batch > (1u << 22)) return fail(CSK_E_INVALID, "mlp_create: max_batch outside [1, 2^22]");
  csk_mlp* m = new (std::nothrow) csk_mlp();
  if (!m) return fail(CSK_E_NOMEM, "mlp_create: host allocation failed");
  m->max_batch = max_batch;
  // He-uniform weights U(-sqrt(6 / fan_in), +sqrt(6 / fan_in)) from SplitMix64(seed); biases 0
  std::vector<float> P(kParams, 0.0f);
  uint64_t st = seed;
  auto uni = [&]() { return (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0); };
  for (uint32_t i = 0; i < 64u * 32u; ++i) P[kOffW1 + i] = (float)((2.0 * uni() - 1.0) * std::sqrt(6.0 / 27.0));
  for (uint32_t i = 0; i < 64u * 64u; ++i) P[kOffW2 + i] = (float)((2.0 * uni() - 1.0) * std::sqrt(6.0 / 64.0));
  for (uint32_t i = 0; i < 64u; ++i) P[kOffW3 + i] = (float)((2.0 * uni() - 1.0) * std::sqrt(6.0 / 64.0));
  for (uint32_t r = 0; r < 64u; ++r)   // the 5 padding inputs carry no weight
    for (uint32_t c = 27; c < 32u; ++c) P[kOffW1 + r * 32 + c] = 0.0f;
  hipError_t e = hipGetDevice(&m->device);
  const uint64_t hb = (uint64_t)max_batch * kHidden;
  if (e == hipSuccess) e = bmalloc(&m->p, kParams);
  if (e == hipSuccess) e = bmalloc(&m->g, kParams);
  if (e == hipSuccess) e = bmalloc(&m->m1, kParams);
  if (e == hipSuccess) e = bmalloc(&m->m2, kParams);
  if (e == hipSuccess) e = bmalloc(&m->H1, hb);
  if (e == hipSuccess) e = bmalloc(&m->H2, hb);
  if (e == hipSuccess) e = bmalloc(&m->dA2, hb);
  if (e == hipSuccess) e = bmalloc(&m->dA1, hb);
  if (e == hipSuccess) e = bmalloc(&m->z, max_batch);
  if (e == hipSuccess) e = bmalloc(&m->dz, max_batch);
  if (e == hipSuccess) e = bmalloc(&m->loss, 1);
  m->part_floats = ((uint64_t)max_batch + kSplitK - 1) / kSplitK * kHidden * kHidden;
  if (e == hipSuccess) e = bmalloc(&m->part, m->part_floats);
  if (e == hipSuccess) e = hipMemcpy(m->p, P.data(), kParams * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_fill_u32((uint32_t*)m->m1, kParams, 0u, nullptr);
  if (e == hipSuccess) e = launch_fill_u32((uint32_t*)m->m2, kParams, 0u, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    mlp_free(m);
    delete m;
    return hip_fail(e, "mlp_create");
  }
  *out = m;
  return CSK_OK;
}

csk_status csk_mlp_destroy(csk_mlp* m) {
  if (m == nullptr) return CSK_OK;
  (void)hipDeviceSynchronize();
  mlp_free(m);
  delete m;
  return CSK_OK;
}

csk_status csk_mlp_params(csk_mlp* m, float* out, const float* in) {
  if (m == nullptr || (out == nullptr && in == nullptr)) return fail(CSK_E_INVALID, "mlp_params: NULL argument");
  if (in != nullptr) {
    CSK_HIP(hipMemcpy(m->p, in, kParams * sizeof(float), hipMemcpyHostToDevice), "mlp_params");
    m->step = 0;
    CSK_HIP(launch_fill_u32((uint32_t*)m->m1, kParams, 0u, nullptr), "mlp_params");
    CSK_HIP(launch_fill_u32((uint32_t*)m->m2, kParams, 0u, nullptr), "mlp_params");
  }
  if (out != nullptr) CSK_HIP(hipMemcpy(out, m->p, kParams * sizeof(float), hipMemcpyDeviceToHost), "mlp_params");
  CSK_HIP(hipDeviceSynchronize(), "mlp_params");
  return CSK_OK;
}

csk_status csk_mlp_grads(csk_mlp* m, float* out) {
  if (m == nullptr || out == nullptr) return fail(CSK_E_INVALID, "mlp_grads: NULL argument");
  CSK_HIP(hipDeviceSynchronize(), "mlp_grads");
  CSK_HIP(hipMemcpy(out, m->g, kParams * sizeof(float), hipMemcpyDeviceToHost), "mlp_grads");
  return CSK_OK;
}

csk_status csk_mlp_forward(csk_mlp* m, const float* x, uint64_t n, float* logits, void* stream) {
  if (m == nullptr || (n > 0 && (x == nullptr || logits == nullptr))) return fail(CSK_E_INVALID, "mlp_forward: NULL");
  hipStream_t st = (hipStream_t)stream;
  for (uint64_t off = 0; off < n; off += m->max_batch) {
    const uint32_t b = (uint32_t)((n - off < m->max_batch) ? n - off : m->max_batch);
    CSK_HIP(mlp_forward_rows(m, x + off * kFeatPad, b, logits + off, nullptr, st), "mlp_forward");
  }
  return CSK_OK;
}

csk_status csk_mlp_train_step(csk_mlp* m, const float* x, const float* y, uint32_t n, float lr, float* loss,
                              void* stream) {
  if (m == nullptr || x == nullptr || y == nullptr) return fail(CSK_E_INVALID, "mlp_train_step: NULL argument");
  if (n < 1 || n > m->max_batch) return fail(CSK_E_INVALID, "mlp_train_step: n=%u outside [1, %u]", n, m->max_batch);
  hipStream_t st = (hipStream_t)stream;
  float* P = m->p;
  float* G = m->g;
  CSK_HIP(launch_fill_u32((uint32_t*)m->loss, 1, 0u, st), "mlp_train_step");
  CSK_HIP(mlp_forward_rows(m, x, n, m->z, y, st), "mlp_train_step (forward)");
  // output layer: dw3 = H2^T dz, db3 = sum dz
  CSK_HIP(launch_colsum(m->H2, n, kHidden, kHidden, m->dz, G + kOffW3, st), "mlp_train_step");
  CSK_HIP(launch_colsum(m->dz, n, 1, 1, nullptr, G + kOffB3, st), "mlp_train_step");
  // second layer: dA2 = (dz w3^T) masked by ReLU; dW2 = dA2^T H1; db2 = colsum dA2
  CSK_HIP(launch_head_back(m->dz, m->H2, P + kOffW3, n, m->dA2, st), "mlp_train_step");
  CSK_HIP(launch_gemm_bf16(kHidden, kHidden, n, m->dA2, 1, kHidden, m->H1, kHidden, 1, G + kOffW2, kHidden, 1, 0.0f,
                           st, m->part, m->part_floats),
          "mlp_train_step");
  CSK_HIP(launch_colsum(m->dA2, n, kHidden, kHidden, nullptr, G + kOffB2, st), "mlp_train_step");
  // first layer: dA1 = (dA2 W2) masked by ReLU; dW1 = dA1^T X; db1 = colsum dA1
  CSK_HIP(launch_gemm_bf16(n, kHidden, kHidden, m->dA2, kHidden, 1, P + kOffW2, kHidden, 1, m->dA1, kHidden, 1, 0.0f,
                           st),
          "mlp_train_step");
  CSK_HIP(launch_relu_back(m->dA1, m->H1, (uint64_t)n * kHidden, st), "mlp_train_step");
  CSK_HIP(launch_gemm_bf16(kHidden, kFeatPad, n, m->dA1, 1, kHidden, x, kFeatPad, 1, G + kOffW1, kFeatPad, 1, 0.0f,
                           st, m->part, m->part_floats),
          "mlp_train_step");
  CSK_HIP(launch_colsum(m->dA1, n, kHidden, kHidden, nullptr, G + kOffB1, st), "mlp_train_step");
  // Adam
  m->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const double lr_t = lr * std::sqrt(1.0 - std::pow(b2, (double)m->step)) / (1.0 - std::pow(b1, (double)m->step));
  CSK_HIP(launch_adam(P, G, m->m1, m->m2, kParams, (float)lr_t, (float)b1, (float)b2, 1e-8f, st), "mlp_train_step");
  if (loss != nullptr)
    CSK_HIP(hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToDevice, st), "mlp_train_step");
  return CSK_OK;
}

csk_status csk_gemm_bf16(uint32_t M, uint32_t N, uint32_t K, const float* A, uint64_t sai, uint64_t sak,
                         const float* B, uint64_t sbk, uint64_t sbj, float* C, uint64_t sci, uint64_t scj,
                         float beta, void* stream) {
  if (M > (1u << 20) || N > (1u << 20)) return fail(CSK_E_INVALID, "gemm_bf16: M=%u or N=%u above 2^20", M, N);
  if (M == 0 || N == 0) return CSK_OK;
  if (C == nullptr || (K > 0 && (A == nullptr || B == nullptr))) return fail(CSK_E_INVALID, "gemm_bf16: NULL pointer");
  CSK_HIP(launch_gemm_bf16(M, N, K, A, sai, sak, B, sbk, sbj, C, sci, scj, beta, (hipStream_t)stream), "gemm_bf16");
  return CSK_OK;
}

csk_status csk_sample_counts(const float* pos, uint64_t n, uint64_t index0, double delta_c, double L, uint64_t seed,
                             uint32_t threshold, uint32_t* counts, uint32_t* bitmap, void* stream) {
  Mesh coarse;
  csk_status rc = check_mesh(nullptr, delta_c, L, &coarse);
  if (rc != CSK_OK) return rc;
  if (n > 0 && (pos == nullptr || counts == nullptr)) return fail(CSK_E_INVALID, "sample_counts: NULL pointer");
  if (n == 0) return CSK_OK;
  CSK_HIP(launch_sample_counts(pos, n, index0, seed, threshold, coarse, counts, bitmap, (hipStream_t)stream),
          "sample_counts");
  return CSK_OK;
}

csk_status csk_cell_features(const uint32_t* counts, double delta_c, double L, const uint64_t* cells, uint64_t m,
                             float* feat, void* stream) {
  Mesh coarse;
  csk_status rc = check_mesh(nullptr, delta_c, L, &coarse);
  if (rc != CSK_OK) return rc;
  if (m > 0 && (counts == nullptr || cells == nullptr || feat == nullptr))
    return fail(CSK_E_INVALID, "cell_features: NULL pointer");
  if (m == 0) return CSK_OK;
  CSK_HIP(launch_features(counts, (uint32_t)coarse.G, cells, m, feat, (hipStream_t)stream), "cell_features");
  return CSK_OK;
}

csk_status csk_route_split_workspace(uint32_t na, uint32_t factor, uint64_t* bytes) {
  if (bytes == nullptr) return fail(CSK_E_INVALID, "route_split_workspace: bytes is NULL");
  if (factor < 1 || factor > 32 || na > kMaxAdmitted || (uint64_t)na * factor * factor * factor > kSplitMaxChildren)
    return fail(CSK_E_INVALID, "route_split_workspace: na=%u, factor=%u outside the limits", na, factor);
  *bytes = split_workspace_bytes(na, factor);
  return CSK_OK;
}

csk_status csk_route_split(const float* pos, uint64_t n, double delta, double L, uint32_t factor,
                           const uint64_t* admitted, uint32_t na, uint64_t* table_keys, uint32_t* table_counts,
                           uint32_t table_slots, float* rest_pos, uint64_t* rest_count, uint32_t* err,
                           void* workspace, uint64_t workspace_bytes, void* stream) {
  Mesh mesh;
  csk_status rc = check_mesh(nullptr, delta, L, &mesh);
  if (rc != CSK_OK) return rc;
  if (factor < 1 || factor > 32 || (uint32_t)mesh.G % factor != 0)
    return fail(CSK_E_INVALID, "route_split: factor %u does not divide G=%d", factor, mesh.G);
  if (na > kMaxAdmitted) return fail(CSK_E_INVALID, "route_split: %u admitted cells above %u", na, kMaxAdmitted);
  const uint64_t children = (uint64_t)na * factor * factor * factor;
  if (children > kSplitMaxChildren)
    return fail(CSK_E_INVALID, "route_split: %u cells of %u^3 children exceed %u", na, factor, kSplitMaxChildren);
  if (table_slots < 2 || (table_slots & (table_slots - 1)) != 0)
    return fail(CSK_E_INVALID, "route_split: table_slots=%u is not a power of two", table_slots);
  if (children > table_slots / 2)
    return fail(CSK_E_INVALID, "route_split: %u cells of %u^3 children exceed half of %u slots", na, factor,
                table_slots);
  if (n > 0 && workspace_bytes < split_workspace_bytes(na, factor))
    return fail(CSK_E_INVALID, "route_split: workspace of %llu bytes below the %llu needed",
                (unsigned long long)workspace_bytes, (unsigned long long)split_workspace_bytes(na, factor));
  if (n > 0 && (pos == nullptr || rest_pos == nullptr || rest_count == nullptr || err == nullptr ||
                table_keys == nullptr || table_counts == nullptr || workspace == nullptr ||
                (na > 0 && admitted == nullptr)))
    return fail(CSK_E_INVALID, "route_split: NULL pointer");
  if (n == 0) return CSK_OK;
  CSK_HIP(launch_route_split(pos, n, mesh, factor, admitted, na, table_keys, table_counts, table_slots - 1, rest_pos,
                             (unsigned long long*)rest_count, err, workspace, (hipStream_t)stream),
          "route_split");
  return CSK_OK;
}

namespace {

// Device scratch of one call, freed (after the device is idle) when the call returns.
struct CallScratch {
  std::vector<void*> ptrs;
  ~CallScratch() {
    for (void* q : ptrs) (void)hipFree(q);
  }
  template <typename T>
  hipError_t get(T** p, uint64_t count) {
    hipError_t e = bmalloc(p, count);
    if (e == hipSuccess) ptrs.push_back((void*)*p);
    return e;
  }
};

}  // namespace

csk_status csk_exact_counts(const float* pos, uint64_t n, double delta, double L, uint64_t* table_keys,
                            uint32_t* table_counts, uint32_t table_slots, uint32_t* err, void* stream) {
  Mesh mesh;
  csk_status rc = check_mesh(nullptr, delta, L, &mesh);
  if (rc != CSK_OK) return rc;
  if (table_slots < 2 || table_slots > (1u << 31) || (table_slots & (table_slots - 1)) != 0)
    return fail(CSK_E_INVALID, "exact_counts: table_slots=%u is not a power of two in [2, 2^31]", table_slots);
  if (n >= (1ull << 31)) return fail(CSK_E_INVALID, "exact_counts: n=%llu reaches 2^31", (unsigned long long)n);
  if (n > 0 && (pos == nullptr || table_keys == nullptr || table_counts == nullptr || err == nullptr))
    return fail(CSK_E_INVALID, "exact_counts: NULL pointer");
  if (n == 0) return CSK_OK;
  CSK_HIP(launch_exact_count(pos, n, mesh, table_keys, table_counts, table_slots - 1, err, (hipStream_t)stream),
          "exact_counts");
  return CSK_OK;
}

csk_status csk_table_topk(const uint64_t* table_keys, const uint32_t* table_counts, uint32_t table_slots, uint32_t k,
                          uint64_t* keys, uint32_t* counts, uint32_t* k_out, void* stream) {
  if (k_out == nullptr || table_keys == nullptr || table_counts == nullptr)
    return fail(CSK_E_INVALID, "table_topk: NULL argument");
  *k_out = 0;
  if (table_slots < 2 || table_slots > (1u << 31) || (table_slots & (table_slots - 1)) != 0)
    return fail(CSK_E_INVALID, "table_topk: table_slots=%u is not a power of two in [2, 2^31]", table_slots);
  if (k > (1u << 22)) return fail(CSK_E_INVALID, "table_topk: k=%u above 2^22", k);
  if (k == 0) return CSK_OK;
  if (keys == nullptr || counts == nullptr) return fail(CSK_E_INVALID, "table_topk: NULL output");
  hipStream_t st = (hipStream_t)stream;
  CallScratch cs;
  SelState* sel = nullptr;
  uint64_t* sk = nullptr;
  int32_t* se = nullptr;
  uint32_t* rank = nullptr;
  uint32_t* err = nullptr;
  CSK_HIP(cs.get(&sel, 1), "table_topk: scratch");
  CSK_HIP(cs.get(&sk, k), "table_topk: scratch");
  CSK_HIP(cs.get(&se, k), "table_topk: scratch");
  CSK_HIP(cs.get(&rank, k), "table_topk: scratch");
  CSK_HIP(cs.get(&err, 1), "table_topk: scratch");
  CSK_HIP(launch_fill_u32(err, 1, 0u, st), "table_topk");
  // counts below 2^31 order as int32; empty slots (count 0, key all ones) are never gathered
  CSK_HIP(launch_select_pairs(table_keys, (const int32_t*)table_counts, table_slots, k, sel, sk, se, rank, keys,
                              (int32_t*)counts, err, st),
          "table_topk");
  SelState h;
  CSK_HIP(hipMemcpyAsync(&h, sel, sizeof(SelState), hipMemcpyDeviceToHost, st), "table_topk");
  CSK_HIP(hipStreamSynchronize(st), "table_topk");
  *k_out = h.n_sel < k ? h.n_sel : k;
  return CSK_OK;
}

csk_status csk_cell_list(const uint32_t* counts, uint64_t ncells, uint32_t min_count, const uint32_t* bitmap,
                         uint64_t* cells, uint64_t cap, uint64_t* total, void* stream) {
  if (total == nullptr) return fail(CSK_E_INVALID, "cell_list: total is NULL");
  *total = 0;
  if (ncells > 0 && (counts == nullptr || (cap > 0 && cells == nullptr)))
    return fail(CSK_E_INVALID, "cell_list: NULL pointer");
  if (ncells == 0) return CSK_OK;
  hipStream_t st = (hipStream_t)stream;
  uint64_t chunk = 0;
  const uint32_t nb = cell_list_blocks(ncells, &chunk);   // at least the bitmap path's count
  CallScratch cs;
  uint64_t* blocks = nullptr;
  unsigned long long* dtotal = nullptr;
  CSK_HIP(cs.get(&blocks, nb), "cell_list: scratch");
  CSK_HIP(cs.get(&dtotal, 1), "cell_list: scratch");
  CSK_HIP(launch_cell_list(counts, ncells, min_count, bitmap, blocks, cells, cap, dtotal, st), "cell_list");
  unsigned long long h = 0;
  CSK_HIP(hipMemcpyAsync(&h, dtotal, sizeof(h), hipMemcpyDeviceToHost, st), "cell_list");
  CSK_HIP(hipStreamSynchronize(st), "cell_list");
  *total = h;
  return CSK_OK;
}

csk_status csk_cells_clear(uint32_t* counts, uint32_t* bitmap, uint64_t ncells, void* stream) {
  if (ncells > 0 && (counts == nullptr || bitmap == nullptr)) return fail(CSK_E_INVALID, "cells_clear: NULL pointer");
  if (ncells == 0) return CSK_OK;
  CSK_HIP(launch_bitmap_clear(bitmap, ncells, counts, (hipStream_t)stream), "cells_clear");
  return CSK_OK;
}

csk_status csk_cell_labels(const uint64_t* cells, uint64_t m, const uint64_t* fine_keys, uint32_t nk, double delta,
                           double L, uint32_t factor, float* labels, void* stream) {
  Mesh mesh;
  csk_status rc = check_mesh(nullptr, delta, L, &mesh);
  if (rc != CSK_OK) return rc;
  if (factor < 1 || (uint32_t)mesh.G % factor != 0)
    return fail(CSK_E_INVALID, "cell_labels: factor %u does not divide G=%d", factor, mesh.G);
  if (nk > (1u << 17)) return fail(CSK_E_INVALID, "cell_labels: %u fine keys above 2^17", nk);
  if ((m > 0 && (cells == nullptr || labels == nullptr)) || (nk > 0 && fine_keys == nullptr))
    return fail(CSK_E_INVALID, "cell_labels: NULL pointer");
  if (m == 0) return CSK_OK;
  hipStream_t st = (hipStream_t)stream;
  CallScratch cs;
  uint64_t* tmp = nullptr;
  uint64_t* par = nullptr;
  CSK_HIP(cs.get(&tmp, nk), "cell_labels: scratch");
  CSK_HIP(cs.get(&par, nk), "cell_labels: scratch");
  CSK_HIP(launch_parents_sorted(fine_keys, nk, (uint64_t)mesh.G, factor, tmp, par, st), "cell_labels");
  CSK_HIP(launch_labels(cells, m, par, nk, labels, st), "cell_labels");
  CSK_HIP(hipStreamSynchronize(st), "cell_labels");
  return CSK_OK;
}

csk_status csk_route_admit(const uint64_t* cells, const float* logits, uint64_t m, uint32_t A, uint64_t* admitted,
                           uint32_t* na, void* stream) {
  if (na == nullptr) return fail(CSK_E_INVALID, "route_admit: na is NULL");
  *na = 0;
  if (m >= (1ull << 31)) return fail(CSK_E_INVALID, "route_admit: m=%llu reaches 2^31", (unsigned long long)m);
  if (A > (1u << 16)) return fail(CSK_E_INVALID, "route_admit: A=%u above 2^16", A);
  if (m > 0 && A > 0 && (cells == nullptr || logits == nullptr || admitted == nullptr))
    return fail(CSK_E_INVALID, "route_admit: NULL pointer");
  const uint32_t take = (uint32_t)(m < A ? m : A);
  if (take == 0) return CSK_OK;
  hipStream_t st = (hipStream_t)stream;
  CallScratch cs;
  int32_t* ord = nullptr;
  SelState* sel = nullptr;
  uint64_t *sk = nullptr, *ok = nullptr;
  int32_t *se = nullptr, *oe = nullptr;
  uint32_t *rank = nullptr, *err = nullptr;
  CSK_HIP(cs.get(&ord, m), "route_admit: scratch");
  CSK_HIP(cs.get(&sel, 1), "route_admit: scratch");
  CSK_HIP(cs.get(&sk, take), "route_admit: scratch");
  CSK_HIP(cs.get(&se, take), "route_admit: scratch");
  CSK_HIP(cs.get(&ok, take), "route_admit: scratch");
  CSK_HIP(cs.get(&oe, take), "route_admit: scratch");
  CSK_HIP(cs.get(&rank, take), "route_admit: scratch");
  CSK_HIP(cs.get(&err, 1), "route_admit: scratch");
  CSK_HIP(launch_fill_u32(err, 1, 0u, st), "route_admit");
  CSK_HIP(launch_logit_order(logits, m, ord, st), "route_admit");
  CSK_HIP(launch_select_pairs(cells, ord, (uint32_t)m, take, sel, sk, se, rank, ok, oe, err, st), "route_admit");
  CSK_HIP(launch_rank_sort(ok, take, admitted, st), "route_admit");
  CSK_HIP(hipStreamSynchronize(st), "route_admit");
  *na = take;
  return CSK_OK;
}

csk_status csk_topk_with_table(csk_sketch* s, const uint64_t* table_keys, const uint32_t* table_counts,
                               uint32_t table_slots, uint32_t k, uint64_t* keys, int32_t* est, uint32_t* k_out,
                               void* stream) {
  if (s == nullptr || k_out == nullptr || table_keys == nullptr || table_counts == nullptr)
    return fail(CSK_E_INVALID, "topk_with_table: NULL argument");
  if (table_slots < 2 || (table_slots & (table_slots - 1)) != 0)
    return fail(CSK_E_INVALID, "topk_with_table: table_slots=%u is not a power of two", table_slots);
  *k_out = 0;
  if (k > 0 && (keys == nullptr || est == nullptr)) return fail(CSK_E_INVALID, "topk_with_table: NULL output");
  if (k > s->max_cand) return fail(CSK_E_INVALID, "topk_with_table: k=%u above max_candidates", k);
  hipStream_t st = (hipStream_t)stream;
  CSK_HIP(launch_table_to_set(table_keys, table_slots, s->set, s->slots - 1, s->set_count(), s->max_cand, s->err(), st),
          "topk_with_table");
  if (k > s->sel_cap) {
    CSK_HIP(hipStreamSynchronize(st), "topk_with_table: grow scratch");
    if (s->sel_key) (void)hipFree(s->sel_key);
    if (s->sel_est) (void)hipFree(s->sel_est);
    s->bytes -= (uint64_t)s->sel_cap * (sizeof(uint64_t) + sizeof(int32_t));
    s->sel_key = nullptr;
    s->sel_est = nullptr;
    s->sel_cap = 0;
    CSK_HIP(dmalloc(s, &s->sel_key, k), "topk_with_table: scratch");
    CSK_HIP(dmalloc(s, &s->sel_est, k), "topk_with_table: scratch");
    s->sel_cap = k;
  }
  if (k > 0) {
    CSK_HIP(launch_topk(s->set, s->slots, s->tables(), s->M, s->max_cand, k, s->sel, s->cand_key, s->cand_est,
                        s->sel_key, s->sel_est, keys, est, s->err(), st, table_keys, table_counts, table_slots - 1),
            "topk_with_table");
  }
  CSK_HIP(hipMemcpyAsync(s->host_sel, s->sel, sizeof(SelState), hipMemcpyDeviceToHost, st), "topk_with_table");
  uint32_t bits = 0;
  csk_status rc = take_latch(s, st, &bits);
  if (rc != CSK_OK) return rc;
  rc = latch_status(bits);
  if (rc != CSK_OK) return rc;
  const uint32_t m = k ? s->host_sel->m : 0;
  const uint32_t got = (k < m) ? k : m;
  *k_out = got;
  if (got < k && s->partial_set)
    return fail(CSK_W_INCOMPLETE, "topk_with_table: only %u of %u candidates", got, k);
  return CSK_OK;
}

// ---------------------------------------------------------------- the sync-free routed step

namespace {

uint64_t align256(uint64_t b) { return (b + 255) & ~255ull; }

// Admission scratch: SelState | ord (cap int32) | sk, ok (A uint64) | se, oe, rank (A words) | err.
uint64_t admit_workspace_bytes(uint64_t cap, uint32_t A) {
  return align256(sizeof(SelState)) + align256(cap * 4) + 2 * align256((uint64_t)A * 8) +
         3 * align256((uint64_t)A * 4) + 256;
}

// The most admitted cells an exclusion of this factor and table serves.
uint32_t routed_na_max(uint32_t factor, uint32_t table_slots) {
  const uint64_t f3 = (uint64_t)factor * factor * factor;
  uint64_t na = kMaxAdmitted;
  if (na * f3 > kSplitMaxChildren) na = kSplitMaxChildren / f3;
  if (na * f3 > table_slots / 2) na = (table_slots / 2) / f3;
  return (uint32_t)na;
}

csk_status topk_with_table_impl(csk_sketch* s, const uint64_t* table_keys, const uint32_t* table_counts,
                                uint32_t table_slots, uint32_t k, uint64_t* keys, int32_t* est, uint32_t* out,
                                hipStream_t st, const char* who) {
  if (s == nullptr || out == nullptr || table_keys == nullptr || table_counts == nullptr)
    return fail(CSK_E_INVALID, "%s: NULL argument", who);
  if (table_slots < 2 || (table_slots & (table_slots - 1)) != 0)
    return fail(CSK_E_INVALID, "%s: table_slots=%u is not a power of two", who, table_slots);
  if (k > 0 && (keys == nullptr || est == nullptr)) return fail(CSK_E_INVALID, "%s: NULL output", who);
  if (k > s->max_cand) return fail(CSK_E_INVALID, "%s: k=%u above max_candidates", who, k);
  CSK_HIP(launch_table_to_set(table_keys, table_slots, s->set, s->slots - 1, s->set_count(), s->max_cand, s->err(), st),
          who);
  if (k > s->sel_cap) {   // first call with a larger k: grow the scratch (synchronizes)
    CSK_HIP(hipStreamSynchronize(st), who);
    if (s->sel_key) (void)hipFree(s->sel_key);
    if (s->sel_est) (void)hipFree(s->sel_est);
    s->bytes -= (uint64_t)s->sel_cap * (sizeof(uint64_t) + sizeof(int32_t));
    s->sel_key = nullptr;
    s->sel_est = nullptr;
    s->sel_cap = 0;
    CSK_HIP(dmalloc(s, &s->sel_key, k), who);
    CSK_HIP(dmalloc(s, &s->sel_est, k), who);
    s->sel_cap = k;
  }
  if (k > 0) {
    CSK_HIP(launch_topk(s->set, s->slots, s->tables(), s->M, s->max_cand, k, s->sel, s->cand_key, s->cand_est,
                        s->sel_key, s->sel_est, keys, est, s->err(), st, table_keys, table_counts, table_slots - 1),
            who);
  } else {
    CSK_HIP(launch_fill_u32((uint32_t*)s->sel, sizeof(SelState) / 4, 0u, st), who);
  }
  CSK_HIP(launch_topk_out(s->sel, k, s->partial_set ? 1u : 0u, out, st), who);
  return CSK_OK;
}

}  // namespace

csk_status csk_cell_list_workspace(uint64_t ncells, uint64_t* bytes) {
  if (bytes == nullptr) return fail(CSK_E_INVALID, "cell_list_workspace: bytes is NULL");
  uint64_t chunk = 0;
  *bytes = (uint64_t)cell_list_blocks(ncells, &chunk) * sizeof(uint64_t);
  return CSK_OK;
}

csk_status csk_cell_list_async(const uint32_t* counts, uint64_t ncells, uint32_t min_count, const uint32_t* bitmap,
                               uint64_t* cells, uint64_t cap, uint64_t* total, void* workspace,
                               uint64_t workspace_bytes, void* stream) {
  if (total == nullptr || counts == nullptr || (cap > 0 && cells == nullptr) || workspace == nullptr)
    return fail(CSK_E_INVALID, "cell_list_async: NULL pointer");
  uint64_t chunk = 0;
  const uint64_t need = (uint64_t)cell_list_blocks(ncells, &chunk) * sizeof(uint64_t);
  if (workspace_bytes < need)
    return fail(CSK_E_INVALID, "cell_list_async: workspace of %llu bytes below the %llu needed",
                (unsigned long long)workspace_bytes, (unsigned long long)need);
  hipStream_t st = (hipStream_t)stream;
  if (ncells == 0) {
    CSK_HIP(launch_fill_u32((uint32_t*)total, 2, 0u, st), "cell_list_async");
    return CSK_OK;
  }
  CSK_HIP(launch_cell_list(counts, ncells, min_count, bitmap, (uint64_t*)workspace, cells, cap,
                           (unsigned long long*)total, st),
          "cell_list_async");
  return CSK_OK;
}

csk_status csk_route_score(csk_mlp* m, const uint32_t* counts, double delta_c, double L, const uint64_t* cells,
                           const uint64_t* m_dev, uint64_t cap, float* logits, void* stream) {
  if (m == nullptr) return fail(CSK_E_INVALID, "route_score: NULL model");
  Mesh coarse;
  csk_status rc = check_mesh(nullptr, delta_c, L, &coarse);
  if (rc != CSK_OK) return rc;
  if (cap > 0 && (counts == nullptr || cells == nullptr || m_dev == nullptr || logits == nullptr))
    return fail(CSK_E_INVALID, "route_score: NULL pointer");
  CSK_HIP(launch_route_score(counts, (uint32_t)coarse.G, cells, m_dev, cap, m->p, logits, (hipStream_t)stream),
          "route_score");
  return CSK_OK;
}

csk_status csk_route_admit_workspace(uint64_t cap, uint32_t A, uint64_t* bytes) {
  if (bytes == nullptr) return fail(CSK_E_INVALID, "route_admit_workspace: bytes is NULL");
  *bytes = admit_workspace_bytes(cap, A);
  return CSK_OK;
}

csk_status csk_route_admit_async(const uint64_t* cells, const float* logits, const uint64_t* m, uint64_t cap,
                                 uint32_t A, uint64_t* admitted, uint32_t* na, void* workspace,
                                 uint64_t workspace_bytes, void* stream) {
  if (cap >= (1ull << 31)) return fail(CSK_E_INVALID, "route_admit_async: cap=%llu reaches 2^31", (unsigned long long)cap);
  if (A < 1 || A > (1u << 16)) return fail(CSK_E_INVALID, "route_admit_async: A=%u outside 1..2^16", A);
  if (m == nullptr || na == nullptr || admitted == nullptr || workspace == nullptr ||
      (cap > 0 && (cells == nullptr || logits == nullptr)))
    return fail(CSK_E_INVALID, "route_admit_async: NULL pointer");
  if (workspace_bytes < admit_workspace_bytes(cap, A))
    return fail(CSK_E_INVALID, "route_admit_async: workspace of %llu bytes below the %llu needed",
                (unsigned long long)workspace_bytes, (unsigned long long)admit_workspace_bytes(cap, A));
  uint8_t* w = (uint8_t*)workspace;
  SelState* sel = (SelState*)w;
  w += align256(sizeof(SelState));
  int32_t* ord = (int32_t*)w;
  w += align256(cap * 4);
  uint64_t* sk = (uint64_t*)w;
  w += align256((uint64_t)A * 8);
  uint64_t* ok = (uint64_t*)w;
  w += align256((uint64_t)A * 8);
  int32_t* se = (int32_t*)w;
  w += align256((uint64_t)A * 4);
  int32_t* oe = (int32_t*)w;
  w += align256((uint64_t)A * 4);
  uint32_t* rank = (uint32_t*)w;
  w += align256((uint64_t)A * 4);
  uint32_t* err = (uint32_t*)w;
  hipStream_t st = (hipStream_t)stream;
  CSK_HIP(launch_fill_u32(err, 1, 0u, st), "route_admit_async");
  CSK_HIP(launch_admit_dev(cells, logits, m, cap, A, ord, sel, sk, se, rank, ok, oe, err, admitted, na, st),
          "route_admit_async");
  return CSK_OK;
}

csk_status csk_route_update_workspace(uint32_t factor, uint32_t table_slots, uint64_t* bytes) {
  if (bytes == nullptr) return fail(CSK_E_INVALID, "route_update_workspace: bytes is NULL");
  if (factor < 1 || factor > 32) return fail(CSK_E_INVALID, "route_update_workspace: factor %u outside 1..32", factor);
  *bytes = (uint64_t)routed_na_max(factor, table_slots) * factor * factor * factor * sizeof(uint32_t);
  return CSK_OK;
}

csk_status csk_sketch_update_routed(csk_sketch* s, const float* pos, uint64_t n, double delta, double L,
                                    uint32_t factor, const uint64_t* admitted, const uint32_t* na,
                                    uint64_t* table_keys, uint32_t* table_counts, uint32_t table_slots, uint32_t* err,
                                    void* workspace, uint64_t workspace_bytes, void* stream) {
  if (s == nullptr) return fail(CSK_E_INVALID, "update_routed: NULL handle");
  Mesh mesh;
  csk_status rc = check_mesh(s, delta, L, &mesh);
  if (rc != CSK_OK) return rc;
  if (mesh.group != 1u) return fail(CSK_E_INVALID, "update_routed: the sketch counts groups of cells");
  if (factor < 1 || factor > 32 || (uint32_t)mesh.G % factor != 0)
    return fail(CSK_E_INVALID, "update_routed: factor %u does not divide G=%d", factor, mesh.G);
  if (table_slots < 2 || (table_slots & (table_slots - 1)) != 0)
    return fail(CSK_E_INVALID, "update_routed: table_slots=%u is not a power of two", table_slots);
  const uint32_t f3 = factor * factor * factor;
  const uint32_t na_max = routed_na_max(factor, table_slots);
  if (na_max < 1) return fail(CSK_E_INVALID, "update_routed: a table of %u slots takes no %u^3 cell", table_slots, factor);
  if (workspace_bytes < (uint64_t)na_max * f3 * sizeof(uint32_t))
    return fail(CSK_E_INVALID, "update_routed: workspace of %llu bytes below the %llu needed",
                (unsigned long long)workspace_bytes, (unsigned long long)na_max * f3 * sizeof(uint32_t));
  if (n > (1ull << 40)) return fail(CSK_E_INVALID, "update_routed: n above 2^40");
  if ((n > 0 && pos == nullptr) || admitted == nullptr || na == nullptr || table_keys == nullptr ||
      table_counts == nullptr || err == nullptr || workspace == nullptr)
    return fail(CSK_E_INVALID, "update_routed: NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  const Tables t = s->tables();
  RouteExclude ex;
  ex.admitted = admitted;
  ex.na = na;
  ex.na_max = na_max;
  ex.factor = factor;
  ex.fmagic = (uint32_t)(((1ull << 32) + factor - 1) / factor);
  ex.f3 = f3;
  ex.gc = (uint32_t)mesh.G / factor;
  ex.child = (uint32_t*)workspace;
  ex.err = err;
  latch_mesh(s, delta, L, mesh);
  CSK_HIP(launch_fill_u32(ex.child, (uint64_t)na_max * f3, 0u, st), "update_routed");
  const uint64_t piece_max = 1ull << 30;
  for (uint64_t off = 0; off < n; off += piece_max) {
    const uint64_t m = (n - off < piece_max) ? n - off : piece_max;
    const float* p = pos + 3 * off;
    BinPlan plan;
    bool binned = s->upd_mode != CSK_UPDATE_DIRECT && s->d == 5 &&
                  plan_bin_wg(m, s->d, s->w, bin_wg_cap(s->d, s->upd_max_wg), plan) && plan.fast;
    bool sorted = false;
    if (binned) {
      // the sort-word kernel on the row tables (two rows per pass beside the exclusion's
      // table) when the handle's tiling asks for it: at 2^22 - 39 322 counters per row it
      // took 3.96 ms per 2^28 particles against 3.81 for the general kernel, which is the
      // default: two rows per LDS pass, or three when the handle's tiling asks and they fit
      // (two measured 5.31 ms against 5.68 there: three spill registers)
      const uint32_t lds_s = sortbin_lds_bytes(5, 2, plan.Pr, plan.P, true, mesh.nch, true);
      sorted = s->upd_form == kFormSortWord && plan.Pr <= 512 && t.tabi != nullptr && lds_s <= kMaxLds;
      if (sorted) {
        plan.sort = kSortRows;
        plan.rp = 2u;
        plan.nt = kBin2Threads;
        plan.pf = 0u;
        plan.lds_bytes = lds_s;
      } else {
        const uint32_t lds3 = bin3_lds_bytes(plan, s->d, 3, true);
        const bool three = s->upd_rp == 3 && lds3 <= kMaxLds;
        plan.rp = three ? 3u : 2u;
        plan.lds_bytes = three ? lds3 : bin3_lds_bytes(plan, s->d, 2, true);
        binned = plan.lds_bytes <= kMaxLds;
      }
    }
    if (!binned) {
      CSK_HIP(launch_update_direct_routed(p, m, mesh, t, s->M, s->err(), ex, st), "update_routed (direct)");
      continue;
    }
    CSK_HIP(ensure_update_scratch(s, plan, st), "update_routed: token scratch");
    if (sorted) {
      BinArgs a = make_bin_args(p, m, mesh, t, plan, s->tok, s->cnt, s->M, s->err());
      a.ex = ex;
      CSK_HIP(launch_sortbin_routed(a, mesh.mode, st), "update_routed (bin)");
    } else {
      CSK_HIP(launch_bin_routed(p, m, mesh, t, plan, s->tok, s->cnt, s->M, s->err(), ex, st), "update_routed (bin)");
    }
    CSK_HIP(launch_accumulate(s->tok, s->cnt, plan, s->w, s->M, st), "update_routed (accumulate)");
  }
  CSK_HIP(launch_route_table(ex, (uint32_t)mesh.G, table_keys, table_counts, table_slots - 1, err, st),
          "update_routed (table)");
  return CSK_OK;
}

csk_status csk_topk_with_table_async(csk_sketch* s, const uint64_t* table_keys, const uint32_t* table_counts,
                                     uint32_t table_slots, uint32_t k, uint64_t* keys, int32_t* est, uint32_t* out,
                                     void* stream) {
  return topk_with_table_impl(s, table_keys, table_counts, table_slots, k, keys, est, out, (hipStream_t)stream,
                              "topk_with_table_async");
}
