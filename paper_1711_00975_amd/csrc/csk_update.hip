// csk_update.hip — the update (Sec. 2.2 Add; Alg. 4 Update; Sec. 3.1 stages 1-3) on gfx950,
// in two kernels:
//   bin         one pass over the positions: exact cell key, d tabulated row words, and a
//               16-bit token (15-bit counter offset + sign) per row, counting-sorted in LDS
//               by counter slice (2^15 counters) and appended as coalesced runs to a
//               per-(slice, workgroup) region.  No global atomics on the hot path.
//   accumulate  one workgroup per slice: sums the slice's tokens into an LDS copy of the
//               slice with LDS atomics, then adds it to the counters with a plain
//               read-modify-write (the workgroup owns the slice).
// and a one-atomic-per-row direct update for short streams.  The bin plan (workgroups,
// slices, token capacity) is chosen here too.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csk_kernel_util.h"

namespace csk {

// ------------------------------------------------------------------ bin


// LDS layout (uint32 words): tables [tab_rows_lds * 1536] | cursor [P] | hist [Pr] |
// base [Pr] | stage [tile] | wsum [NW + 1].
template <bool TAB_LDS>
__global__ __launch_bounds__(kBinThreads) void bin_kernel(BinArgs a) {
  extern __shared__ uint32_t lds[];
  const BinPlan& pl = a.plan;
  uint32_t* tabs = lds;
  uint32_t* cursor = tabs + pl.tab_rows_lds * kTableWords;
  uint32_t* hist = cursor + pl.P;
  uint32_t* base = hist + pl.Pr;
  uint32_t* stage = base + pl.Pr;
  uint32_t* wsum = stage + kBinTile;
  uint32_t* total = wsum + kBinThreads / 64;
  const uint32_t tid = threadIdx.x;
  const uint32_t g = blockIdx.x;

  if (TAB_LDS) load_tables(tabs, a.tab, pl.tab_rows_lds);
  for (uint32_t i = tid; i < pl.P; i += kBinThreads) cursor[i] = 0;
  __syncthreads();

  for (uint64_t tile = g; tile < pl.ntiles; tile += pl.nwg) {
    const uint64_t first = tile * (uint64_t)kBinTile;
    uint64_t key[kBinPPT];
    uint32_t valid = 0;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < kBinPPT; ++j) {
      const uint64_t i = first + (uint64_t)j * kBinThreads + tid;
      key[j] = 0;
      if (i < a.n) {
        if (particle_key(a.pos, i, a.mesh, key[j])) valid |= 1u << j;
        else bad = true;
      }
    }
    if (bad) atomicOr(a.err, kErrDomain);

    for (uint32_t r = 0; r < a.d; ++r) {
      const uint32_t* tab_r = TAB_LDS ? tabs + r * kTableWords : a.tab + r * kTableWords;
      for (uint32_t b = tid; b < pl.Pr; b += kBinThreads) hist[b] = 0;
      __syncthreads();
      uint32_t sv[kBinPPT], rk[kBinPPT];
#pragma unroll
      for (int j = 0; j < kBinPPT; ++j) {
        sv[j] = 0;
        rk[j] = 0;
        if (valid & (1u << j)) {
          const uint32_t h = row_hash(tab_r, key[j]);
          const uint32_t b = bucket_of(h, a.w);
          const uint32_t neg = (h >> 31) & (a.cm ^ 1u);
          const uint32_t sl = b >> kSliceBits;
          sv[j] = (sl << 16) | (b & (kSlice - 1)) | (neg << 15);
          rk[j] = atomicAdd(&hist[sl], 1u);
        }
      }
      __syncthreads();
      block_exclusive_scan<kBinThreads>(hist, base, pl.Pr, wsum, total);
#pragma unroll
      for (int j = 0; j < kBinPPT; ++j) {
        if (valid & (1u << j)) stage[base[sv[j] >> 16] + rk[j]] = sv[j];
      }
      __syncthreads();
      const uint32_t ntok = *total;
      const uint64_t region_row = (uint64_t)r * pl.Pr;
      for (uint32_t q = tid; q < ntok; q += kBinThreads) {
        const uint32_t v = stage[q];
        const uint32_t sl = v >> 16;
        const uint32_t c = cursor[region_row + sl] + (q - base[sl]);
        if (c < pl.cap) {
          a.tok[((uint64_t)g * pl.P + region_row + sl) * (uint64_t)pl.cap + c] = (uint16_t)(v & 0xFFFFu);
        } else {
          // region full: add this one update straight to the counter (rare; same sum)
          const uint32_t bkt = (sl << kSliceBits) | (v & (kSlice - 1));
          atomicAdd(&a.M[(uint64_t)r * a.w + bkt], (v & 0x8000u) ? -1 : 1);
        }
      }
      __syncthreads();
      for (uint32_t b = tid; b < pl.Pr; b += kBinThreads) cursor[region_row + b] += hist[b];
      __syncthreads();
    }
  }
  for (uint32_t s = tid; s < pl.P; s += kBinThreads) a.cnt[(uint64_t)s * pl.nwg + g] = cursor[s];
}


// ------------------------------------------------------------------ bin (d <= 8)

// Row-interleaved variant for d <= 8 (MODE: how the mesh computes its floor).  Every row
// word of a particle comes from one pass over the key bytes; all d tokens of a tile stay
// in registers; rows are counting-sorted in LDS two at a time (bin = row-in-pass * Pr +
// slice) while the previous pass's runs are written out.  Tokens of particles outside
// the stream or the domain go to a dummy bin that is never written.  A run that would
// overflow its region goes to the counters through atomics instead (same sum).
// Token scratch is workgroup-major: region (g, s) starts at (g * P + s) * cap.
// LDS layout (words): [EX: the exclusion's table, kExLdsWords] | Ti [1536 * DP] | dst [RP*Pr + 1] |
// cursor [P] | hist [RP*Pr + 1] | base [RP*Pr + 1] | stage [RP * tile] | wsum [NW].
// EX (the learned router's rest sketch): a particle in an admitted coarse cell is counted in
// the exclusion's child counters and goes to the dummy bin instead of the sketch.
constexpr uint32_t kDstDrop = 0xFFFFFFFFu;      // dummy bin: never written
constexpr uint32_t kDstOverflow = 0xFFFFFFFEu;  // run added with atomics
constexpr uint32_t kDstBias = 1u << 16;         // keeps offset + cursor - base positive

template <int D, uint32_t MODE, int NT, int RP, int HM, int KB, bool EX = false>
__device__ __forceinline__ void bin3_body(const BinArgs* __restrict__ ap, const float* __restrict__ pos, uint64_t n,
                                          uint32_t g) {
  const BinArgs& a = *ap;   // read in place (argument segment or descriptor), not copied
  constexpr int DP = HashWords<D, HM>::value;
  constexpr int PPT = bin2_ppt(D), TILE = NT * PPT, NW = NT / 64;
  extern __shared__ __align__(16) uint32_t lds2[];
  const BinPlan& pl = a.plan;
  const uint32_t nbins = RP * pl.Pr + 1;                 // + the dummy bin
  const uint32_t dummy = nbins - 1;
  const ExLds ext = ex_lds(lds2);                                   // EX only
  uint32_t* ti = lds2 + (EX ? kExLdsWords : 0);
  uint32_t* dst = ti + kTableWords * DP;
  uint32_t* cursor = dst + nbins;
  uint32_t* hist = cursor + pl.P;
  uint32_t* base = hist + nbins;
  uint32_t* stage = base + nbins;
  uint32_t* wsum = stage + RP * TILE;
  const uint32_t tid = threadIdx.x, wave = tid >> 6;
  uint16_t* __restrict__ tokg = a.tok + (uint64_t)g * pl.P * pl.cap;   // this workgroup's regions

  for (uint32_t i = tid; i < pl.P; i += NT) cursor[i] = 0;
  for (uint32_t i = tid; i < nbins; i += NT) hist[i] = 0;
  stage_tables<DP>(ti, HM == kHashPacked ? a.tabp : a.tabi, (uint32_t)KB);   // fold point KB >= nch
  if constexpr (EX) ex_fill(a.ex.admitted, adm_count(a.ex), ext);   // ends with a barrier

  const uint32_t per = (nbins + NT - 1) / NT;           // scan: bins per thread
  const uint32_t blo = min(nbins, tid * per), bhi = min(nbins, blo + per);
  bool pending = false;                                  // a sorted pass waits in stage
  uint32_t pend_row0 = 0, pend_total = 0;

  auto write_out = [&]() {
    for (uint32_t q = tid; q < pend_total; q += NT) {
      const uint32_t v = stage[q];
      const uint32_t dq = dst[v >> 16];
      if (dq < kDstOverflow) {
        tokg[dq - kDstBias + q] = (uint16_t)(v & 0xFFFFu);
      } else if (dq == kDstOverflow) {
        // region full: add this one update straight to the counter (rare; same sum)
        const uint32_t bin = v >> 16;
        const uint32_t r = pend_row0 + bin / pl.Pr, sl = bin % pl.Pr;
        const uint32_t bkt = (sl << kSliceBits) | (v & (kSlice - 1));
        atomicAdd(&a.M[(uint64_t)r * a.w + bkt], (v & 0x8000u) ? -1 : 1);
      }
    }
  };

  const uint64_t ntiles = (n + TILE - 1) / TILE;
  for (uint64_t tile = g; tile < ntiles; tile += pl.nwg) {
    const uint64_t first = tile * (uint64_t)TILE;
    const bool full = first + TILE <= n;
    // all PPT position loads are issued before any is used (a clamped index keeps the
    // loads unconditional; particles beyond the stream are masked below)
    float px[PPT], py[PPT], pz[PPT];
    uint64_t pw[PPT];
    const uint64_t last = n - 1;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      uint64_t i = first + (uint64_t)j * NT + tid;
      i = i < last ? i : last;
      if constexpr (MODE == kMeshPacked) {
        pw[j] = __builtin_nontemporal_load((const uint64_t*)pos + i);
      } else {
        px[j] = __builtin_nontemporal_load(pos + 3 * i);
        py[j] = __builtin_nontemporal_load(pos + 3 * i + 1);
        pz[j] = __builtin_nontemporal_load(pos + 3 * i + 2);
      }
    }
    // sv = (bin in its sort pass) << 16 | token; bin = (row % RP) * Pr + slice, or the dummy
    // bin for a particle outside the stream or the domain
    uint32_t sv[D][PPT];
    uint32_t valid = 0, inside = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const bool in = full || (first + (uint64_t)j * NT + tid) < n;
      uint64_t key;   // always a key of the mesh, so the table lookups stay in range
      bool ok;
      if constexpr (EX) {
        static_assert(MODE != kMeshPacked, "the exclusion reads float positions");
        int32_t ix, iy, iz;
        ok = ((int)cell_index_m<MODE>(px[j], a.mesh, ix) & (int)cell_index_m<MODE>(py[j], a.mesh, iy) &
              (int)cell_index_m<MODE>(pz[j], a.mesh, iz)) && in;
        key = ((uint64_t)((uint32_t)ix * (uint32_t)a.mesh.G + (uint32_t)iy)) * (uint64_t)(uint32_t)a.mesh.G +
              (uint64_t)(uint32_t)iz;   // ungrouped: the caller checks
        valid |= (uint32_t)ok << j;
        if (ok) {
          uint32_t child;
          const int32_t c = ex_find(adm_coarse(ix, iy, iz, a.ex, child), ext);
          if (c >= 0) {
            atomicAdd(&a.ex.child[(uint32_t)c * a.ex.f3 + child], 1u);
            ok = false;   // counted exactly; its tokens go to the dummy bin
          }
        }
      } else {
        if constexpr (MODE == kMeshPacked) ok = packed_key(pw[j], a.mesh, key) && in;
        else ok = cell_key_m<MODE>(px[j], py[j], pz[j], a.mesh, key) && in;
        valid |= (uint32_t)ok << j;
      }
      inside |= (uint32_t)in << j;
      uint32_t bk[D], sg[D];
      rows_bucket_sign_kb<D, HM, KB>(ti, key, a.w, a.wshift, bk, sg);
#pragma unroll
      for (int r = 0; r < D; ++r) {
        const uint32_t b = bk[r];
        const uint32_t neg = sg[r] & (a.cm ^ 1u);
        const uint32_t bin = (uint32_t)(r % RP) * pl.Pr + (b >> kSliceBits);
        sv[r][j] = ok ? ((bin << 16) | (b & (kSlice - 1)) | (neg << 15)) : (dummy << 16);
      }
    }
    // particles of the stream that are outside the domain latch the error
    if (inside & ~valid) atomicOr(a.err, kErrDomain);

#pragma unroll
    for (int r0 = 0; r0 < D; r0 += RP) {
      const int nr = (D - r0 < RP) ? D - r0 : RP;
      if (pending) write_out();
      static_assert(RP >= 1 && RP <= 4 && RP * TILE <= 65536, "ranks are packed two per word");
      // rank of row r0 + q: low half of rk[q / 2] for even q, high half for odd q
      uint32_t rk[(RP + 1) / 2][PPT];
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
#pragma unroll
        for (int q = 0; q < RP; ++q) {
          if (q < nr) {
            const uint32_t x = atomicAdd(&hist[sv[(r0 + q < D) ? r0 + q : r0][j] >> 16], 1u);
            if (q & 1) rk[q >> 1][j] |= x << 16;
            else rk[q >> 1][j] = x;
          }
        }
      }
      __syncthreads();  // counts complete; the previous pass is written out
      uint32_t cnt_local = 0;
      for (uint32_t b = blo; b < bhi; ++b) cnt_local += hist[b];
      const uint32_t incl = wave_incl_scan(cnt_local);
      if ((tid & 63u) == 63u) wsum[wave] = incl;
      __syncthreads();
      uint32_t run = incl - cnt_local, total = 0;
      for (int w2 = 0; w2 < NW; ++w2) {
        const uint32_t x = wsum[w2];
        if (w2 < (int)wave) run += x;
        total += x;
      }
      const uint32_t slice0 = (uint32_t)r0 * pl.Pr;
      for (uint32_t b = blo; b < bhi; ++b) {
        const uint32_t hb = hist[b];
        hist[b] = 0;
        base[b] = run;
        if (b < (uint32_t)nr * pl.Pr) {
          const uint32_t cur = cursor[slice0 + b];
          if (cur + hb <= pl.cap) {
            dst[b] = (slice0 + b) * pl.cap + cur + kDstBias - run;
            cursor[slice0 + b] = cur + hb;
          } else {
            dst[b] = kDstOverflow;
          }
        } else {
          dst[b] = kDstDrop;   // the dummy bin (and unused row bins of the last pass)
        }
        run += hb;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
#pragma unroll
        for (int q = 0; q < RP; ++q) {
          if (q < nr) {
            const uint32_t v = sv[(r0 + q < D) ? r0 + q : r0][j];
            const uint32_t r = (q & 1) ? (rk[q >> 1][j] >> 16) : (rk[q >> 1][j] & 0xFFFFu);
            stage[base[v >> 16] + r] = v;
          }
        }
      }
      __syncthreads();
      pending = true;
      pend_row0 = (uint32_t)r0;
      pend_total = total;
    }
  }
  if (pending) write_out();
  for (uint32_t s = tid; s < pl.P; s += NT) a.cnt[(uint64_t)s * pl.nwg + g] = cursor[s];
}

template <int D, uint32_t MODE, int NT, int RP, int HM, int KB>
__global__ __launch_bounds__(NT) void bin3_kernel(BinArgs a) {
  bin3_body<D, MODE, NT, RP, HM, KB>(&a, a.pos, a.n, blockIdx.x);
}

template <int D, uint32_t MODE, int NT, int RP, int HM>
__global__ __launch_bounds__(NT) void bin3_ex_kernel(BinArgs a) {
  bin3_body<D, MODE, NT, RP, HM, kChars, true>(&a, a.pos, a.n, blockIdx.x);
}

// Many sketches in one launch: workgroup blockIdx.x serves sketch wg_sketch[blockIdx.x] as
// its workgroup blockIdx.x - wg_first[sketch]; the per-call stream of each sketch comes in
// `call`, the rest of its arguments from descs.
template <int D, uint32_t MODE, int NT, int RP, int HM, int KB>
__global__ __launch_bounds__(NT) void bin3_batch_kernel(const BinArgs* __restrict__ descs,
                                                        const uint16_t* __restrict__ wg_sketch,
                                                        const uint32_t* __restrict__ wg_first, BatchCall call) {
  const uint32_t i = wg_sketch[blockIdx.x];
  bin3_body<D, MODE, NT, RP, HM, KB>(descs + i, call.pos[i], call.n[i], blockIdx.x - wg_first[i]);
}

bool plan_bin(uint64_t n, uint32_t d, uint32_t w, BinPlan& p) {
  return plan_bin_wg(n, d, w, (d <= (uint32_t)kTabLdsRows) ? 256u : 512u, p);
}

bool plan_bin_wg(uint64_t n, uint32_t d, uint32_t w, uint64_t max_wg, BinPlan& p) {
  p.Pr = (w + kSlice - 1) / kSlice;
  p.P = d * p.Pr;
  p.fast = (d <= (uint32_t)kTabLdsRows) ? 1u : 0u;
  p.tile = p.fast ? kBin2Threads * bin2_ppt((int)d) : kBinTile;
  p.ntiles = (n + p.tile - 1) / p.tile;
  if (p.Pr > kMaxSlicesPerRow || p.ntiles == 0) return false;
  uint64_t words;
  if (p.fast) {
    const uint32_t dp = (d <= 4) ? 4u : (d <= 6 ? 6u : 8u);
    p.tab_rows_lds = 0;
    const uint64_t nb = (uint64_t)kBin2Rows * p.Pr + 1;
    words = (uint64_t)kTableWords * dp + nb + p.P + 2 * nb + (uint64_t)kBin2Rows * p.tile + kBin2Threads / 64;
  } else {
    p.tab_rows_lds = 0;
    words = (uint64_t)p.P + 2ull * p.Pr + kBinTile + kBinThreads / 64 + 1;
  }
  if (words * 4 > kMaxLds) return false;
  p.lds_bytes = (uint32_t)(words * 4);
  if (max_wg < 1) max_wg = 1;
  p.nwg = (uint32_t)(p.ntiles < max_wg ? p.ntiles : max_wg);
  const uint64_t tiles_per_wg = (p.ntiles + p.nwg - 1) / p.nwg;
  const uint64_t per_wg = tiles_per_wg * p.tile;     // most particles one workgroup sees
  // a full slice holds 2^15 of the w buckets of its row: mean tokens = per_wg * 2^15 / w
  const uint64_t span = (w < kSlice) ? w : kSlice;
  uint64_t cap = (per_wg * span * 13 + (uint64_t)w * 10 - 1) / ((uint64_t)w * 10) + 64;  // 1.3x mean + 64
  if (cap > per_wg) cap = per_wg;                    // a region never gets more than this
  cap = (cap + 7) & ~7ull;
  if ((uint64_t)p.P * cap + kDstBias >= 0x7FFFFFFFull) return false;   // 32-bit region offsets
  p.cap = (uint32_t)cap;
  p.sort = 0;
  p.rp = kBin2Rows;
  p.pf = 0;
  p.nt = kBin2Threads;
  return true;
}

bool plan_sortbin(BinPlan& p, uint32_t d, const Mesh& mesh, const Tables& t, uint32_t form, uint32_t want_nt,
                  uint32_t want_rp, uint32_t want_pf, bool rows_ok) {
  p.sort = 0;
  const bool packed = t.tabs != nullptr;
  const bool rows = !packed && rows_ok && t.tabi != nullptr;
  if (form == kFormGeneral || (!packed && !rows) || !p.fast || d < 5 || d > 8 || p.Pr > 512 ||
      mesh.mode == kMeshPacked || mesh.group != 1u)
    return false;
  if (want_nt != 0 && want_nt != 512 && want_nt != 1024) return false;
  if (want_rp != 0 && want_rp != 2 && want_rp != 3) return false;
  if (want_pf > 2 || (want_pf == 2 && want_nt == 1024)) return false;
  if (want_nt == 512 && d != 5) return false;   // the 512-thread forms are compiled for d = 5
  if (want_nt == 512 && want_rp == 2 && want_pf == 1) return false;   // not compiled
  if (rows && (want_nt == 512 || want_pf == 2)) return false;         // 1024 threads only
  // automatic: the sort-word kernel from 32 slices per row (w >= 2^20) on.  Narrower rows
  // have few bins per pass, and its two LDS atomics per token (count, then scatter) then
  // contend on the same few words: at w = 2^16 it measured 59 us per 2^20 particles
  // against 46 us for the general kernel, at w = 2^22 3.24 against 3.64 ms per 2^28.
  if (form == kFormAuto && p.Pr < 32) return false;
  // automatic, row tables: from d = 6 on.  Per 2^28 particles of the 2^30-particle stream's
  // recipe, d = 5 at w = 2^22 - 39 322 took 3.75 ms against 3.71 for the general kernel,
  // d = 6 at w = 2^21 4.34 against 4.42, d = 8 at w = 2^22 - 3 5.53 against 9.62.
  if (form == kFormAuto && rows && d == 5) return false;
  uint32_t rp = want_rp ? want_rp : 3u;
  if (want_rp == 0 && sortbin_lds_bytes(d, rp, p.Pr, p.P, rows, mesh.nch, false) > kMaxLds) rp = 2u;
  const uint32_t lds = sortbin_lds_bytes(d, rp, p.Pr, p.P, rows, mesh.nch, false);
  if (lds > kMaxLds) return false;
  const uint32_t nt = want_nt ? want_nt : (want_pf == 2 ? 512u : 1024u);
  p.sort = rows ? kSortRows : kSortPacked;
  p.nt = nt;
  p.rp = rp;
  p.pf = (nt == 512 && want_pf != 1) ? 1u : 0u;
  p.lds_bytes = lds;
  return true;
}

// Key bytes hashed: d = 5 with packed fields looks up exactly those its mesh needs (5 below
// 2^40, else 6); every other form looks up all six.
template <int D, uint32_t MM>
static void launch_bin3_m(int hm, dim3 grid, dim3 block, uint32_t lds, hipStream_t s, const BinArgs& a) {
  if constexpr (D >= 5) {
    if (hm == kHashPacked) {
      if (D == 5 && key_bytes_kb(a.mesh.nch) == 5)
        hipLaunchKernelGGL((bin3_kernel<D, MM, kBin2Threads, kBin2Rows, kHashPacked, 5>), grid, block, lds, s, a);
      else
        hipLaunchKernelGGL((bin3_kernel<D, MM, kBin2Threads, kBin2Rows, kHashPacked, kChars>), grid, block, lds, s, a);
      return;
    }
  }
  if (hm == kHashMulHi)
    hipLaunchKernelGGL((bin3_kernel<D, MM, kBin2Threads, kBin2Rows, kHashMulHi, kChars>), grid, block, lds, s, a);
  else
    hipLaunchKernelGGL((bin3_kernel<D, MM, kBin2Threads, kBin2Rows, kHashShift, kChars>), grid, block, lds, s, a);
}

template <int D>
static void launch_bin3_dm(uint32_t mode, int hm, dim3 grid, dim3 block, uint32_t lds, hipStream_t s,
                           const BinArgs& a) {
  if (mode == kMeshPacked) launch_bin3_m<D, kMeshPacked>(hm, grid, block, lds, s, a);
  else if (mode == kMeshPow2Ratio) launch_bin3_m<D, kMeshPow2Ratio>(hm, grid, block, lds, s, a);
  else if (mode == kMeshExactRatio) launch_bin3_m<D, kMeshExactRatio>(hm, grid, block, lds, s, a);
  else launch_bin3_m<D, kMeshGeneral>(hm, grid, block, lds, s, a);
}

static void launch_bin3_d(uint32_t d, uint32_t mode, int hm, dim3 grid, dim3 block, uint32_t lds, hipStream_t s,
                          const BinArgs& a) {
  switch (d) {
    case 1: launch_bin3_dm<1>(mode, hm, grid, block, lds, s, a); break;
    case 2: launch_bin3_dm<2>(mode, hm, grid, block, lds, s, a); break;
    case 3: launch_bin3_dm<3>(mode, hm, grid, block, lds, s, a); break;
    case 4: launch_bin3_dm<4>(mode, hm, grid, block, lds, s, a); break;
    case 5: launch_bin3_dm<5>(mode, hm, grid, block, lds, s, a); break;
    case 6: launch_bin3_dm<6>(mode, hm, grid, block, lds, s, a); break;
    case 7: launch_bin3_dm<7>(mode, hm, grid, block, lds, s, a); break;
    default: launch_bin3_dm<8>(mode, hm, grid, block, lds, s, a); break;
  }
}

BinArgs make_bin_args(const float* pos, uint64_t n, const Mesh& mesh, const Tables& t, const BinPlan& plan,
                      uint16_t* tok, uint32_t* cnt, int32_t* M, uint32_t* err) {
  BinArgs a;
  a.pos = pos;
  a.n = n;
  a.mesh = mesh;
  a.tab = t.tab;
  a.tabi = t.tabi;
  a.tabp = t.tabp;
  a.tabs = t.tabs;
  a.d = t.d;
  a.w = t.w;
  a.wshift = t.wshift;
  a.cm = t.cm;
  a.plan = plan;
  a.tok = tok;
  a.cnt = cnt;
  a.M = M;
  a.err = err;
  a.ex = RouteExclude{};
  return a;
}

template <int D, uint32_t MM, int HM>
static void launch_bin3_batch_one(dim3 grid, uint32_t lds, hipStream_t s, const BinArgs* descs,
                                  const uint16_t* wg_sketch, const uint32_t* wg_first, const BatchCall& call) {
  // a batch hashes all six key bytes (its meshes may need different counts)
  hipLaunchKernelGGL((bin3_batch_kernel<D, MM, kBin2Threads, kBin2Rows, HM, kChars>), grid, dim3(kBin2Threads), lds,
                     s, descs, wg_sketch, wg_first, call);
}

template <int D, uint32_t MM>
static void launch_bin3_batch_m(int hm, dim3 grid, uint32_t lds, hipStream_t s, const BinArgs* descs,
                                const uint16_t* wg_sketch, const uint32_t* wg_first, const BatchCall& call) {
  if constexpr (D >= 5) {
    if (hm == kHashPacked) {
      launch_bin3_batch_one<D, MM, kHashPacked>(grid, lds, s, descs, wg_sketch, wg_first, call);
      return;
    }
  }
  if (hm == kHashMulHi) launch_bin3_batch_one<D, MM, kHashMulHi>(grid, lds, s, descs, wg_sketch, wg_first, call);
  else launch_bin3_batch_one<D, MM, kHashShift>(grid, lds, s, descs, wg_sketch, wg_first, call);
}

template <int D>
static void launch_bin3_batch_d(uint32_t mode, int hm, dim3 grid, uint32_t lds, hipStream_t s, const BinArgs* descs,
                                const uint16_t* wg_sketch, const uint32_t* wg_first, const BatchCall& call) {
  if (mode == kMeshPow2Ratio) launch_bin3_batch_m<D, kMeshPow2Ratio>(hm, grid, lds, s, descs, wg_sketch, wg_first, call);
  else if (mode == kMeshExactRatio)
    launch_bin3_batch_m<D, kMeshExactRatio>(hm, grid, lds, s, descs, wg_sketch, wg_first, call);
  else launch_bin3_batch_m<D, kMeshGeneral>(hm, grid, lds, s, descs, wg_sketch, wg_first, call);
}

hipError_t launch_bin_batch(const BinArgs* descs, const uint16_t* wg_sketch, const uint32_t* wg_first,
                            uint32_t nwg_total, uint32_t lds_bytes, uint32_t d, uint32_t mode, int hm,
                            const BatchCall& call, hipStream_t s) {
  const dim3 grid(nwg_total);
  switch (d) {
    case 1: launch_bin3_batch_d<1>(mode, hm, grid, lds_bytes, s, descs, wg_sketch, wg_first, call); break;
    case 2: launch_bin3_batch_d<2>(mode, hm, grid, lds_bytes, s, descs, wg_sketch, wg_first, call); break;
    case 3: launch_bin3_batch_d<3>(mode, hm, grid, lds_bytes, s, descs, wg_sketch, wg_first, call); break;
    case 4: launch_bin3_batch_d<4>(mode, hm, grid, lds_bytes, s, descs, wg_sketch, wg_first, call); break;
    case 5: launch_bin3_batch_d<5>(mode, hm, grid, lds_bytes, s, descs, wg_sketch, wg_first, call); break;
    case 6: launch_bin3_batch_d<6>(mode, hm, grid, lds_bytes, s, descs, wg_sketch, wg_first, call); break;
    case 7: launch_bin3_batch_d<7>(mode, hm, grid, lds_bytes, s, descs, wg_sketch, wg_first, call); break;
    default: launch_bin3_batch_d<8>(mode, hm, grid, lds_bytes, s, descs, wg_sketch, wg_first, call); break;
  }
  return hipGetLastError();
}

hipError_t launch_bin(const float* pos, uint64_t n, const Mesh& mesh, const Tables& t, const BinPlan& plan,
                      uint16_t* tok, uint32_t* cnt, int32_t* M, uint32_t* err, hipStream_t s) {
  const BinArgs a = make_bin_args(pos, n, mesh, t, plan, tok, cnt, M, err);
  if (plan.sort) return launch_sortbin(a, mesh.mode, s);
  if (plan.fast) {
    const dim3 grid(plan.nwg), block(kBin2Threads);
    launch_bin3_d(t.d, mesh.mode, t.hash_mode(), grid, block, plan.lds_bytes, s, a);
  } else {
    hipLaunchKernelGGL(bin_kernel<false>, dim3(plan.nwg), dim3(kBinThreads), plan.lds_bytes, s, a);
  }
  return hipGetLastError();
}

// The general bin kernel with the router's exclusion (d = 5, float positions, ungrouped
// mesh; the plan's LDS includes kExLdsWords).
template <uint32_t MM, int RP>
static void launch_bin3_ex_mr(int hm, dim3 grid, dim3 block, uint32_t lds, hipStream_t s, const BinArgs& a) {
  if (hm == kHashPacked)
    hipLaunchKernelGGL((bin3_ex_kernel<5, MM, kBin2Threads, RP, kHashPacked>), grid, block, lds, s, a);
  else if (hm == kHashMulHi)
    hipLaunchKernelGGL((bin3_ex_kernel<5, MM, kBin2Threads, RP, kHashMulHi>), grid, block, lds, s, a);
  else
    hipLaunchKernelGGL((bin3_ex_kernel<5, MM, kBin2Threads, RP, kHashShift>), grid, block, lds, s, a);
}

template <uint32_t MM>
static void launch_bin3_ex_m(int hm, dim3 grid, dim3 block, uint32_t lds, hipStream_t s, const BinArgs& a) {
  if (a.plan.rp == 3) launch_bin3_ex_mr<MM, 3>(hm, grid, block, lds, s, a);
  else launch_bin3_ex_mr<MM, kBin2Rows>(hm, grid, block, lds, s, a);
}

uint32_t bin3_lds_bytes(const BinPlan& p, uint32_t d, uint32_t rp, bool ex) {
  const uint64_t dp = (d <= 4) ? 4u : (d <= 6 ? 6u : 8u);
  const uint64_t nb = (uint64_t)rp * p.Pr + 1;
  const uint64_t words = (uint64_t)kTableWords * dp + nb + p.P + 2 * nb + (uint64_t)rp * p.tile + kBin2Threads / 64 +
                         (ex ? kExLdsWords : 0u);
  return words * 4 > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)(words * 4);
}

hipError_t launch_bin_routed(const float* pos, uint64_t n, const Mesh& mesh, const Tables& t, const BinPlan& plan,
                             uint16_t* tok, uint32_t* cnt, int32_t* M, uint32_t* err, const RouteExclude& ex,
                             hipStream_t s) {
  if (t.d != 5 || !plan.fast || plan.sort || (plan.rp != 2 && plan.rp != 3) || mesh.mode == kMeshPacked ||
      mesh.group != 1u)
    return hipErrorInvalidValue;
  BinArgs a = make_bin_args(pos, n, mesh, t, plan, tok, cnt, M, err);
  a.ex = ex;
  const dim3 grid(plan.nwg), block(kBin2Threads);
  if (mesh.mode == kMeshPow2Ratio) launch_bin3_ex_m<kMeshPow2Ratio>(t.hash_mode(), grid, block, plan.lds_bytes, s, a);
  else if (mesh.mode == kMeshExactRatio)
    launch_bin3_ex_m<kMeshExactRatio>(t.hash_mode(), grid, block, plan.lds_bytes, s, a);
  else launch_bin3_ex_m<kMeshGeneral>(t.hash_mode(), grid, block, plan.lds_bytes, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ accumulate


__device__ __forceinline__ void accumulate_body(const AccArgs& a, uint32_t s) {
  extern __shared__ uint32_t lds[];
  int32_t* acc = (int32_t*)lds;  // kSlice counters
  const BinPlan& pl = a.plan;
  const uint32_t r = s / pl.Pr, sl = s % pl.Pr;
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = lane_id();
  for (uint32_t i = tid; i < kSlice; i += kAccThreads) acc[i] = 0;
  __syncthreads();
  constexpr uint32_t U = 4;
  for (uint32_t g = wave; g < pl.nwg; g += kAccThreads / 64) {
    const uint32_t c = min(a.cnt[(uint64_t)s * pl.nwg + g], pl.cap);
    const uint16_t* reg = a.tok + ((uint64_t)g * pl.P + s) * (uint64_t)pl.cap;
    const uint4* t4 = (const uint4*)reg;
    const uint32_t nfull = c / 8;  // whole 16-byte chunks
    for (uint32_t q0 = 0; q0 < nfull; q0 += 64 * U) {
      uint4 v[U];
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        const uint32_t q = q0 + u * 64 + lane;
        v[u] = (q < nfull) ? t4[q] : make_uint4(0, 0, 0, 0);
      }
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        if (q0 + u * 64 + lane < nfull) {
          const uint32_t wds[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
          for (uint32_t e = 0; e < 8; ++e) {
            const uint32_t tk = (wds[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
            atomicAdd(&acc[tk & (kSlice - 1)], (tk & 0x8000u) ? -1 : 1);
          }
        }
      }
    }
    if (lane < c - nfull * 8) {
      const uint32_t tk = reg[nfull * 8 + lane];
      atomicAdd(&acc[tk & (kSlice - 1)], (tk & 0x8000u) ? -1 : 1);
    }
  }
  __syncthreads();
  const uint32_t b0 = sl * kSlice;
  const uint32_t len = min(kSlice, a.w - b0);
  int32_t* Mrow = a.M + (uint64_t)r * a.w + b0;
  for (uint32_t i = tid; i < len; i += kAccThreads) Mrow[i] = (int32_t)((uint32_t)Mrow[i] + (uint32_t)acc[i]);
}

__global__ __launch_bounds__(kAccThreads) void accumulate_kernel(AccArgs a) { accumulate_body(a, blockIdx.x); }

// Many sketches in one launch: block blockIdx.x sums slice blockIdx.x - acc_first[sketch]
// of sketch acc_sketch[blockIdx.x].
__global__ __launch_bounds__(kAccThreads) void accumulate_batch_kernel(const AccArgs* __restrict__ descs,
                                                                       const uint16_t* __restrict__ acc_sketch,
                                                                       const uint32_t* __restrict__ acc_first) {
  const uint32_t i = acc_sketch[blockIdx.x];
  accumulate_body(descs[i], blockIdx.x - acc_first[i]);
}

hipError_t launch_accumulate(const uint16_t* tok, const uint32_t* cnt, const BinPlan& plan, uint32_t w,
                             int32_t* M, hipStream_t s) {
  AccArgs a;
  a.tok = tok;
  a.cnt = cnt;
  a.plan = plan;
  a.w = w;
  a.M = M;
  hipLaunchKernelGGL(accumulate_kernel, dim3(plan.P), dim3(kAccThreads), kSlice * sizeof(int32_t), s, a);
  return hipGetLastError();
}

hipError_t launch_accumulate_batch(const AccArgs* descs, const uint16_t* acc_sketch, const uint32_t* acc_first,
                                   uint32_t nblocks, hipStream_t s) {
  hipLaunchKernelGGL(accumulate_batch_kernel, dim3(nblocks), dim3(kAccThreads), kSlice * sizeof(int32_t), s, descs,
                     acc_sketch, acc_first);
  return hipGetLastError();
}

// ------------------------------------------------------------------ direct update

// Fallback when the binned plan does not fit in LDS (very wide or very many rows):
// one global atomic per row per particle.
__global__ __launch_bounds__(256) void update_direct_kernel(const float* __restrict__ pos, uint64_t n, Mesh mesh,
                                                            const uint32_t* __restrict__ tab, uint32_t d,
                                                            uint32_t w, uint32_t cm, int32_t* __restrict__ M,
                                                            uint32_t* __restrict__ err) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    uint64_t key;
    if (!particle_key(pos, i, mesh, key)) {
      atomicOr(err, kErrDomain);
      continue;
    }
    for (uint32_t r = 0; r < d; ++r) {
      const uint32_t h = row_hash(tab + r * kTableWords, key);
      const uint32_t neg = (h >> 31) & (cm ^ 1u);
      atomicAdd(&M[(uint64_t)r * w + bucket_of(h, w)], neg ? -1 : 1);
    }
  }
}

hipError_t launch_update_direct(const float* pos, uint64_t n, const Mesh& mesh, const Tables& t, int32_t* M,
                                uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(update_direct_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, pos, n, mesh, t.tab,
                     t.d, t.w, t.cm, M, err);
  return hipGetLastError();
}

// The direct update with the router's exclusion (any d, float positions, ungrouped mesh):
// a particle in an admitted coarse cell adds 1 to its child counter instead of d counters.
__global__ __launch_bounds__(256) void update_direct_ex_kernel(const float* __restrict__ pos, uint64_t n, Mesh mesh,
                                                               const uint32_t* __restrict__ tab, uint32_t d,
                                                               uint32_t w, uint32_t cm, int32_t* __restrict__ M,
                                                               uint32_t* __restrict__ err, RouteExclude ex) {
  __shared__ __align__(16) uint32_t ex_words[kExLdsWords];
  const ExLds ext = ex_lds(ex_words);
  ex_fill(ex.admitted, adm_count(ex), ext);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    int32_t ix, iy, iz;
    const bool ok = (int)cell_index(pos[3 * i], mesh, ix) & (int)cell_index(pos[3 * i + 1], mesh, iy) &
                    (int)cell_index(pos[3 * i + 2], mesh, iz);
    if (!ok) {
      atomicOr(err, kErrDomain);
      continue;
    }
    uint32_t child;
    const int32_t c = ex_find(adm_coarse(ix, iy, iz, ex, child), ext);
    if (c >= 0) {
      atomicAdd(&ex.child[(uint32_t)c * ex.f3 + child], 1u);
      continue;
    }
    const uint64_t key =
        ((uint64_t)((uint32_t)ix * (uint32_t)mesh.G + (uint32_t)iy)) * (uint64_t)(uint32_t)mesh.G + (uint32_t)iz;
    for (uint32_t r = 0; r < d; ++r) {
      const uint32_t h = row_hash(tab + r * kTableWords, key);
      const uint32_t neg = (h >> 31) & (cm ^ 1u);
      atomicAdd(&M[(uint64_t)r * w + bucket_of(h, w)], neg ? -1 : 1);
    }
  }
}

hipError_t launch_update_direct_routed(const float* pos, uint64_t n, const Mesh& mesh, const Tables& t, int32_t* M,
                                       uint32_t* err, const RouteExclude& ex, hipStream_t s) {
  if (mesh.mode == kMeshPacked || mesh.group != 1u) return hipErrorInvalidValue;
  hipLaunchKernelGGL(update_direct_ex_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, pos, n, mesh, t.tab,
                     t.d, t.w, t.cm, M, err, ex);
  return hipGetLastError();
}

// Bin workgroups of one update: the requested cap, else 256 (tables in LDS) or 512.
uint32_t bin_wg_cap(uint32_t d, uint32_t requested) {
  return requested ? requested : ((d <= (uint32_t)kTabLdsRows) ? 256u : 512u);
}

}  // namespace csk
