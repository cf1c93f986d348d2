// csk_sortbin_body.h — the sort-word bin kernel of the update (Sec. 2.2 Add; Alg. 4 Update;
// Sec. 3.1 stages 1-3), shared by its two translation units: csk_sortbin.hip (the packed
// sort-word table, w = 2^lw) and csk_sortbin_rows.hip (row-interleaved tables with
// multiply-high buckets for any w, and the router's exclusion).
//
// Per particle: the exact cell key, then the token of every row with its slice:
//   sort-word table  ONE pass over the key's bytes through a packed table that yields, for
//                    every row at once, the token's 16-bit payload and its slice.  The table is
//                    the packed top-bits table with each row's field permuted at set-up (hash
//                    XOR acts bit by bit, so a fixed permutation of every entry's bits commutes
//                    with the XOR): field' = (slice << 16) | (sign << 15) | (offset in the
//                    2^15-counter slice), i.e. exactly the sort word, minus the row-in-pass that
//                    a per-row constant adds;
//   row tables       the full 32-bit row words from the interleaved tables, bucket = high word
//                    of (h31 << 1) * w, and the same sort word assembled from it.
//
// Tokens are counting-sorted in LDS, RP rows per pass:
//   count    one LDS add per token on its bin
//   scan     bin bases (wave scans with DPP, one barrier for the wave totals); every bin
//            gets its destination (region offset - base, in bytes) and its scatter cursor
//   scatter  one LDS add-with-return on the bin's cursor gives the staging slot
//   write    staged words go out in order, each as a 16-bit store at dst[bin] + 2 slot,
//            overlapped with the next pass's counting
// Regions are workgroup-major as in the general bin kernel: region (g, s) starts at
// (g * P + s) * cap tokens; a run that would overflow its region is added to M with
// atomics instead (same sum).  With PF the positions of the workgroup's next tile are
// loaded while the current tile is sorted.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csk_kernel_util.h"

namespace csk {
namespace sortbin {

constexpr uint32_t kDropDst = 0xFFFFFFFFu;      // dummy bin: never written
constexpr uint32_t kOverflowDst = 0xFFFFFFFEu;  // run added with atomics
constexpr uint32_t kBiasTok = 1u << 16;         // keeps region offset + cursor - base positive

// Inclusive scan over the wave with DPP row shifts and row broadcasts (wave64).
__device__ __forceinline__ uint32_t wave_scan_dpp(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// LDS layout (words), nb = RP * Pr + 1 bins a pass (the last one the dummy):
//   [EX: the exclusion's table, kExLdsWords] | tables [kb * 256 * dp] | hist [nb] | cur [nb] |
//   dst [nb] | stage [RP * tile] | wsum [16] | cursor [P]
// dp = 4 for the sort-word table (all six key bytes staged), RowPad(d) for the row tables
// (the mesh's kb = nch key bytes).
struct SortLds {
  uint32_t ts, hist, cur, dst, stage, wsum, cursor, words;
};
__host__ __device__ __forceinline__ SortLds sort_lds(uint32_t dp, uint32_t kb, uint32_t rp, uint32_t Pr, uint32_t P,
                                                     uint32_t tile, bool ex) {
  SortLds L;
  const uint32_t nb = rp * Pr + 1u;
  L.ts = ex ? kExLdsWords : 0u;
  L.hist = L.ts + 256u * dp * kb;
  L.cur = L.hist + nb;
  L.dst = L.cur + nb;
  L.stage = (L.dst + nb + 3u) & ~3u;
  L.wsum = L.stage + rp * tile;
  L.cursor = L.wsum + 16u;
  L.words = L.cursor + P;
  return L;
}

// The tile of the general kernel's plans: 1024 threads x bin2_ppt(D) particles.
template <int D>
constexpr int sort_tile() { return kBin2Threads * bin2_ppt(D); }

// ROWS false: the sort-word table (w = 2^lw, packed fields); ROWS true: the row-interleaved
// tables over the mesh's nch key bytes, bucket = high word of (h31 << 1) * w (any w; for
// w = 2^lw it is the plain shift).  EX: the router's exclusion (d = 5): a particle in an admitted coarse
// cell is counted in the exclusion's child counters and goes to the dummy bin instead.
template <int D, uint32_t MODE, int NT, int RP, bool PF, bool ROWS, bool EX>
__device__ __forceinline__ void sortbin_body(const BinArgs* __restrict__ ap, const float* __restrict__ pos,
                                             uint64_t n, uint32_t g) {
  constexpr int TILE = sort_tile<D>(), PPT = TILE / NT;
  constexpr int DP = ROWS ? RowPad<D>::value : 4;
  constexpr int F = packed_bits(D);
  constexpr uint32_t FMASK = (F >= 32) ? 0xFFFFFFFFu : ((1u << F) - 1u);
  constexpr uint32_t NW = NT / 64;
  constexpr uint32_t NBMAX = RP * 512 + 1;             // bins of a pass for Pr <= 512, + the dummy
  constexpr uint32_t BPT = (NBMAX + NT - 1) / NT;      // scan bins per thread
  static_assert(NT % 256 == 0 && PPT * NT == TILE, "tile = NT x PPT, whole uint4 reads of the wave totals");
  static_assert(RP * TILE <= 65535, "staging slots fit 16 bits");
  static_assert(!EX || (D == 5 && MODE != kMeshPacked), "the exclusion is compiled for d = 5, float positions");
  const BinArgs& a = *ap;
  const BinPlan& pl = a.plan;
  extern __shared__ __align__(16) uint32_t lds5[];
  const uint32_t Pr = pl.Pr, cap = pl.cap;
  // the packed form keeps the compile-time layout of 512 slices per row (no register
  // holds an offset); the others size the bins by the plan's Pr
  const SortLds Ly = sort_lds(DP, ROWS ? a.mesh.nch : (uint32_t)kChars, RP, (ROWS || EX) ? Pr : 512u, pl.P, TILE, EX);
  const ExLds ext = ex_lds(lds5);   // EX only
  uint32_t* ts = lds5 + Ly.ts;
  uint32_t* hist = lds5 + Ly.hist;
  uint32_t* cur = lds5 + Ly.cur;
  uint32_t* dst = lds5 + Ly.dst;
  uint32_t* stage = lds5 + Ly.stage;
  uint32_t* wsum = lds5 + Ly.wsum;
  uint32_t* cursor = lds5 + Ly.cursor;
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
  const uint32_t nb = RP * Pr + 1, dummy = nb - 1;
  const uint32_t pos_sign = a.cm ^ 1u;   // ROWS: Count-Min tokens carry no sign
  // byte address of token slot t of this workgroup's regions is tokb + 2 * (t + kBiasTok)
  char* __restrict__ tokb = (char*)(a.tok + (uint64_t)g * pl.P * cap) - 2u * kBiasTok;

  for (uint32_t i = tid; i < pl.P; i += NT) cursor[i] = 0;
  for (uint32_t i = tid; i < nb; i += NT) hist[i] = 0;
  if constexpr (ROWS) stage_tables<DP>(ts, a.tabi, a.mesh.nch, a.mesh.nch);   // the nch bytes keys use
  else stage_tables<4>(ts, a.tabs, a.mesh.nch);   // ends with a barrier
  if constexpr (EX) ex_fill(a.ex.admitted, adm_count(a.ex), ext);   // ends with a barrier

  uint32_t rowc[D];   // per-row constant: (row in pass) * Pr in the bin half of the word
#pragma unroll
  for (int r = 0; r < D; ++r) rowc[r] = ((uint32_t)(r % RP) * Pr) << 16;

  bool pending = false;
  uint32_t pend_row0 = 0, pend_total = 0;
  auto write_out = [&]() {
    const uint32_t total = pend_total;
#pragma unroll 1
    for (uint32_t q0 = 0; q0 < total; q0 += 4 * NT) {
      uint32_t v[4], dq[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t q = q0 + u * NT + tid;
        v[u] = stage[q < total ? q : 0];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t q = q0 + u * NT + tid;
        dq[u] = (q < total) ? dst[v[u] >> 16] : kDropDst;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t q = q0 + u * NT + tid;
        if (dq[u] < kOverflowDst) {
          *(uint16_t*)(tokb + (dq[u] + 2u * q)) = (uint16_t)(v[u] & 0xFFFFu);
        } else if (dq[u] == kOverflowDst) {
          // region full: add this one update straight to the counter (rare; same sum)
          const uint32_t bin = v[u] >> 16;
          const uint32_t r = pend_row0 + bin / Pr, sl = bin % Pr;
          const uint32_t bkt = (sl << kSliceBits) | (v[u] & (kSlice - 1));
          atomicAdd(&a.M[(uint64_t)r * a.w + bkt], (v[u] & 0x8000u) ? -1 : 1);
        }
      }
    }
  };

  // bins of the scan: thread t owns bins [BPT t, BPT t + BPT) of the nb
  const uint32_t blo = min(nb, BPT * tid), bhi = min(nb, blo + BPT);

  const uint64_t ntiles = (n + TILE - 1) / TILE;
  const uint64_t last = n - 1;
  float px[PPT], py[PPT], pz[PPT];
  // Positions are addressed from the stream base: a per-tile base with 32-bit lane offsets
  // measured 15.7 ms per update of the 2^30-particle stream against 13.4, and buffer loads
  // through a per-tile resource (as the candidate pass uses) 3.25 against 3.18 ms per 2^28.
  auto load_tile = [&](uint64_t tile) {
    const uint64_t first = tile * (uint64_t)TILE;
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        uint64_t i = first + (uint64_t)j * NT + tid;
        i = i < last ? i : last;   // unconditional loads; lanes past the stream are masked later
        px[j] = __builtin_nontemporal_load(pos + 3 * i);
        py[j] = __builtin_nontemporal_load(pos + 3 * i + 1);
        pz[j] = __builtin_nontemporal_load(pos + 3 * i + 2);
      }
  };
  if (PF && g < ntiles) load_tile(g);

  for (uint64_t tile = g; tile < ntiles; tile += pl.nwg) {
    const uint64_t first = tile * (uint64_t)TILE;
    const bool full = first + TILE <= n;
    if (!PF) load_tile(tile);
    uint32_t sv[D][PPT];
    uint32_t inside = 0, valid = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const bool in = full || (first + (uint64_t)j * NT + tid) < n;
      uint64_t key;   // every byte indexes its table in range, whatever the particle
      bool ok;
      if constexpr (EX) {
        int32_t ix, iy, iz;
        ok = ((int)cell_index_m<MODE>(px[j], a.mesh, ix) & (int)cell_index_m<MODE>(py[j], a.mesh, iy) &
              (int)cell_index_m<MODE>(pz[j], a.mesh, iz)) && in;
        key = ((uint64_t)((uint32_t)ix * (uint32_t)a.mesh.G + (uint32_t)iy)) * (uint64_t)(uint32_t)a.mesh.G +
              (uint64_t)(uint32_t)iz;   // ungrouped (plan)
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
        ok = cell_key_m<MODE, false>(px[j], py[j], pz[j], a.mesh, key) && in;  // ungrouped (plan)
        valid |= (uint32_t)ok << j;
      }
      inside |= (uint32_t)in << j;
      if constexpr (ROWS) {
        // a loop over the mesh's key bytes, as the sort-word table takes: unrolled over a
        // fixed byte count, the eight particles' lookups are hoisted together and spill
        uint32_t h[DP];
        row_hashes<DP>(ts, key, a.mesh.nch, h);
#pragma unroll
        for (int r = 0; r < D; ++r) {
          // bin = (row in pass) * Pr + slice: an add, as Pr need not be a power of two
          const uint32_t b = bucket_of(h[r], a.w);
          const uint32_t v = (((b >> kSliceBits) << 16) + rowc[r]) | (((h[r] >> 31) & pos_sign) << 15) |
                             (b & (kSlice - 1));
          sv[r][j] = ok ? v : (dummy << 16);
        }
      } else {
        uint32_t q[4];
        row_hashes<4>(ts, key, a.mesh.nch, q);
#pragma unroll
        for (int r = 0; r < D; ++r) {   // Pr = w / 2^15 is a power of two: or = add
          const uint32_t v = (field_bits<F>(q, r) & FMASK) | rowc[r];
          sv[r][j] = ok ? v : (dummy << 16);
        }
      }
    }
    if (PF && tile + pl.nwg < ntiles) load_tile(tile + pl.nwg);
    if (inside & ~valid) atomicOr(a.err, kErrDomain);

#pragma unroll
    for (int r0 = 0; r0 < D; r0 += RP) {
      const int nr = (D - r0 < RP) ? D - r0 : RP;
      if (pending) write_out();
      // count
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
#pragma unroll
        for (int qq = 0; qq < RP; ++qq)
          if (qq < nr) atomicAdd(&hist[sv[r0 + qq < D ? r0 + qq : r0][j] >> 16], 1u);
      }
      __syncthreads();   // counts complete; the previous pass is written out
      uint32_t hc[BPT], csum = 0;
#pragma unroll
      for (uint32_t e = 0; e < BPT; ++e) {
        hc[e] = (blo + e < bhi) ? hist[blo + e] : 0u;
        csum += hc[e];
      }
      const uint32_t incl = wave_scan_dpp(csum);
      if (lane == 63u) wsum[wave] = incl;
      __syncthreads();
      uint32_t before = 0, total = 0;
#pragma unroll
      for (uint32_t w4 = 0; w4 < NW / 4; ++w4) {
        const uint4 s4 = ((const uint4*)wsum)[w4];
        const uint32_t sw[4] = {s4.x, s4.y, s4.z, s4.w};
#pragma unroll
        for (uint32_t e = 0; e < 4; ++e) {
          before += (4 * w4 + e < wave) ? sw[e] : 0u;
          total += sw[e];
        }
      }
      uint32_t run = before + incl - csum;
      const uint32_t slice0 = (uint32_t)r0 * Pr;
#pragma unroll
      for (uint32_t e = 0; e < BPT; ++e) {
        const uint32_t b = blo + e;
        if (b < bhi) {
          const uint32_t hb = hc[e];
          hist[b] = 0;
          cur[b] = run;
          uint32_t dv = kDropDst;   // the dummy bin and unused row bins of the last pass
          if (b < (uint32_t)nr * Pr) {
            const uint32_t c = cursor[slice0 + b];
            if (c + hb <= cap) {
              dv = 2u * ((slice0 + b) * cap + c + kBiasTok - run);
              cursor[slice0 + b] = c + hb;
            } else {
              dv = kOverflowDst;
            }
          }
          dst[b] = dv;
          run += hb;
        }
      }
      __syncthreads();
      // scatter
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
#pragma unroll
        for (int qq = 0; qq < RP; ++qq) {
          if (qq < nr) {
            const uint32_t v = sv[r0 + qq < D ? r0 + qq : r0][j];
            const uint32_t slot = atomicAdd(&cur[v >> 16], 1u);
            stage[slot] = v;
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

template <int D, uint32_t MODE, int NT, int RP, bool PF, bool ROWS, bool EX>
__global__ __launch_bounds__(NT) void sortbin_kernel(BinArgs a) {
  sortbin_body<D, MODE, NT, RP, PF, ROWS, EX>(&a, a.pos, a.n, blockIdx.x);
}

template <int D, uint32_t MODE, int NT, int RP, bool PF>
__global__ __launch_bounds__(NT) void sortbin_batch_kernel(const BinArgs* __restrict__ descs,
                                                           const uint16_t* __restrict__ wg_sketch,
                                                           const uint32_t* __restrict__ wg_first, BatchCall call) {
  const uint32_t i = wg_sketch[blockIdx.x];
  sortbin_body<D, MODE, NT, RP, PF, false, false>(descs + i, call.pos[i], call.n[i], blockIdx.x - wg_first[i]);
}

}  // namespace sortbin
}  // namespace csk
