// csk_sortbin.hip — the bin kernel of the update (Sec. 2.2 Add; Alg. 4 Update; Sec. 3.1
// stages 1-3) for the configurations it is tuned for: d = 5..8 rows and w = 2^lw counters
// per row with w <= 2^24 and lw + 1 <= floor(128 / d) (the packed-hash condition).
//
// Per particle: the exact cell key, then ONE pass over the key's bytes through a packed
// "sort-word" table that yields, for every row at once, the token's 16-bit payload and its
// slice.  The table is the packed top-bits table with each row's field permuted at set-up
// (hash XOR acts bit by bit, so a fixed permutation of every entry's bits commutes with
// the XOR): field' = (slice << 16) | (sign << 15) | (offset in the 2^15-counter slice),
// i.e. exactly the sort word, minus the row-in-pass that a per-row constant adds.
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
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csk_kernel_util.h"

namespace csk {

namespace {

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

// LDS layout (words), all offsets but the last fixed at compile time:
//   Ts [6 * 256 * 4] | hist [NBP] | cur [NBP] | dst [NBP] | stage [RP * TILE] | wsum [16] | cursor [P]
template <int D, int NT, int RP>
struct SortLayout {
  static constexpr int TILE = kBin2Threads * bin2_ppt(D);   // the tile of the general kernel's plans
  static constexpr int PPT = TILE / NT;
  static constexpr uint32_t NBP = RP * 512 + 1;  // bins of a pass for Pr <= 512, + the dummy
  static constexpr uint32_t kTs = 0;
  static constexpr uint32_t kHist = kTableWords * 4;
  static constexpr uint32_t kCur = kHist + NBP;
  static constexpr uint32_t kDst = kCur + NBP;
  static constexpr uint32_t kStage = (kDst + NBP + 3) & ~3u;
  static constexpr uint32_t kWsum = kStage + RP * TILE;
  static constexpr uint32_t kCursor = kWsum + 16;
  static constexpr uint32_t words(uint32_t P) { return kCursor + P; }
};

template <int D, uint32_t MODE, int NT, int RP, bool PF>
__device__ __forceinline__ void sortbin_body(const BinArgs* __restrict__ ap, const float* __restrict__ pos,
                                             uint64_t n, uint32_t g) {
  using Lay = SortLayout<D, NT, RP>;
  constexpr int PPT = Lay::PPT, TILE = Lay::TILE;
  constexpr int F = packed_bits(D);
  constexpr uint32_t FMASK = (F >= 32) ? 0xFFFFFFFFu : ((1u << F) - 1u);
  constexpr uint32_t NW = NT / 64;
  constexpr uint32_t BPT = (Lay::NBP + NT - 1) / NT;   // scan bins per thread
  static_assert(NT % 256 == 0 && PPT * NT == TILE, "tile = NT x PPT, whole uint4 reads of the wave totals");
  static_assert(RP * TILE <= 65535, "staging slots fit 16 bits");
  const BinArgs& a = *ap;
  const BinPlan& pl = a.plan;
  extern __shared__ __align__(16) uint32_t lds5[];
  uint32_t* ts = lds5 + Lay::kTs;
  uint32_t* hist = lds5 + Lay::kHist;
  uint32_t* cur = lds5 + Lay::kCur;
  uint32_t* dst = lds5 + Lay::kDst;
  uint32_t* stage = lds5 + Lay::kStage;
  uint32_t* wsum = lds5 + Lay::kWsum;
  uint32_t* cursor = lds5 + Lay::kCursor;
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
  const uint32_t Pr = pl.Pr, cap = pl.cap;
  const uint32_t nb = RP * Pr + 1, dummy = nb - 1;
  // byte address of token slot t of this workgroup's regions is tokb + 2 * (t + kBiasTok)
  char* __restrict__ tokb = (char*)(a.tok + (uint64_t)g * pl.P * cap) - 2u * kBiasTok;

  for (uint32_t i = tid; i < pl.P; i += NT) cursor[i] = 0;
  for (uint32_t i = tid; i < Lay::NBP; i += NT) hist[i] = 0;
  stage_tables<4>(ts, a.tabs, a.mesh.nch);   // ends with a barrier

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
      uint64_t key;   // always a key of the mesh, so the table lookups stay in range
      const bool ok = cell_key_m<MODE, false>(px[j], py[j], pz[j], a.mesh, key) && in;  // ungrouped (plan)
      inside |= (uint32_t)in << j;
      valid |= (uint32_t)ok << j;
      uint32_t q[4];
      row_hashes<4>(ts, key, a.mesh.nch, q);
#pragma unroll
      for (int r = 0; r < D; ++r) {
        const uint32_t v = (field_bits<F>(q, r) & FMASK) | rowc[r];
        sv[r][j] = ok ? v : (dummy << 16);
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

template <int D, uint32_t MODE, int NT, int RP, bool PF>
__global__ __launch_bounds__(NT) void sortbin_kernel(BinArgs a) {
  sortbin_body<D, MODE, NT, RP, PF>(&a, a.pos, a.n, blockIdx.x);
}

template <int D, uint32_t MODE, int NT, int RP, bool PF>
__global__ __launch_bounds__(NT) void sortbin_batch_kernel(const BinArgs* __restrict__ descs,
                                                           const uint16_t* __restrict__ wg_sketch,
                                                           const uint32_t* __restrict__ wg_first, BatchCall call) {
  const uint32_t i = wg_sketch[blockIdx.x];
  sortbin_body<D, MODE, NT, RP, PF>(descs + i, call.pos[i], call.n[i], blockIdx.x - wg_first[i]);
}

struct Launch {
  bool batch;
  dim3 grid;
  uint32_t lds;
  hipStream_t s;
  const BinArgs* a;
  const BinArgs* descs;
  const uint16_t* wg_sketch;
  const uint32_t* wg_first;
  const BatchCall* call;
};

template <int D, uint32_t MODE, int NT, int RP, bool PF>
void launch_one(const Launch& L) {
  if (L.batch)
    hipLaunchKernelGGL((sortbin_batch_kernel<D, MODE, NT, RP, PF>), L.grid, dim3(NT), L.lds, L.s, L.descs,
                       L.wg_sketch, L.wg_first, *L.call);
  else
    hipLaunchKernelGGL((sortbin_kernel<D, MODE, NT, RP, PF>), L.grid, dim3(NT), L.lds, L.s, *L.a);
}

// The compiled forms: (threads, rows per pass, prefetch).  1024 threads keep 16 waves per
// CU with at most 128 VGPRs each (no room for a prefetched tile); 512 threads keep 8 waves
// with room for it.
template <int D, uint32_t MODE>
void launch_m(uint32_t nt, uint32_t rp, uint32_t pf, const Launch& L) {
  if constexpr (D == 5) {
    if (nt == 512) {   // the 512-thread forms are compiled for d = 5 only (the plan checks)
      if (rp == 3) {
        if (pf) launch_one<D, MODE, 512, 3, true>(L);
        else launch_one<D, MODE, 512, 3, false>(L);
      } else {
        launch_one<D, MODE, 512, 2, true>(L);
      }
      return;
    }
  }
  (void)pf;
  if (rp == 3) launch_one<D, MODE, 1024, 3, false>(L);
  else launch_one<D, MODE, 1024, 2, false>(L);
}

template <int D>
void launch_d(uint32_t mode, uint32_t nt, uint32_t rp, uint32_t pf, const Launch& L) {
  if (mode == kMeshPow2Ratio) launch_m<D, kMeshPow2Ratio>(nt, rp, pf, L);
  else if (mode == kMeshExactRatio) launch_m<D, kMeshExactRatio>(nt, rp, pf, L);
  else launch_m<D, kMeshGeneral>(nt, rp, pf, L);
}

void launch_any(uint32_t d, uint32_t mode, uint32_t nt, uint32_t rp, uint32_t pf, const Launch& L) {
  switch (d) {
    case 5: launch_d<5>(mode, nt, rp, pf, L); break;
    case 6: launch_d<6>(mode, nt, rp, pf, L); break;
    case 7: launch_d<7>(mode, nt, rp, pf, L); break;
    default: launch_d<8>(mode, nt, rp, pf, L); break;
  }
}

}  // namespace

uint32_t sortbin_lds_bytes(uint32_t d, uint32_t rp, uint32_t P) {
  // the layout does not depend on the thread count
  uint32_t words = 0;
  switch (d) {
    case 5: words = (rp == 3) ? SortLayout<5, 1024, 3>::words(P) : SortLayout<5, 1024, 2>::words(P); break;
    case 6: words = (rp == 3) ? SortLayout<6, 1024, 3>::words(P) : SortLayout<6, 1024, 2>::words(P); break;
    case 7: words = (rp == 3) ? SortLayout<7, 1024, 3>::words(P) : SortLayout<7, 1024, 2>::words(P); break;
    default: words = (rp == 3) ? SortLayout<8, 1024, 3>::words(P) : SortLayout<8, 1024, 2>::words(P); break;
  }
  return words * 4u;
}

hipError_t launch_sortbin(const BinArgs& a, uint32_t mode, hipStream_t s) {
  const Launch L{false, dim3(a.plan.nwg), a.plan.lds_bytes, s, &a, nullptr, nullptr, nullptr, nullptr};
  launch_any(a.d, mode, a.plan.nt, a.plan.rp, a.plan.pf, L);
  return hipGetLastError();
}

hipError_t launch_sortbin_batch(const BinArgs* descs, const uint16_t* wg_sketch, const uint32_t* wg_first,
                                uint32_t nwg_total, uint32_t lds_bytes, uint32_t d, uint32_t mode, const BinPlan& form,
                                uint32_t kb, const BatchCall& call, hipStream_t s) {
  (void)kb;   // the kernel hashes the key bytes each sketch's mesh needs
  const Launch L{true, dim3(nwg_total), lds_bytes, s, nullptr, descs, wg_sketch, wg_first, &call};
  launch_any(d, mode, form.nt, form.rp, form.pf, L);
  return hipGetLastError();
}

}  // namespace csk
