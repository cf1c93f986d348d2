// csk_sortbin.hip — launches of the sort-word bin kernel (csk_sortbin_body.h) on the packed
// sort-word table: d = 5..8 rows and w = 2^lw counters per row with w <= 2^24 and
// lw + 1 <= floor(128 / d) (the packed-hash condition), single sketches and batches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csk_sortbin_body.h"

namespace csk {

namespace {

using namespace sortbin;

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
    hipLaunchKernelGGL((sortbin_kernel<D, MODE, NT, RP, PF, false, false>), L.grid, dim3(NT), L.lds, L.s,
                       *L.a);
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

uint32_t sortbin_lds_bytes(uint32_t d, uint32_t rp, uint32_t Pr, uint32_t P, bool rows, uint32_t nch, bool ex) {
  // the layout does not depend on the thread count
  const uint32_t dp = rows ? (d <= 4 ? 4u : (d <= 6 ? 6u : 8u)) : 4u;
  const uint32_t tile = (uint32_t)kBin2Threads * (uint32_t)bin2_ppt((int)d);
  return sort_lds(dp, rows ? nch : (uint32_t)kChars, rp, (rows || ex) ? Pr : 512u, P, tile, ex).words * 4u;
}

hipError_t launch_sortbin(const BinArgs& a, uint32_t mode, hipStream_t s) {
  if (a.plan.sort == kSortRows) return launch_sortbin_rows(a, mode, s);
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
