// csk_sortbin_rows.hip — launches of the sort-word bin kernel (csk_sortbin_body.h) on the
// row-interleaved tables with multiply-high buckets: d = 5..8 rows of any width w <= 2^24
// (the widths the packed sort-word table cannot serve), and, for d = 5, the update of the
// learned router's rest sketch with its exclusion.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csk_sortbin_body.h"

namespace csk {

namespace {

using namespace sortbin;

template <int D, uint32_t MODE, int RP, bool EX>
void launch_rows_one(const BinArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((sortbin_kernel<D, MODE, kBin2Threads, RP, false, true, EX>), dim3(a.plan.nwg),
                     dim3(kBin2Threads), a.plan.lds_bytes, s, a);
}

// Compiled forms: 1024 threads, no prefetch; two or three rows per pass.
template <int D, uint32_t MODE>
void launch_rows_m(const BinArgs& a, hipStream_t s) {
  if (a.plan.rp == 3) launch_rows_one<D, MODE, 3, false>(a, s);
  else launch_rows_one<D, MODE, 2, false>(a, s);
}

template <int D>
void launch_rows_d(const BinArgs& a, uint32_t mode, hipStream_t s) {
  if (mode == kMeshPow2Ratio) launch_rows_m<D, kMeshPow2Ratio>(a, s);
  else if (mode == kMeshExactRatio) launch_rows_m<D, kMeshExactRatio>(a, s);
  else launch_rows_m<D, kMeshGeneral>(a, s);
}

}  // namespace

hipError_t launch_sortbin_rows(const BinArgs& a, uint32_t mode, hipStream_t s) {
  switch (a.d) {
    case 5: launch_rows_d<5>(a, mode, s); break;
    case 6: launch_rows_d<6>(a, mode, s); break;
    case 7: launch_rows_d<7>(a, mode, s); break;
    default: launch_rows_d<8>(a, mode, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_sortbin_routed(const BinArgs& a, uint32_t mode, hipStream_t s) {
  if (mode == kMeshPow2Ratio) launch_rows_one<5, kMeshPow2Ratio, 2, true>(a, s);
  else if (mode == kMeshExactRatio) launch_rows_one<5, kMeshExactRatio, 2, true>(a, s);
  else launch_rows_one<5, kMeshGeneral, 2, true>(a, s);
  return hipGetLastError();
}

}  // namespace csk
