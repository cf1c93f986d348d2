// csk_router.h — launch interface of the learned-router kernels (csk_router.hip).
// Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csk_device.h"
#include "csk_internal.h"

namespace csk {

constexpr uint32_t kSampleStream = 4;   // Philox stream of the sampling coin
constexpr int kFeatPad = 32;            // 27 neighbour features, padded to an MFMA K step
constexpr int kHidden = 64;             // hidden width of both layers
constexpr uint32_t kMaxAdmitted = 512;  // coarse cells an exact table takes at most
// MLP parameter layout (fp32 master copy): W1 [64][32], b1 [64], W2 [64][64], b2 [64],
// w3 [64], b3 [1]
constexpr uint32_t kOffW1 = 0, kOffB1 = 2048, kOffW2 = 2112, kOffB2 = 6208, kOffW3 = 6272, kOffB3 = 6336;
constexpr uint32_t kParams = 6337;

hipError_t launch_sample_counts(const float* pos, uint64_t n, uint64_t index0, uint64_t seed, uint32_t threshold,
                                const Mesh& coarse, uint32_t* counts, uint32_t* bitmap, hipStream_t s);
hipError_t launch_features(const uint32_t* counts, uint32_t Gc, const uint64_t* cells, uint64_t m, float* feat,
                           hipStream_t s);
// C = beta C + A B with bf16 operands and fp32 sums.  With `partial` (device scratch of
// partial_floats floats), products with k >= 2 kSplitK and fewer than 256 tiles are split
// over k in chunks of about kSplitK and the chunks summed in a fixed order.
constexpr uint32_t kSplitK = 256;
hipError_t launch_gemm_bf16(uint32_t M, uint32_t N, uint32_t K, const float* A, uint64_t sai, uint64_t sak,
                            const float* B, uint64_t sbk, uint64_t sbj, float* C, uint64_t sci, uint64_t scj,
                            float beta, hipStream_t s, float* partial = nullptr, uint64_t partial_floats = 0,
                            bool split = false);
hipError_t launch_bias_act(float* Y, uint32_t M, uint32_t N, const float* bias, bool relu, hipStream_t s);
hipError_t launch_head(const float* H2, uint32_t M, const float* w3, const float* b3, float* z, const float* y,
                       float* dz, float* loss, bool round, hipStream_t s);
hipError_t launch_head_back(const float* dz, const float* H2, const float* w3, uint32_t M, float* dA, hipStream_t s);
hipError_t launch_relu_back(float* dA, const float* H, uint64_t total, hipStream_t s);
hipError_t launch_colsum(const float* X, uint32_t M, uint32_t N, uint32_t ld, const float* w, float* out, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m1, float* m2, uint32_t n, float lr_t, float b1, float b2,
                       float eps, hipStream_t s);
// The routing split: workgroups of kSplitThreads, kSplitPPT particles per lane per wave
// tile, at most kSplitMaxWaves waves (each with one contiguous range of the stream), at
// most kSplitMaxChildren admitted children (the LDS counters of one workgroup).
constexpr int kSplitThreads = 1024;
constexpr int kSplitPPT = 8;        // count pass
constexpr int kSplitWritePPT = 4;   // write pass (divides kSplitPPT: same wave ranges)
constexpr uint64_t kSplitWaveTile = 64ull * kSplitPPT;
constexpr uint32_t kSplitMaxWaves = 4096;
constexpr uint32_t kSplitMaxChildren = 32768;
uint32_t split_waves(uint64_t n, uint64_t* wchunk);
uint64_t split_workspace_bytes(uint32_t na, uint32_t factor);
hipError_t launch_route_split(const float* pos, uint64_t n, const Mesh& mesh, uint32_t factor, const uint64_t* admitted,
                              uint32_t na, uint64_t* tkeys, uint32_t* tcounts, uint32_t tmask, float* rest_pos,
                              unsigned long long* rest_count, uint32_t* err, void* workspace, hipStream_t s);


constexpr uint32_t kCellListBlocks = 65536;   // workgroups of the ordered cell listing
hipError_t launch_exact_count(const float* pos, uint64_t n, const Mesh& mesh, uint64_t* tkeys, uint32_t* tcounts,
                              uint32_t tmask, uint32_t* err, hipStream_t s);
uint32_t cell_list_blocks(uint64_t ncells, uint64_t* chunk);
hipError_t launch_cell_list(const uint32_t* counts, uint64_t ncells, uint32_t min_count, const uint32_t* bitmap,
                            uint64_t* block_scratch, uint64_t* cells, uint64_t cap, unsigned long long* total,
                            hipStream_t s);
hipError_t launch_bitmap_clear(uint32_t* bitmap, uint64_t ncells, uint32_t* counts, hipStream_t s);
hipError_t launch_parents_sorted(const uint64_t* keys, uint32_t n, uint64_t G, uint32_t factor, uint64_t* tmp,
                                 uint64_t* out, hipStream_t s);
hipError_t launch_rank_sort(const uint64_t* in, uint32_t n, uint64_t* out, hipStream_t s);
hipError_t launch_labels(const uint64_t* cells, uint64_t m, const uint64_t* par, uint32_t np, float* labels,
                         hipStream_t s);
hipError_t launch_logit_order(const float* z, uint64_t m, int32_t* out, hipStream_t s);

// ---- the sync-free routed step
// Features and fp32 logits of cells[0 .. min(*m_dev, cap)) (params: the MLP's 6337 fp32
// parameters, device).
hipError_t launch_route_score(const uint32_t* counts, uint32_t Gc, const uint64_t* cells, const uint64_t* m_dev,
                              uint64_t cap, const float* params, float* z, hipStream_t s);
// Admission over a device count: ord (cap words), st, sk / se / rank / ok / oe (A each) and
// err are scratch; admitted (A keys, ascending) and *na (device) are the result.
hipError_t launch_admit_dev(const uint64_t* cells, const float* logits, const uint64_t* m_dev, uint64_t cap, uint32_t A,
                            int32_t* ord, SelState* st, uint64_t* sk, int32_t* se, uint32_t* rank, uint64_t* ok,
                            int32_t* oe, uint32_t* err, uint64_t* admitted, uint32_t* na, hipStream_t s);
// The exclusion's child counters added to the exact table (table_slot probing).
hipError_t launch_route_table(const RouteExclude& ex, uint32_t G, uint64_t* tkeys, uint32_t* tcounts, uint32_t tmask,
                              uint32_t* err, hipStream_t s);

}  // namespace csk
