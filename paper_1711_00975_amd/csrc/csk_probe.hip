// csk_probe.hip — measurement probes for the ceilings the update is priced against: the
// achievable read bandwidth of 12-byte particle records (the update's own load pattern),
// the LDS atomic rate on a 128 KiB array, the device-scope global atomic rate into tables of
// a given size (resident in L2, in the MALL, or in HBM), and the rate of workgroup-scope
// atomics into a per-XCD copy of a table (performed in that XCD's L2).  Built as
// libcsk_probe.so and used only by the benchmark; not part of the C ABI of the sketch.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 1024;
constexpr int kPPT = 8;

// Every 12-byte record of pos read once, eight per thread in flight (clamped index), with
// the bits folded into one word per thread so the loads stay live.
__global__ __launch_bounds__(kThreads) void stream_read_kernel(const float* __restrict__ pos, uint64_t n,
                                                               uint32_t* __restrict__ sink) {
  const uint64_t tile = (uint64_t)kThreads * kPPT;
  const uint64_t last = n - 1;
  uint32_t acc = 0;
  for (uint64_t first = (uint64_t)blockIdx.x * tile; first < n; first += (uint64_t)gridDim.x * tile) {
    float x[kPPT], y[kPPT], z[kPPT];
#pragma unroll
    for (int j = 0; j < kPPT; ++j) {
      uint64_t i = first + (uint64_t)j * kThreads + threadIdx.x;
      i = i < last ? i : last;
      x[j] = __builtin_nontemporal_load(pos + 3 * i);
      y[j] = __builtin_nontemporal_load(pos + 3 * i + 1);
      z[j] = __builtin_nontemporal_load(pos + 3 * i + 2);
    }
#pragma unroll
    for (int j = 0; j < kPPT; ++j) acc ^= __float_as_uint(x[j]) ^ __float_as_uint(y[j]) ^ __float_as_uint(z[j]);
  }
  sink[(uint64_t)blockIdx.x * kThreads + threadIdx.x] = acc;
}

__device__ __forceinline__ uint32_t lcg(uint32_t x) { return x * 1664525u + 1013904223u; }

// iters random ds_add per thread on 2^15 LDS words (128 KiB); sums written to sink.
__global__ __launch_bounds__(kThreads) void lds_atomic_kernel(uint64_t iters, uint32_t* __restrict__ sink) {
  extern __shared__ uint32_t lds[];
  for (uint32_t i = threadIdx.x; i < 32768u; i += kThreads) lds[i] = 0;
  __syncthreads();
  uint32_t x = (blockIdx.x * kThreads + threadIdx.x) * 2654435761u + 1u;
  for (uint64_t it = 0; it < iters; ++it) {
    x = lcg(x);
    atomicAdd(&lds[x >> 17], 1u);   // 15-bit index
  }
  __syncthreads();
  sink[(uint64_t)blockIdx.x * kThreads + threadIdx.x] = lds[threadIdx.x];
}

// iters random device-scope atomicAdd per thread into 2^log2_words int32 words.
__global__ __launch_bounds__(256) void global_atomic_kernel(int32_t* __restrict__ table, uint32_t log2_words,
                                                            uint64_t iters) {
  uint32_t x = (blockIdx.x * 256u + threadIdx.x) * 2654435761u + 7u;
  const uint32_t shift = 32u - log2_words;
  for (uint64_t it = 0; it < iters; ++it) {
    x = lcg(x);
    atomicAdd(&table[x >> shift], 1);
  }
}

// The XCD (accelerator complex die) this wave runs on: hardware register XCC_ID, bits 3:0.
__device__ __forceinline__ uint32_t xcc_id() {
  return (uint32_t)__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u;
}

// iters random workgroup-scope atomicAdd per thread into this XCD's private copy of a table
// of 2^log2_words words (table holds 8 copies).  Such an atomic is performed in the L2 of the
// XCD that issues it; the rate is what a per-XCD privatised update could reach.
__global__ __launch_bounds__(256) void xcd_atomic_kernel(int32_t* __restrict__ table, uint32_t log2_words,
                                                         uint64_t iters) {
  int32_t* __restrict__ mine = table + ((uint64_t)xcc_id() << log2_words);
  uint32_t x = (blockIdx.x * 256u + threadIdx.x) * 2654435761u + 11u;
  const uint32_t shift = 32u - log2_words;
  for (uint64_t it = 0; it < iters; ++it) {
    x = lcg(x);
    __hip_atomic_fetch_add(&mine[x >> shift], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

}  // namespace

// blocks * 256 * iters workgroup-scope atomics, each into the issuing XCD's copy of a
// 2^log2_words-word table: table (device) holds 8 << log2_words int32.  0 or a HIP error.
extern "C" int probe_xcd_atomics(int32_t* table, uint32_t log2_words, uint64_t iters, uint32_t blocks, void* stream) {
  if (blocks == 0 || log2_words < 1 || log2_words > 28) return -1;
  hipLaunchKernelGGL(xcd_atomic_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, table, log2_words, iters);
  return (int)hipGetLastError();
}

// n records at pos (device); sink (device) holds blocks * 1024 words.  0 or a HIP error.
extern "C" int probe_stream_read(const float* pos, uint64_t n, uint32_t* sink, uint32_t blocks, void* stream) {
  if (n == 0 || blocks == 0) return 0;
  hipLaunchKernelGGL(stream_read_kernel, dim3(blocks), dim3(kThreads), 0, (hipStream_t)stream, pos, n, sink);
  return (int)hipGetLastError();
}

// blocks * 1024 * iters LDS atomics; sink (device) holds blocks * 1024 words.
extern "C" int probe_lds_atomics(uint64_t iters, uint32_t blocks, uint32_t* sink, void* stream) {
  if (blocks == 0) return 0;
  hipLaunchKernelGGL(lds_atomic_kernel, dim3(blocks), dim3(kThreads), 32768 * sizeof(uint32_t), (hipStream_t)stream,
                     iters, sink);
  return (int)hipGetLastError();
}

// blocks * 256 * iters atomics into table (device, 2^log2_words int32, 1 <= log2_words <= 31).
extern "C" int probe_global_atomics(int32_t* table, uint32_t log2_words, uint64_t iters, uint32_t blocks,
                                    void* stream) {
  if (blocks == 0 || log2_words < 1 || log2_words > 31) return -1;
  hipLaunchKernelGGL(global_atomic_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, table, log2_words, iters);
  return (int)hipGetLastError();
}
