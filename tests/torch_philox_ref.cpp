// Philox4x32-10 words from PyTorch's own engine (at::philox_engine, a header-only
// implementation independent of this repository's generator), for the CPU pins of the
// workload generator and the router's sample coin.  Built by the tests with g++.
#include <ATen/core/PhiloxRNGEngine.h>

#include <cstdint>

// counter (c0, c1, c2, c3) and key (k0, k1): the engine's offset is (c0, c1), its
// subsequence (c2, c3) and its seed (k0, k1); four calls return the block's four words.
extern "C" void torch_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  const uint64_t seed = (uint64_t)key[0] | ((uint64_t)key[1] << 32);
  const uint64_t sub = (uint64_t)ctr[2] | ((uint64_t)ctr[3] << 32);
  const uint64_t off = (uint64_t)ctr[0] | ((uint64_t)ctr[1] << 32);
  at::philox_engine e(seed, sub, off);
  for (int i = 0; i < 4; ++i) out[i] = e();
}
