// csk_router.hip — kernels of the learned router: a 1 % sample pre-pass gives coarse
// cell counts, a 27 -> 64 -> 64 -> 1 MLP (bf16 operands on MFMA, fp32 accumulation)
// scores coarse cells, the highest-scored ones are counted exactly in a device hash table
// and every other particle goes on to a Count Sketch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csk_kernel_util.h"
#include "csk_router.h"

namespace csk {

// ------------------------------------------------------------------ sampling

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4x32 bijection with the
// published multipliers and Weyl key increments.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    // each 32 x 32 -> 64-bit product in one v_mad_u64_u32
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Particle g = index0 + i is in the sample when word g of the Philox stream kSampleStream
// under the seed (word g mod 4 of counter (g / 4 lo, g / 4 hi, kSampleStream, 0)) is below
// `threshold`.  Each thread draws kSampleU consecutive counters per round (4 kSampleU
// particles), then loads the positions of the sampled ones, up to four at a time with every
// load issued before any is used: about one particle in a hundred is sampled, so a round
// waits on one memory round trip instead of one per counter.  With a bitmap, a cell's bit
// is set when its count leaves 0.
constexpr int kSampleU = 4;
__global__ __launch_bounds__(256) void sample_counts_kernel(const float* __restrict__ pos, uint64_t n, uint64_t index0,
                                                            uint64_t seed, uint32_t threshold, Mesh coarse,
                                                            uint32_t* __restrict__ counts,
                                                            uint32_t* __restrict__ bitmap) {
  const uint64_t c_lo = index0 >> 2, c_hi = (index0 + n + 3) >> 2;   // counters that cover the range
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * kSampleU;
  for (uint64_t c0 = c_lo + ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kSampleU; c0 < c_hi; c0 += stride) {
    uint32_t hits = 0;   // bit 4 u + q: particle 4 (c0 + u) + q is sampled
#pragma unroll
    for (int u = 0; u < kSampleU; ++u) {
      const uint64_t c = c0 + (uint64_t)u;
      uint32_t r[4] = {(uint32_t)c, (uint32_t)(c >> 32), kSampleStream, 0u};
      philox4x32_10(r, (uint32_t)seed, (uint32_t)(seed >> 32));
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint64_t g = 4 * c + (uint64_t)q;
        const bool take = c < c_hi && g >= index0 && g - index0 < n && r[q] < threshold;
        hits |= (uint32_t)take << (4 * u + q);
      }
    }
    while (hits) {
      uint64_t ii[4];
      bool have[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        have[k] = hits != 0;
        const uint32_t b = have[k] ? (uint32_t)__ffs(hits) - 1u : 0u;
        hits &= hits - 1u;
        ii[k] = have[k] ? 4 * c0 + b - index0 : 0;
      }
      float px[4], py[4], pz[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (have[k]) {
          px[k] = pos[3 * ii[k]];
          py[k] = pos[3 * ii[k] + 1];
          pz[k] = pos[3 * ii[k] + 2];
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        uint64_t key;
        if (have[k] && cell_key(px[k], py[k], pz[k], coarse, key)) {
          const uint32_t old = atomicAdd(&counts[key], 1u);
          if (bitmap != nullptr && old == 0) atomicOr(&bitmap[key >> 5], 1u << (key & 31u));   // first touch
        }
      }
    }
  }
}

// feat[j][0..26] = log1p(count) of coarse cell j's 27 periodic neighbours, ordered
// (dx, dy, dz) in {-1, 0, 1}^3 lexicographically; feat[j][27..31] = 0.
__global__ __launch_bounds__(256) void features_kernel(const uint32_t* __restrict__ counts, uint32_t Gc,
                                                       const uint64_t* __restrict__ cells, uint64_t m,
                                                       float* __restrict__ feat) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
    const uint64_t key = cells[j];
    const uint64_t G = Gc;
    const int64_t cx = (int64_t)(key / (G * G)), cy = (int64_t)((key / G) % G), cz = (int64_t)(key % G);
    float* f = feat + j * kFeatPad;
    int q = 0;
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          const uint64_t x = (uint64_t)((cx + dx + (int64_t)G) % (int64_t)G);
          const uint64_t y = (uint64_t)((cy + dy + (int64_t)G) % (int64_t)G);
          const uint64_t z = (uint64_t)((cz + dz + (int64_t)G) % (int64_t)G);
          f[q++] = log1pf((float)counts[(x * G + y) * G + z]);
        }
    for (; q < kFeatPad; ++q) f[q] = 0.0f;
  }
}

// Features and the float32 forward pass of the router's model for cells j < min(*m, cap):
// x = log1p of the 27 neighbour counts (in the order of features_kernel), h1 = relu(W1 x +
// b1), h2 = relu(W2 h1 + b2), z = w3 . h2 + b3; every sum is fmaf in index order, then the
// bias, all in fp32.  The parameters sit in LDS (W1 transposed, so that a feature's 64
// weights are consecutive) and are read as broadcast operands; each thread scores one cell,
// its features in LDS, h1 in registers.  The loops over a feature and over a layer-2 output
// stay rolled, so that the weights are not hoisted into registers (the unrolled form took
// 425 VGPRs: one wave per SIMD).
constexpr int kScoreThreads = 256;
__global__ __launch_bounds__(kScoreThreads) void route_score_kernel(const uint32_t* __restrict__ counts, uint32_t Gc,
                                                                    const uint64_t* __restrict__ cells,
                                                                    const uint64_t* __restrict__ m_dev, uint64_t cap,
                                                                    const float* __restrict__ P,
                                                                    float* __restrict__ z) {
  __shared__ __align__(16) float w1t[27 * kHidden];              // w1t[q][o] = W1[o][q]
  __shared__ __align__(16) float w[kParams - kOffB1];            // b1, W2, b2, w3, b3
  __shared__ float xs[27 * kScoreThreads];                       // xs[q][thread]
  for (uint32_t i = threadIdx.x; i < 27u * kHidden; i += blockDim.x) {
    const uint32_t q = i / kHidden, o = i % kHidden;
    w1t[i] = P[kOffW1 + o * kFeatPad + q];
  }
  for (uint32_t i = threadIdx.x; i < kParams - kOffB1; i += blockDim.x) w[i] = P[kOffB1 + i];
  __syncthreads();
  const float* b1 = w;
  const float* W2 = w + (kOffW2 - kOffB1);
  const float* b2 = w + (kOffB2 - kOffB1);
  const float* w3 = w + (kOffW3 - kOffB1);
  const float b3 = w[kOffB3 - kOffB1];
  const uint64_t m = *m_dev < cap ? *m_dev : cap;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
    const uint64_t key = cells[j];
    const uint64_t G = Gc;
    const int64_t cx = (int64_t)(key / (G * G)), cy = (int64_t)((key / G) % G), cz = (int64_t)(key % G);
#pragma unroll
    for (int q = 0; q < 27; ++q) {
      const int dx = q / 9 - 1, dy = (q / 3) % 3 - 1, dz = q % 3 - 1;
      const uint64_t nx = (uint64_t)((cx + dx + (int64_t)G) % (int64_t)G);
      const uint64_t ny = (uint64_t)((cy + dy + (int64_t)G) % (int64_t)G);
      const uint64_t nz = (uint64_t)((cz + dz + (int64_t)G) % (int64_t)G);
      xs[q * kScoreThreads + threadIdx.x] = log1pf((float)counts[(nx * G + ny) * G + nz]);
    }
    float h1[kHidden];
#pragma unroll
    for (int o = 0; o < kHidden; ++o) h1[o] = 0.0f;
#pragma unroll 1
    for (int q = 0; q < 27; ++q) {
      const float xq = xs[q * kScoreThreads + threadIdx.x];
      const float4* wq = (const float4*)(w1t + q * kHidden);
#pragma unroll
      for (int o4 = 0; o4 < kHidden / 4; ++o4) {
        const float4 c = wq[o4];
        h1[4 * o4] = fmaf(c.x, xq, h1[4 * o4]);
        h1[4 * o4 + 1] = fmaf(c.y, xq, h1[4 * o4 + 1]);
        h1[4 * o4 + 2] = fmaf(c.z, xq, h1[4 * o4 + 2]);
        h1[4 * o4 + 3] = fmaf(c.w, xq, h1[4 * o4 + 3]);
      }
    }
#pragma unroll
    for (int o = 0; o < kHidden; ++o) h1[o] = fmaxf(h1[o] + b1[o], 0.0f);
    float out = 0.0f;
#pragma unroll 1
    for (int o = 0; o < kHidden; ++o) {
      const float4* wo = (const float4*)(W2 + o * kHidden);
      float t = 0.0f;
#pragma unroll
      for (int q4 = 0; q4 < kHidden / 4; ++q4) {
        const float4 c = wo[q4];
        t = fmaf(c.x, h1[4 * q4], t);
        t = fmaf(c.y, h1[4 * q4 + 1], t);
        t = fmaf(c.z, h1[4 * q4 + 2], t);
        t = fmaf(c.w, h1[4 * q4 + 3], t);
      }
      out = fmaf(w3[o], fmaxf(t + b2[o], 0.0f), out);
    }
    z[j] = out + b3;
  }
}

// ------------------------------------------------------------------ MLP

// fp32 -> bf16, round to nearest even (finite inputs)
__device__ __forceinline__ short to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_value(short h) { return __uint_as_float((uint32_t)(uint16_t)h << 16); }

// Partial product of one 16x16 tile of C over k in [k_lo, k_hi): A(i, k) = A[i * sai + k * sak],
// B(k, j) = B[k * sbk + j * sbj] read as fp32, products accumulated in fp32 by gfx950's
// v_mfma_f32_16x16x32_bf16; elements outside the matrices read as 0.  Lane l holds A row
// l % 16 at k = 8 (l / 16) .. +7 and B column l % 16 at the same k; the result is rows
// 4 (l / 16) .. +3 of column l % 16.
// SPLIT = false: every operand is rounded to bf16 (one product per k block).
// SPLIT = true: every operand x is carried as hi = bf16(x) plus lo = bf16(x - hi), and the
// tile sums hi.hi + hi.lo + lo.hi (three products): the operands keep 16 significant bits
// and the result is within a few fp32 roundings of the fp32 product (lo.lo, below 2^-16
// relative, is left out).
template <bool SPLIT>
__device__ __forceinline__ f32x4 gemm_tile(uint32_t M, uint32_t N, uint32_t k_lo, uint32_t k_hi,
                                           const float* __restrict__ A, uint64_t sai, uint64_t sak,
                                           const float* __restrict__ B, uint64_t sbk, uint64_t sbj, uint32_t i0,
                                           uint32_t j0, uint32_t lane) {
  const uint32_t r = lane & 15u, kq = (lane >> 4) * 8;
  const uint32_t ia = i0 + r, jb = j0 + r;
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (uint32_t k0 = k_lo; k0 < k_hi; k0 += 32) {
    s16x8 ah, bh, al, bl;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint32_t k = k0 + kq + (uint32_t)e;
      const float av = (ia < M && k < k_hi) ? A[ia * sai + k * sak] : 0.0f;
      const float bv = (jb < N && k < k_hi) ? B[k * sbk + jb * sbj] : 0.0f;
      ah[e] = to_bf16(av);
      bh[e] = to_bf16(bv);
      if (SPLIT) {
        al[e] = to_bf16(av - bf16_value(ah[e]));
        bl[e] = to_bf16(bv - bf16_value(bh[e]));
      }
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ah), __builtin_bit_cast(bf16x8, bh), acc,
                                                  0, 0, 0);
    if (SPLIT) {
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ah), __builtin_bit_cast(bf16x8, bl),
                                                    acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, al), __builtin_bit_cast(bf16x8, bh),
                                                    acc, 0, 0, 0);
    }
  }
  return acc;
}

// C[i][j] = beta * C[i][j] + sum_k A(i, k) * B(k, j) for i < M, j < N.  One wave per 16x16
// tile of C; elements outside C are not written.
template <bool SPLIT>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(uint32_t M, uint32_t N, uint32_t K, const float* __restrict__ A,
                                                        uint64_t sai, uint64_t sak, const float* __restrict__ B,
                                                        uint64_t sbk, uint64_t sbj, float* __restrict__ C,
                                                        uint64_t sci, uint64_t scj, float beta) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t tiles_n = (N + 15) / 16;
  const uint64_t tile = (uint64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const uint64_t tiles = (uint64_t)((M + 15) / 16) * tiles_n;
  if (tile >= tiles) return;   // whole waves only: every lane of a wave shares its tile
  const uint32_t i0 = (uint32_t)(tile / tiles_n) * 16, j0 = (uint32_t)(tile % tiles_n) * 16;
  const f32x4 acc = gemm_tile<SPLIT>(M, N, 0, K, A, sai, sak, B, sbk, sbj, i0, j0, lane);
  const uint32_t r = lane & 15u, kq = (lane >> 4) * 4;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t i = i0 + kq + (uint32_t)e, j = j0 + r;
    if (i < M && j < N) {
      float* c = C + i * sci + j * scj;
      *c = (beta != 0.0f ? beta * *c : 0.0f) + acc[e];
    }
  }
}

// Split over k for products with a long k and few tiles (the weight gradients, k = batch
// rows): chunk y = blockIdx.y covers k in [y kc, (y + 1) kc) and writes its partial tile to
// P[y][i][j] (M x N row-major); splitk_reduce_kernel sums the chunks in order.
__global__ __launch_bounds__(256) void gemm_bf16_splitk_kernel(uint32_t M, uint32_t N, uint32_t K, uint32_t kc,
                                                               const float* __restrict__ A, uint64_t sai, uint64_t sak,
                                                               const float* __restrict__ B, uint64_t sbk, uint64_t sbj,
                                                               float* __restrict__ P) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t tiles_n = (N + 15) / 16;
  const uint64_t tile = (uint64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const uint64_t tiles = (uint64_t)((M + 15) / 16) * tiles_n;
  if (tile >= tiles) return;
  const uint32_t i0 = (uint32_t)(tile / tiles_n) * 16, j0 = (uint32_t)(tile % tiles_n) * 16;
  const uint32_t k_lo = blockIdx.y * kc, k_hi = (k_lo + kc < K) ? k_lo + kc : K;
  const f32x4 acc = gemm_tile<false>(M, N, k_lo, k_hi, A, sai, sak, B, sbk, sbj, i0, j0, lane);
  float* out = P + (uint64_t)blockIdx.y * M * N;
  const uint32_t r = lane & 15u, kq = (lane >> 4) * 4;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t i = i0 + kq + (uint32_t)e, j = j0 + r;
    if (i < M && j < N) out[(uint64_t)i * N + j] = acc[e];
  }
}

__global__ __launch_bounds__(256) void splitk_reduce_kernel(const float* __restrict__ P, uint32_t nsplit, uint32_t M,
                                                            uint32_t N, float* __restrict__ C, uint64_t sci,
                                                            uint64_t scj, float beta) {
  const uint64_t total = (uint64_t)M * N;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (uint32_t y = 0; y < nsplit; ++y) s += P[(uint64_t)y * total + t];
    const uint32_t i = (uint32_t)(t / N), j = (uint32_t)(t % N);
    float* c = C + i * sci + j * scj;
    *c = (beta != 0.0f ? beta * *c : 0.0f) + s;
  }
}

// Y[i][j] = act(Y[i][j] + bias[j]) over an M x N row-major block; act = ReLU if relu.
__global__ __launch_bounds__(256) void bias_act_kernel(float* __restrict__ Y, uint32_t M, uint32_t N,
                                                       const float* __restrict__ bias, uint32_t relu) {
  const uint64_t total = (uint64_t)M * N;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
    float v = Y[t] + bias[t % N];
    if (relu) v = v > 0.0f ? v : 0.0f;
    Y[t] = v;
  }
}

// Output layer and loss: z[i] = H2[i] . w3 + b3 in fp32 sums, with H2 and w3 rounded to
// bf16 (round = 1, the training pass) or not (the scoring pass); with labels y,
// dz[i] = (sigmoid(z) - y) / M and loss[0] += mean binary cross-entropy.
__global__ __launch_bounds__(256) void head_kernel(const float* __restrict__ H2, uint32_t M, const float* __restrict__ w3,
                                                   const float* __restrict__ b3, float* __restrict__ z,
                                                   const float* __restrict__ y, float* __restrict__ dz,
                                                   float* __restrict__ loss, uint32_t round) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < M; i += gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int j = 0; j < kHidden; ++j) {
      float wj = w3[j], hj = H2[(uint64_t)i * kHidden + j];
      if (round) {
        wj = bf16_value(to_bf16(wj));
        hj = bf16_value(to_bf16(hj));
      }
      s = fmaf(hj, wj, s);
    }
    s += b3[0];
    z[i] = s;
    if (y != nullptr) {
      const float p = 1.0f / (1.0f + expf(-s));
      dz[i] = (p - y[i]) / (float)M;
      // BCE with logits, stable form: max(z, 0) - z y + log(1 + exp(-|z|))
      const float l = fmaxf(s, 0.0f) - s * y[i] + log1pf(expf(-fabsf(s)));
      atomicAdd(loss, l / (float)M);
    }
  }
}

// dA[i][j] = dz[i] * w3[j] where H2[i][j] > 0 (ReLU), else 0.
__global__ __launch_bounds__(256) void head_back_kernel(const float* __restrict__ dz, const float* __restrict__ H2,
                                                        const float* __restrict__ w3, uint32_t M,
                                                        float* __restrict__ dA) {
  const uint64_t total = (uint64_t)M * kHidden;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t i = (uint32_t)(t / kHidden), j = (uint32_t)(t % kHidden);
    dA[t] = H2[t] > 0.0f ? dz[i] * w3[j] : 0.0f;
  }
}

// dA[t] *= (H[t] > 0)
__global__ __launch_bounds__(256) void relu_back_kernel(float* __restrict__ dA, const float* __restrict__ H, uint64_t total) {
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x)
    if (!(H[t] > 0.0f)) dA[t] = 0.0f;
}

// out[j] = sum_i X[i * ld + j] * (w ? w[i] : 1) for j < N: one block per column, a fixed
// summation order (deterministic).
__global__ __launch_bounds__(256) void colsum_kernel(const float* __restrict__ X, uint32_t M, uint32_t N, uint32_t ld,
                                                     const float* __restrict__ w, float* __restrict__ out) {
  __shared__ float part[256];
  const uint32_t j = blockIdx.x;
  float s = 0.0f;
  for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) s += X[(uint64_t)i * ld + j] * (w ? w[i] : 1.0f);
  part[threadIdx.x] = s;
  __syncthreads();
  for (uint32_t h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0 && j < N) out[j] = part[0];
}

// Adam on the fp32 master weights (bias-corrected step sizes from the host).
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m1, float* __restrict__ m2, uint32_t n, float lr_t,
                                                   float b1, float b2, float eps) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    m1[t] = b1 * m1[t] + (1.0f - b1) * g[t];
    m2[t] = b2 * m2[t] + (1.0f - b2) * g[t] * g[t];
    p[t] -= lr_t * m1[t] / (sqrtf(m2[t]) + eps);
  }
}

// ------------------------------------------------------------------ routing

// The split runs in two passes over the same contiguous ranges of the stream, one range
// per wave: pass 1 counts each range's rest particles, a scan turns the counts into output
// offsets, pass 2 writes each range's rest in stream order (a wave ballot orders the
// appends, no workgroup barrier) and counts the admitted particles in a workgroup-private
// LDS array of the admitted cells' children.  The per-workgroup arrays are summed and
// inserted into the exact table once.  Admitted cells are found through an LDS hash of
// their keys (one probe or two), not a search.

struct SplitArgs {
  const float* pos;
  uint64_t n;
  Mesh mesh;
  uint32_t factor;      // fine cells per coarse cell along an axis
  uint32_t fmagic;      // ceil(2^32 / factor): i / factor = umulhi(i, fmagic) for i < 2^16
  uint32_t f3;          // factor^3
  const uint64_t* admitted;
  uint32_t na;
  uint32_t nwaves;      // waves with a range
  uint64_t wchunk;      // particles per wave (a multiple of kSplitWaveTile)
};

static_assert(kAdmHashSlots == 2 * kMaxAdmitted, "the admitted-key hash is loaded at most 1/2");
constexpr uint64_t kEmptySlot = kAdmEmpty;

// Fill the LDS hash (key -> position in the admitted list); ends with a barrier.
__device__ __forceinline__ void adm_hash_build(const SplitArgs& a, uint64_t* hkey, uint16_t* hidx) {
  adm_hash_fill(a.admitted, a.na, hkey, hidx);
}

// Classes of a wave tile's PPT particles: cls[j] = position of the admitted coarse
// parent in the sorted list, -1 (rest) or -2 (outside the domain); child[j] = position of
// the fine cell inside its coarse cell.  The two first probes of every particle are
// loaded before any is used, so that the LDS latencies overlap; a longer probe run
// (rare at load 1/2) finishes in a loop.
template <uint32_t MODE, int PPT>
__device__ __forceinline__ void split_classes(const float (&p)[PPT][3], const SplitArgs& a, const uint64_t* hkey,
                                              const uint16_t* hidx, int32_t (&cls)[PPT], uint32_t (&child)[PPT]) {
  const uint32_t f = a.factor;
  const uint64_t Gc = (uint64_t)((uint32_t)a.mesh.G / f);
  uint64_t ckey[PPT];
  uint32_t sl[PPT];
  bool ok[PPT];
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    int32_t ix, iy, iz;
    ok[j] = (int)cell_index_m<MODE>(p[j][0], a.mesh, ix) & (int)cell_index_m<MODE>(p[j][1], a.mesh, iy) &
            (int)cell_index_m<MODE>(p[j][2], a.mesh, iz);
    const uint32_t cx = __umulhi((uint32_t)ix, a.fmagic), cy = __umulhi((uint32_t)iy, a.fmagic),
                   cz = __umulhi((uint32_t)iz, a.fmagic);
    ckey[j] = ((uint64_t)cx * Gc + cy) * Gc + cz;
    child[j] = (((uint32_t)ix - cx * f) * f + ((uint32_t)iy - cy * f)) * f + ((uint32_t)iz - cz * f);
    sl[j] = adm_hash(ckey[j]);
  }
  uint64_t k0[PPT], k1[PPT];
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    k0[j] = hkey[sl[j]];
    k1[j] = hkey[(sl[j] + 1) & (kAdmHashSlots - 1)];
  }
  bool slow_any = false;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const bool h0 = k0[j] == ckey[j], e0 = k0[j] == kEmptySlot;
    const bool h1 = k1[j] == ckey[j], e1 = k1[j] == kEmptySlot;
    const bool found = h0 || (!e0 && h1);
    const uint32_t at = h0 ? sl[j] : ((sl[j] + 1) & (kAdmHashSlots - 1));
    const int32_t c = found ? (int32_t)hidx[at] : -1;
    cls[j] = ok[j] ? c : -2;
    const bool slow = !h0 && !e0 && !h1 && !e1;   // both probes held other keys
    slow_any |= slow;
    sl[j] = slow ? ((sl[j] + 2) & (kAdmHashSlots - 1)) : kAdmHashSlots;
  }
  if (slow_any) {
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      if (sl[j] == kAdmHashSlots || !ok[j]) continue;
      uint32_t q = sl[j];
      for (uint32_t probe = 2; probe < kAdmHashSlots; ++probe) {
        const uint64_t k = hkey[q];
        if (k == ckey[j]) {
          cls[j] = (int32_t)hidx[q];
          break;
        }
        if (k == kEmptySlot) break;
        q = (q + 1) & (kAdmHashSlots - 1);
      }
    }
  }
}

// Loads of one wave tile: PPT particles per lane (j * 64 + lane), all issued before
// the first use (indices clamped to the last particle; the caller masks by validity).
template <int PPT>
__device__ __forceinline__ void split_load(const SplitArgs& a, uint64_t t0, uint32_t lane, float (&p)[PPT][3]) {
  const uint64_t last = a.n - 1;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    uint64_t i = t0 + (uint64_t)j * 64 + lane;
    i = i < last ? i : last;
    p[j][0] = a.pos[3 * i];
    p[j][1] = a.pos[3 * i + 1];
    p[j][2] = a.pos[3 * i + 2];
  }
}

template <uint32_t MODE>
__global__ __launch_bounds__(kSplitThreads) void split_count_kernel(SplitArgs a, uint64_t* __restrict__ wave_rest,
                                                                    uint32_t* __restrict__ err) {
  __shared__ uint64_t hkey[kAdmHashSlots];
  __shared__ uint16_t hidx[kAdmHashSlots];
  adm_hash_build(a, hkey, hidx);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wid = blockIdx.x * (kSplitThreads / 64) + (threadIdx.x >> 6);
  if (wid >= a.nwaves) return;   // whole waves; no barrier follows
  const uint64_t lo = (uint64_t)wid * a.wchunk;
  const uint64_t hi = lo + a.wchunk < a.n ? lo + a.wchunk : a.n;
  uint32_t rest = 0;
  bool bad = false;
  for (uint64_t t0 = lo; t0 < hi; t0 += kSplitWaveTile) {
    float p[kSplitPPT][3];
    split_load(a, t0, lane, p);
    int32_t cls[kSplitPPT];
    uint32_t child[kSplitPPT];
    split_classes<MODE>(p, a, hkey, hidx, cls, child);
#pragma unroll
    for (int j = 0; j < kSplitPPT; ++j) {
      const uint64_t i = t0 + (uint64_t)j * 64 + lane;
      if (i < hi) {
        rest += cls[j] == -1;
        bad |= cls[j] == -2;
      }
    }
  }
  if (bad) atomicOr(err, 1u);
  for (int off = 32; off > 0; off >>= 1) rest += __shfl_down(rest, off, 64);
  if (lane == 0) wave_rest[wid] = rest;
}

// Exclusive scan of the nw <= 4096 wave counts, offset by *rest_count; *rest_count grows by
// the total.
__global__ __launch_bounds__(1024) void split_scan_kernel(uint64_t* __restrict__ v, uint32_t nw,
                                                          unsigned long long* __restrict__ rest_count) {
  __shared__ uint64_t part[1024];
  const uint32_t lo = threadIdx.x * 4;
  uint64_t x[4], s = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    x[q] = lo + q < nw ? v[lo + q] : 0;
    s += x[q];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (uint32_t off = 1; off < 1024; off <<= 1) {   // inclusive Hillis-Steele scan
    const uint64_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  const uint64_t base = *rest_count;
  uint64_t run = base + part[threadIdx.x] - s;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (lo + q < nw) {
      v[lo + q] = run;
      run += x[q];
    }
  __syncthreads();
  if (threadIdx.x == 0) *rest_count = base + part[1023];
}

template <uint32_t MODE>
__global__ __launch_bounds__(kSplitThreads) void split_write_kernel(SplitArgs a, const uint64_t* __restrict__ wave_off,
                                                                    float* __restrict__ rest_pos,
                                                                    uint32_t* __restrict__ dense_part) {
  extern __shared__ uint32_t dense[];          // na * f3 counters of this workgroup
  __shared__ uint64_t hkey[kAdmHashSlots];
  __shared__ uint16_t hidx[kAdmHashSlots];
  const uint32_t nd = a.na * a.f3;
  for (uint32_t i = threadIdx.x; i < nd; i += blockDim.x) dense[i] = 0;
  adm_hash_build(a, hkey, hidx);               // ends with a barrier
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wid = blockIdx.x * (kSplitThreads / 64) + (threadIdx.x >> 6);
  if (wid < a.nwaves) {
    const uint64_t lo = (uint64_t)wid * a.wchunk;
    const uint64_t hi = lo + a.wchunk < a.n ? lo + a.wchunk : a.n;
    uint64_t base = wave_off[wid];
    for (uint64_t t0 = lo; t0 < hi; t0 += 64ull * kSplitWritePPT) {
      float p[kSplitWritePPT][3];
      split_load(a, t0, lane, p);
      int32_t cls[kSplitWritePPT];
      uint32_t child[kSplitWritePPT];
      split_classes<MODE>(p, a, hkey, hidx, cls, child);
#pragma unroll
      for (int j = 0; j < kSplitWritePPT; ++j) {
        const uint64_t i = t0 + (uint64_t)j * 64 + lane;
        const int32_t c = cls[j];
        const bool valid = i < hi;
        if (valid && c >= 0) atomicAdd(&dense[(uint32_t)c * a.f3 + child[j]], 1u);
        const bool rest = valid && c == -1;
        const uint64_t mask = __ballot(rest);
        if (rest) {
          const uint64_t o = base + (uint64_t)__popcll(lane ? (mask & (~0ull >> (64 - lane))) : 0ull);
          rest_pos[3 * o] = p[j][0];
          rest_pos[3 * o + 1] = p[j][1];
          rest_pos[3 * o + 2] = p[j][2];
        }
        base += (uint64_t)__popcll(mask);
      }
    }
  }
  __syncthreads();
  uint32_t* out = dense_part + (uint64_t)blockIdx.x * nd;
  for (uint32_t i = threadIdx.x; i < nd; i += blockDim.x) out[i] = dense[i];
}

// Sum of the nb partial arrays, and every child with a nonzero count added to the exact
// table under its fine key (linear probing from table_slot; bit 1 of *err if full).
__global__ __launch_bounds__(256) void split_table_kernel(SplitArgs a, const uint32_t* __restrict__ dense_part,
                                                          uint32_t nb, uint64_t* __restrict__ tkeys,
                                                          uint32_t* __restrict__ tcounts, uint32_t tmask,
                                                          uint32_t* __restrict__ err) {
  const uint32_t nd = a.na * a.f3;
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < nd; e += gridDim.x * blockDim.x) {
    uint32_t cnt = 0;
    for (uint32_t b = 0; b < nb; ++b) cnt += dense_part[(uint64_t)b * nd + e];
    if (cnt == 0) continue;
    const uint32_t f = a.factor, ai = e / a.f3, c = e % a.f3;
    const uint64_t G = (uint64_t)(uint32_t)a.mesh.G, Gc = G / f;
    const uint64_t P = a.admitted[ai];
    const uint64_t px = P / (Gc * Gc), py = (P / Gc) % Gc, pz = P % Gc;
    const uint64_t ix = px * f + c / (f * f), iy = py * f + (c / f) % f, iz = pz * f + c % f;
    const uint64_t key = (ix * G + iy) * G + iz;
    uint32_t sl = table_slot(key, tmask);
    bool placed = false;
    for (uint32_t probe = 0; probe <= tmask; ++probe) {
      uint64_t cur = __hip_atomic_load(&tkeys[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (cur == ~0ull) {
        cur = atomicCAS((unsigned long long*)&tkeys[sl], ~0ull, (unsigned long long)key);
        if (cur == ~0ull) cur = key;
      }
      if (cur == key) {
        atomicAdd(&tcounts[sl], cnt);
        placed = true;
        break;
      }
      sl = (sl + 1) & tmask;
    }
    if (!placed) atomicOr(err, 2u);
  }
}

// ------------------------------------------------------------------ exact counting

// Every in-domain particle adds 1 to its cell key's entry of the table (linear probing
// from table_slot; keys all-ones when empty).  Out-of-domain particles set bit 0 of *err;
// a key that finds no free slot after probing the whole table sets bit 1.
__global__ __launch_bounds__(256) void exact_count_kernel(const float* __restrict__ pos, uint64_t n, Mesh mesh,
                                                          uint64_t* __restrict__ tkeys, uint32_t* __restrict__ tcounts,
                                                          uint32_t tmask, uint32_t* __restrict__ err) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    uint64_t key;
    if (!cell_key(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], mesh, key)) {
      atomicOr(err, 1u);
      continue;
    }
    uint32_t sl = table_slot(key, tmask);
    bool placed = false;
    for (uint32_t probe = 0; probe <= tmask; ++probe) {
      // a slot's key only ever changes from empty to its final value
      uint64_t cur = __hip_atomic_load(&tkeys[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (cur == ~0ull) {
        cur = atomicCAS((unsigned long long*)&tkeys[sl], ~0ull, (unsigned long long)key);
        if (cur == ~0ull) cur = key;
      }
      if (cur == key) {
        atomicAdd(&tcounts[sl], 1u);
        placed = true;
        break;
      }
      sl = (sl + 1) & tmask;
    }
    if (!placed) atomicOr(err, 2u);
  }
}

// ------------------------------------------------------------------ cell lists

// Cells with count >= min_count, in ascending order: block b owns cells [b chunk,
// (b + 1) chunk); pass 1 counts per block, pass 2 scans the block counts, pass 3 writes.
__global__ __launch_bounds__(256) void cell_list_count_kernel(const uint32_t* __restrict__ counts, uint64_t ncells,
                                                              uint64_t chunk, uint32_t min_count,
                                                              uint64_t* __restrict__ block_count) {
  __shared__ uint64_t part[256];
  const uint64_t lo = (uint64_t)blockIdx.x * chunk;
  const uint64_t hi = lo + chunk < ncells ? lo + chunk : ncells;
  uint64_t c = 0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) c += counts[i] >= min_count;
  part[threadIdx.x] = c;
  __syncthreads();
  for (uint32_t h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) block_count[blockIdx.x] = part[0];
}

// Exclusive scan of nb block counts in place (one workgroup of 1024); total in *total.
__global__ __launch_bounds__(1024) void scan_blocks_kernel(uint64_t* __restrict__ v, uint32_t nb,
                                                           unsigned long long* __restrict__ total) {
  __shared__ uint64_t part[1024];
  const uint32_t per = (nb + 1023) / 1024;
  const uint32_t lo = threadIdx.x * per, hi = lo + per < nb ? lo + per : nb;
  uint64_t s = 0;
  for (uint32_t i = lo; i < hi; ++i) s += v[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (uint32_t off = 1; off < 1024; off <<= 1) {   // inclusive Hillis-Steele scan
    const uint64_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  uint64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
  for (uint32_t i = lo; i < hi; ++i) {
    const uint64_t c = v[i];
    v[i] = run;
    run += c;
  }
  if (threadIdx.x == 1023) *total = part[1023];
}

__global__ __launch_bounds__(256) void cell_list_write_kernel(const uint32_t* __restrict__ counts, uint64_t ncells,
                                                              uint64_t chunk, uint32_t min_count,
                                                              const uint64_t* __restrict__ block_off,
                                                              uint64_t* __restrict__ cells, uint64_t cap) {
  __shared__ uint32_t wave_n[4];
  const uint64_t lo = (uint64_t)blockIdx.x * chunk;
  const uint64_t hi = lo + chunk < ncells ? lo + chunk : ncells;
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  uint64_t base = block_off[blockIdx.x];
  for (uint64_t t0 = lo; t0 < hi; t0 += blockDim.x) {   // uniform over the block
    const uint64_t i = t0 + threadIdx.x;
    const bool take = i < hi && counts[i] >= min_count;
    const uint64_t mask = __ballot(take);
    if (lane == 0) wave_n[wave] = (uint32_t)__popcll(mask);
    __syncthreads();
    uint64_t off = base;
    for (uint32_t q = 0; q < wave; ++q) off += wave_n[q];
    const uint64_t below = lane ? (mask & (~0ull >> (64 - lane))) : 0ull;
    off += (uint64_t)__popcll(below);
    if (take && off < cap) cells[off] = i;
    for (uint32_t q = 0; q < 4; ++q) base += wave_n[q];
    __syncthreads();
  }
}

// The same listing from the bitmap of touched cells: word w's bits are cells 32 w .. +31.
// Block b owns words [b chunk, (b + 1) chunk).
// Bits of word w that name cells below ncells (a caller's bitmap may carry stray bits in
// its last word or beyond).
__device__ __forceinline__ uint32_t valid_bits(uint32_t bits, uint64_t w, uint64_t ncells) {
  const uint64_t lo = w * 32;
  if (lo >= ncells) return 0u;
  const uint64_t left = ncells - lo;
  return left >= 32 ? bits : bits & ((1u << left) - 1u);
}

__device__ __forceinline__ uint32_t bits_taken(uint32_t bits, uint64_t w, const uint32_t* __restrict__ counts,
                                               uint32_t min_count) {
  if (min_count <= 1) return (uint32_t)__popc(bits);
  uint32_t q = 0;
  while (bits) {
    const uint32_t b = (uint32_t)__ffs(bits) - 1u;
    bits &= bits - 1u;
    q += counts[w * 32 + b] >= min_count;
  }
  return q;
}

// The bitmap listing reads kBitmapWPT consecutive words per thread (four 16-byte loads in
// flight when the bitmap is 16-byte aligned; chunks are whole multiples of it): at 10^9
// cells the bitmap is 125 MB and almost every word is zero, so the pass is a streaming read.
constexpr uint32_t kBitmapWPT = 16;

__device__ __forceinline__ void load_words(const uint32_t* __restrict__ bitmap, uint64_t w0, uint64_t hi,
                                           bool vec, uint32_t (&wd)[kBitmapWPT]) {
  if (vec && w0 + kBitmapWPT <= hi) {
#pragma unroll
    for (uint32_t k = 0; k < kBitmapWPT / 4; ++k) {
      const uint4 v = ((const uint4*)(bitmap + w0))[k];
      wd[4 * k] = v.x;
      wd[4 * k + 1] = v.y;
      wd[4 * k + 2] = v.z;
      wd[4 * k + 3] = v.w;
    }
  } else {
#pragma unroll
    for (uint32_t k = 0; k < kBitmapWPT; ++k) wd[k] = (w0 + k < hi) ? bitmap[w0 + k] : 0u;
  }
}

__global__ __launch_bounds__(256) void bitmap_list_count_kernel(const uint32_t* __restrict__ bitmap, uint64_t nwords,
                                                                uint64_t ncells, uint64_t chunk,
                                                                const uint32_t* __restrict__ counts,
                                                                uint32_t min_count,
                                                                uint64_t* __restrict__ block_count, uint32_t vec) {
  __shared__ uint64_t part[256];
  const uint64_t lo = (uint64_t)blockIdx.x * chunk;
  const uint64_t hi = lo + chunk < nwords ? lo + chunk : nwords;
  uint64_t c = 0;
  for (uint64_t w0 = lo + (uint64_t)threadIdx.x * kBitmapWPT; w0 < hi; w0 += (uint64_t)blockDim.x * kBitmapWPT) {
    uint32_t wd[kBitmapWPT];
    load_words(bitmap, w0, hi, vec != 0u, wd);
#pragma unroll
    for (uint32_t k = 0; k < kBitmapWPT; ++k) {
      const uint32_t bits = valid_bits(wd[k], w0 + k, ncells);
      if (bits) c += bits_taken(bits, w0 + k, counts, min_count);
    }
  }
  part[threadIdx.x] = c;
  __syncthreads();
  for (uint32_t h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) block_count[blockIdx.x] = part[0];
}

__global__ __launch_bounds__(256) void bitmap_list_write_kernel(const uint32_t* __restrict__ bitmap, uint64_t nwords,
                                                                uint64_t ncells, uint64_t chunk,
                                                                const uint32_t* __restrict__ counts,
                                                                uint32_t min_count,
                                                                const uint64_t* __restrict__ block_off,
                                                                uint64_t* __restrict__ cells, uint64_t cap,
                                                                uint32_t vec) {
  __shared__ uint32_t wsum[4];
  const uint64_t lo = (uint64_t)blockIdx.x * chunk;
  const uint64_t hi = lo + chunk < nwords ? lo + chunk : nwords;
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  uint64_t base = block_off[blockIdx.x];
  for (uint64_t t0 = lo; t0 < hi; t0 += (uint64_t)blockDim.x * kBitmapWPT) {   // uniform over the block
    const uint64_t w0 = t0 + (uint64_t)threadIdx.x * kBitmapWPT;   // this thread's words, in order
    uint32_t wd[kBitmapWPT];
    load_words(bitmap, w0, hi, vec != 0u, wd);
    uint32_t q = 0;
#pragma unroll
    for (uint32_t k = 0; k < kBitmapWPT; ++k) {
      wd[k] = valid_bits(wd[k], w0 + k, ncells);
      if (wd[k]) q += bits_taken(wd[k], w0 + k, counts, min_count);
    }
    const uint32_t incl = wave_incl_scan(q);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint64_t off = base + incl - q;
    uint64_t tile = 0;
    for (uint32_t v = 0; v < 4; ++v) {
      if (v < wave) off += wsum[v];
      tile += wsum[v];
    }
    if (q) {
      for (uint32_t k = 0; k < kBitmapWPT; ++k) {
        uint32_t rem = wd[k];
        while (rem) {
          const uint32_t b = (uint32_t)__ffs(rem) - 1u;
          rem &= rem - 1u;
          const uint64_t cell = (w0 + k) * 32 + b;
          if (min_count <= 1 || counts[cell] >= min_count) {
            if (off < cap) cells[off] = cell;
            ++off;
          }
        }
      }
    }
    base += tile;
    __syncthreads();
  }
}

// Zero the counts of every touched cell and the bitmap itself.
__global__ __launch_bounds__(256) void bitmap_clear_kernel(uint32_t* __restrict__ bitmap, uint64_t nwords,
                                                           uint64_t ncells, uint32_t* __restrict__ counts,
                                                           uint32_t vec) {
  // four words per thread: one 16-byte load (a 16-byte aligned bitmap), and a store only
  // where a word is set
  const uint64_t ng = (nwords + 3) / 4;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ng; i += stride) {
    uint32_t wd[4];
    if (vec && 4 * i + 4 <= nwords) {
      const uint4 v = ((const uint4*)bitmap)[i];
      wd[0] = v.x, wd[1] = v.y, wd[2] = v.z, wd[3] = v.w;
    } else {
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k) wd[k] = (4 * i + k < nwords) ? bitmap[4 * i + k] : 0u;
    }
    if ((wd[0] | wd[1] | wd[2] | wd[3]) == 0u) continue;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
      const uint64_t w = 4 * i + k;
      uint32_t bits = valid_bits(wd[k], w, ncells);
      while (bits) {
        const uint32_t b = (uint32_t)__ffs(bits) - 1u;
        bits &= bits - 1u;
        counts[w * 32 + b] = 0u;
      }
      if (wd[k]) bitmap[w] = 0u;
    }
  }
}

// ------------------------------------------------------------------ labels and admission

// out[i] = coarse parent (fine cell index / factor per axis on the mesh G / factor) of keys[i]
__global__ __launch_bounds__(256) void parent_kernel(const uint64_t* __restrict__ keys, uint32_t n, uint64_t G,
                                                     uint32_t factor, uint64_t* __restrict__ out) {
  const uint64_t Gc = G / factor;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    const uint64_t ix = k / (G * G), iy = (k / G) % G, iz = k % G;
    out[i] = ((ix / factor) * Gc + iy / factor) * Gc + iz / factor;
  }
}

// out[rank(i)] = in[i] with rank(i) = #{j : in[j] < in[i]} + #{j < i : in[j] == in[i]}:
// an ascending stable sort for short lists (quadratic work).
__global__ __launch_bounds__(256) void rank_sort_kernel(const uint64_t* __restrict__ in, uint32_t n,
                                                        uint64_t* __restrict__ out) {
  __shared__ uint64_t tile[256];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t v = i < n ? in[i] : 0;
  uint32_t r = 0;
  for (uint32_t j0 = 0; j0 < n; j0 += 256) {
    __syncthreads();
    if (j0 + threadIdx.x < n) tile[threadIdx.x] = in[j0 + threadIdx.x];
    __syncthreads();
    const uint32_t lim = n - j0 < 256 ? n - j0 : 256;
    for (uint32_t t = 0; t < lim; ++t) r += (tile[t] < v) || (tile[t] == v && j0 + t < i);
  }
  if (i < n) out[r] = v;
}

// labels[j] = 1 if cells[j] is in the ascending list par[0 .. np), else 0
__global__ __launch_bounds__(256) void label_kernel(const uint64_t* __restrict__ cells, uint64_t m,
                                                    const uint64_t* __restrict__ par, uint32_t np,
                                                    float* __restrict__ labels) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
    const uint64_t c = cells[j];
    uint32_t lo = 0, hi = np;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (par[mid] < c) lo = mid + 1;
      else hi = mid;
    }
    labels[j] = (lo < np && par[lo] == c) ? 1.0f : 0.0f;
  }
}

// An int32 whose signed order is the order of the float logits (-0 taken as +0), so that
// the radix select of the top-k ranks cells by logit.
__global__ __launch_bounds__(256) void logit_order_kernel(const float* __restrict__ z, uint64_t m,
                                                          int32_t* __restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
    uint32_t u = __float_as_uint(z[j]);
    if (u == 0x80000000u) u = 0u;
    const uint32_t ord = (u & 0x80000000u) ? ~u : (u | 0x80000000u);   // unsigned order of the floats
    out[j] = (int32_t)(ord ^ 0x80000000u);
  }
}

// The same for the cells j < min(*m, cap) of a device count.
__global__ __launch_bounds__(256) void logit_order_dev_kernel(const float* __restrict__ z,
                                                              const uint64_t* __restrict__ m_dev, uint64_t cap,
                                                              int32_t* __restrict__ out) {
  const uint64_t m = *m_dev < cap ? *m_dev : cap;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
    uint32_t u = __float_as_uint(z[j]);
    if (u == 0x80000000u) u = 0u;
    const uint32_t ord = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    out[j] = (int32_t)(ord ^ 0x80000000u);
  }
}

// The n = min(winners, A) admitted keys in ascending order (the ranks of rank_sort_kernel
// over a device count); *na = n.
__global__ __launch_bounds__(256) void admit_sort_kernel(const uint64_t* __restrict__ in, const SelState* st, uint32_t A,
                                                         uint64_t* __restrict__ out, uint32_t* __restrict__ na) {
  __shared__ uint64_t tile[256];
  const uint32_t n = st->n_sel < A ? st->n_sel : A;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t v = i < n ? in[i] : 0;
  uint32_t r = 0;
  for (uint32_t j0 = 0; j0 < n; j0 += 256) {
    __syncthreads();
    if (j0 + threadIdx.x < n) tile[threadIdx.x] = in[j0 + threadIdx.x];
    __syncthreads();
    const uint32_t lim = n - j0 < 256 ? n - j0 : 256;
    for (uint32_t t = 0; t < lim; ++t) r += (tile[t] < v) || (tile[t] == v && j0 + t < i);
  }
  if (i < n) out[r] = v;
  if (i == 0) *na = n;
}

// The exclusion's child counters into the exact table: child e = position * f3 + c of the
// admitted cell admitted[position] with a nonzero count is added under its fine key
// (linear probing from table_slot; bit 1 of *err if the table is full).
__global__ __launch_bounds__(256) void route_table_kernel(RouteExclude ex, uint32_t G, uint64_t* __restrict__ tkeys,
                                                          uint32_t* __restrict__ tcounts, uint32_t tmask,
                                                          uint32_t* __restrict__ err) {
  const uint32_t na = *ex.na < ex.na_max ? *ex.na : ex.na_max;
  const uint32_t nd = na * ex.f3;
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < nd; e += gridDim.x * blockDim.x) {
    const uint32_t cnt = ex.child[e];
    if (cnt == 0) continue;
    const uint32_t f = ex.factor, c = e % ex.f3;
    const uint64_t Gc = ex.gc, P = ex.admitted[e / ex.f3];
    const uint64_t px = P / (Gc * Gc), py = (P / Gc) % Gc, pz = P % Gc;
    const uint64_t ix = px * f + c / (f * f), iy = py * f + (c / f) % f, iz = pz * f + c % f;
    const uint64_t key = (ix * G + iy) * G + iz;
    uint32_t sl = table_slot(key, tmask);
    bool placed = false;
    for (uint32_t probe = 0; probe <= tmask; ++probe) {
      uint64_t cur = __hip_atomic_load(&tkeys[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (cur == ~0ull) {
        cur = atomicCAS((unsigned long long*)&tkeys[sl], ~0ull, (unsigned long long)key);
        if (cur == ~0ull) cur = key;
      }
      if (cur == key) {
        atomicAdd(&tcounts[sl], cnt);
        placed = true;
        break;
      }
      sl = (sl + 1) & tmask;
    }
    if (!placed) atomicOr(err, 2u);
  }
}

// ------------------------------------------------------------------ launchers

static uint32_t grid_of(uint64_t n, uint32_t threads, uint32_t max_blocks) {
  uint64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return (uint32_t)b;
}

hipError_t launch_sample_counts(const float* pos, uint64_t n, uint64_t index0, uint64_t seed, uint32_t threshold,
                                const Mesh& coarse, uint32_t* counts, uint32_t* bitmap, hipStream_t s) {
  hipLaunchKernelGGL(sample_counts_kernel, dim3(grid_of(n / (4 * kSampleU) + 2, 256, 8192)), dim3(256), 0, s, pos, n,
                     index0, seed,
                     threshold, coarse, counts, bitmap);
  return hipGetLastError();
}

hipError_t launch_features(const uint32_t* counts, uint32_t Gc, const uint64_t* cells, uint64_t m, float* feat,
                           hipStream_t s) {
  hipLaunchKernelGGL(features_kernel, dim3(grid_of(m, 256, 8192)), dim3(256), 0, s, counts, Gc, cells, m, feat);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16(uint32_t M, uint32_t N, uint32_t K, const float* A, uint64_t sai, uint64_t sak,
                            const float* B, uint64_t sbk, uint64_t sbj, float* C, uint64_t sci, uint64_t scj,
                            float beta, hipStream_t s, float* partial, uint64_t partial_floats, bool split) {
  const uint64_t tiles = (uint64_t)((M + 15) / 16) * ((N + 15) / 16);
  uint64_t nsplit = (K + kSplitK - 1) / kSplitK;
  if (partial != nullptr && (uint64_t)M * N > 0 && nsplit * (uint64_t)M * N > partial_floats)
    nsplit = partial_floats / ((uint64_t)M * N);
  if (split) {   // the scoring pass: no split over k
    hipLaunchKernelGGL(gemm_bf16_kernel<true>, dim3((uint32_t)((tiles + 3) / 4)), dim3(256), 0, s, M, N, K, A, sai,
                       sak, B, sbk, sbj, C, sci, scj, beta);
    return hipGetLastError();
  }
  if (partial == nullptr || K < 2 * kSplitK || tiles >= 256 || nsplit < 2) {
    hipLaunchKernelGGL(gemm_bf16_kernel<false>, dim3((uint32_t)((tiles + 3) / 4)), dim3(256), 0, s, M, N, K, A, sai,
                       sak, B, sbk, sbj, C, sci, scj, beta);
    return hipGetLastError();
  }
  const uint32_t kc = (uint32_t)(((K + nsplit - 1) / nsplit + 31) / 32 * 32);
  nsplit = (K + kc - 1) / kc;
  hipLaunchKernelGGL(gemm_bf16_splitk_kernel, dim3((uint32_t)((tiles + 3) / 4), (uint32_t)nsplit), dim3(256), 0, s, M,
                     N, K, kc, A, sai, sak, B, sbk, sbj, partial);
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid_of((uint64_t)M * N, 256, 1024)), dim3(256), 0, s, partial,
                     (uint32_t)nsplit, M, N, C, sci, scj, beta);
  return hipGetLastError();
}

hipError_t launch_bias_act(float* Y, uint32_t M, uint32_t N, const float* bias, bool relu, hipStream_t s) {
  hipLaunchKernelGGL(bias_act_kernel, dim3(grid_of((uint64_t)M * N, 256, 4096)), dim3(256), 0, s, Y, M, N, bias,
                     relu ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_head(const float* H2, uint32_t M, const float* w3, const float* b3, float* z, const float* y,
                       float* dz, float* loss, bool round, hipStream_t s) {
  hipLaunchKernelGGL(head_kernel, dim3(grid_of(M, 256, 4096)), dim3(256), 0, s, H2, M, w3, b3, z, y, dz, loss,
                     round ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_head_back(const float* dz, const float* H2, const float* w3, uint32_t M, float* dA, hipStream_t s) {
  hipLaunchKernelGGL(head_back_kernel, dim3(grid_of((uint64_t)M * kHidden, 256, 4096)), dim3(256), 0, s, dz, H2, w3, M,
                     dA);
  return hipGetLastError();
}

hipError_t launch_relu_back(float* dA, const float* H, uint64_t total, hipStream_t s) {
  hipLaunchKernelGGL(relu_back_kernel, dim3(grid_of(total, 256, 4096)), dim3(256), 0, s, dA, H, total);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* X, uint32_t M, uint32_t N, uint32_t ld, const float* w, float* out, hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel, dim3(N), dim3(256), 0, s, X, M, N, ld, w, out);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m1, float* m2, uint32_t n, float lr_t, float b1, float b2,
                       float eps, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(grid_of(n, 256, 1024)), dim3(256), 0, s, p, g, m1, m2, n, lr_t, b1, b2, eps);
  return hipGetLastError();
}

// Waves and particles per wave of a split of n particles.
uint32_t split_waves(uint64_t n, uint64_t* wchunk) {
  const uint64_t tiles = (n + kSplitWaveTile - 1) / kSplitWaveTile;
  uint64_t nw = tiles < kSplitMaxWaves ? tiles : kSplitMaxWaves;
  if (nw < 1) nw = 1;
  *wchunk = (tiles + nw - 1) / nw * kSplitWaveTile;
  return (uint32_t)nw;
}

uint64_t split_workspace_bytes(uint32_t na, uint32_t factor) {
  const uint64_t blocks = kSplitMaxWaves / (kSplitThreads / 64);
  return kSplitMaxWaves * sizeof(uint64_t) + blocks * na * factor * factor * factor * sizeof(uint32_t);
}

hipError_t launch_route_split(const float* pos, uint64_t n, const Mesh& mesh, uint32_t factor, const uint64_t* admitted,
                              uint32_t na, uint64_t* tkeys, uint32_t* tcounts, uint32_t tmask, float* rest_pos,
                              unsigned long long* rest_count, uint32_t* err, void* workspace, hipStream_t s) {
  SplitArgs a;
  a.pos = pos;
  a.n = n;
  a.mesh = mesh;
  a.factor = factor;
  a.fmagic = (uint32_t)(((1ull << 32) + factor - 1) / factor);
  a.f3 = factor * factor * factor;
  a.admitted = admitted;
  a.na = na;
  a.nwaves = split_waves(n, &a.wchunk);
  const uint32_t nb = (a.nwaves + kSplitThreads / 64 - 1) / (kSplitThreads / 64);
  uint64_t* wave = (uint64_t*)workspace;
  uint32_t* dense_part = (uint32_t*)(wave + kSplitMaxWaves);
  const uint32_t nd = na * a.f3;
  const size_t lds = (size_t)nd * sizeof(uint32_t);
  if (mesh.mode == kMeshPow2Ratio) {
    hipLaunchKernelGGL(split_count_kernel<kMeshPow2Ratio>, dim3(nb), dim3(kSplitThreads), 0, s, a, wave, err);
    hipLaunchKernelGGL(split_scan_kernel, dim3(1), dim3(1024), 0, s, wave, a.nwaves, rest_count);
    hipLaunchKernelGGL(split_write_kernel<kMeshPow2Ratio>, dim3(nb), dim3(kSplitThreads), lds, s, a, wave, rest_pos,
                       dense_part);
  } else if (mesh.mode == kMeshExactRatio) {
    hipLaunchKernelGGL(split_count_kernel<kMeshExactRatio>, dim3(nb), dim3(kSplitThreads), 0, s, a, wave, err);
    hipLaunchKernelGGL(split_scan_kernel, dim3(1), dim3(1024), 0, s, wave, a.nwaves, rest_count);
    hipLaunchKernelGGL(split_write_kernel<kMeshExactRatio>, dim3(nb), dim3(kSplitThreads), lds, s, a, wave, rest_pos,
                       dense_part);
  } else {
    hipLaunchKernelGGL(split_count_kernel<kMeshGeneral>, dim3(nb), dim3(kSplitThreads), 0, s, a, wave, err);
    hipLaunchKernelGGL(split_scan_kernel, dim3(1), dim3(1024), 0, s, wave, a.nwaves, rest_count);
    hipLaunchKernelGGL(split_write_kernel<kMeshGeneral>, dim3(nb), dim3(kSplitThreads), lds, s, a, wave, rest_pos,
                       dense_part);
  }
  if (nd > 0)
    hipLaunchKernelGGL(split_table_kernel, dim3(grid_of(nd, 256, 1024)), dim3(256), 0, s, a, dense_part, nb, tkeys,
                       tcounts, tmask, err);
  return hipGetLastError();
}

hipError_t launch_exact_count(const float* pos, uint64_t n, const Mesh& mesh, uint64_t* tkeys, uint32_t* tcounts,
                              uint32_t tmask, uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(exact_count_kernel, dim3(grid_of(n, 256, 16384)), dim3(256), 0, s, pos, n, mesh, tkeys, tcounts,
                     tmask, err);
  return hipGetLastError();
}

uint32_t cell_list_blocks(uint64_t ncells, uint64_t* chunk) {
  uint64_t nb = (ncells + 4095) / 4096;
  if (nb > kCellListBlocks) nb = kCellListBlocks;
  if (nb < 1) nb = 1;
  *chunk = (ncells + nb - 1) / nb;
  return (uint32_t)nb;
}

hipError_t launch_cell_list(const uint32_t* counts, uint64_t ncells, uint32_t min_count, const uint32_t* bitmap,
                            uint64_t* block_scratch, uint64_t* cells, uint64_t cap, unsigned long long* total,
                            hipStream_t s) {
  uint64_t chunk = 0;
  if (bitmap != nullptr) {
    const uint64_t nwords = (ncells + 31) / 32;
    const uint32_t nb = cell_list_blocks(nwords, &chunk);
    chunk = (chunk + kBitmapWPT - 1) / kBitmapWPT * kBitmapWPT;   // aligned loads; trailing blocks may be empty
    const uint32_t vec = ((uintptr_t)bitmap & 15u) == 0 ? 1u : 0u;
    hipLaunchKernelGGL(bitmap_list_count_kernel, dim3(nb), dim3(256), 0, s, bitmap, nwords, ncells, chunk, counts,
                       min_count, block_scratch, vec);
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(1024), 0, s, block_scratch, nb, total);
    hipLaunchKernelGGL(bitmap_list_write_kernel, dim3(nb), dim3(256), 0, s, bitmap, nwords, ncells, chunk, counts,
                       min_count, block_scratch, cells, cap, vec);
    return hipGetLastError();
  }
  const uint32_t nb = cell_list_blocks(ncells, &chunk);
  hipLaunchKernelGGL(cell_list_count_kernel, dim3(nb), dim3(256), 0, s, counts, ncells, chunk, min_count,
                     block_scratch);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(1024), 0, s, block_scratch, nb, total);
  hipLaunchKernelGGL(cell_list_write_kernel, dim3(nb), dim3(256), 0, s, counts, ncells, chunk, min_count,
                     block_scratch, cells, cap);
  return hipGetLastError();
}

hipError_t launch_bitmap_clear(uint32_t* bitmap, uint64_t ncells, uint32_t* counts, hipStream_t s) {
  const uint64_t nwords = (ncells + 31) / 32;
  const uint32_t vec = ((uintptr_t)bitmap & 15u) == 0 ? 1u : 0u;
  hipLaunchKernelGGL(bitmap_clear_kernel, dim3(grid_of((nwords + 3) / 4, 256, 8192)), dim3(256), 0, s, bitmap, nwords,
                     ncells, counts, vec);
  return hipGetLastError();
}

hipError_t launch_parents_sorted(const uint64_t* keys, uint32_t n, uint64_t G, uint32_t factor, uint64_t* tmp,
                                 uint64_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(parent_kernel, dim3(grid_of(n, 256, 1024)), dim3(256), 0, s, keys, n, G, factor, tmp);
  hipLaunchKernelGGL(rank_sort_kernel, dim3((n + 255) / 256), dim3(256), 0, s, tmp, n, out);
  return hipGetLastError();
}

hipError_t launch_rank_sort(const uint64_t* in, uint32_t n, uint64_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(rank_sort_kernel, dim3((n + 255) / 256), dim3(256), 0, s, in, n, out);
  return hipGetLastError();
}

hipError_t launch_labels(const uint64_t* cells, uint64_t m, const uint64_t* par, uint32_t np, float* labels,
                         hipStream_t s) {
  hipLaunchKernelGGL(label_kernel, dim3(grid_of(m, 256, 8192)), dim3(256), 0, s, cells, m, par, np, labels);
  return hipGetLastError();
}

hipError_t launch_logit_order(const float* z, uint64_t m, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(logit_order_kernel, dim3(grid_of(m, 256, 8192)), dim3(256), 0, s, z, m, out);
  return hipGetLastError();
}

hipError_t launch_route_score(const uint32_t* counts, uint32_t Gc, const uint64_t* cells, const uint64_t* m_dev,
                              uint64_t cap, const float* params, float* z, hipStream_t s) {
  if (cap == 0) return hipSuccess;
  hipLaunchKernelGGL(route_score_kernel, dim3(grid_of(cap, kScoreThreads, 2048)), dim3(kScoreThreads), 0, s, counts, Gc,
                     cells, m_dev, cap, params, z);
  return hipGetLastError();
}

hipError_t launch_admit_dev(const uint64_t* cells, const float* logits, const uint64_t* m_dev, uint64_t cap, uint32_t A,
                            int32_t* ord, SelState* st, uint64_t* sk, int32_t* se, uint32_t* rank, uint64_t* ok,
                            int32_t* oe, uint32_t* err, uint64_t* admitted, uint32_t* na, hipStream_t s) {
  hipLaunchKernelGGL(logit_order_dev_kernel, dim3(grid_of(cap, 256, 8192)), dim3(256), 0, s, logits, m_dev, cap, ord);
  hipError_t e = launch_select_pairs_dev(cells, ord, m_dev, (uint32_t)cap, A, st, sk, se, rank, ok, oe, err, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(admit_sort_kernel, dim3((A + 255) / 256), dim3(256), 0, s, ok, st, A, admitted, na);
  return hipGetLastError();
}

hipError_t launch_route_table(const RouteExclude& ex, uint32_t G, uint64_t* tkeys, uint32_t* tcounts, uint32_t tmask,
                              uint32_t* err, hipStream_t s) {
  const uint32_t nd = ex.na_max * ex.f3;
  if (nd == 0) return hipSuccess;
  hipLaunchKernelGGL(route_table_kernel, dim3(grid_of(nd, 256, 1024)), dim3(256), 0, s, ex, G, tkeys, tcounts, tmask,
                     err);
  return hipGetLastError();
}

}  // namespace csk
