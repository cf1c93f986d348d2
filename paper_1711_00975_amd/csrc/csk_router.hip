// csk_router.hip — kernels of the learned router: a 1 % sample pre-pass gives coarse
// cell counts, a 27 -> 64 -> 64 -> 1 MLP (bf16 operands on MFMA, fp32 accumulation)
// scores coarse cells, the highest-scored ones are counted exactly in a device hash table
// and every other particle goes on to a Count Sketch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csk_router.h"

namespace csk {

// ------------------------------------------------------------------ sampling

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4x32 bijection with the
// published multipliers and Weyl key increments.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Particle index0 + i is in the sample when the first Philox word of counter
// (index lo, index hi, kSampleStream, 0) under the seed is below `threshold`.
__global__ __launch_bounds__(256) void sample_counts_kernel(const float* __restrict__ pos, uint64_t n, uint64_t index0,
                                                            uint64_t seed, uint32_t threshold, Mesh coarse,
                                                            uint32_t* __restrict__ counts) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t g = index0 + i;
    uint32_t c[4] = {(uint32_t)g, (uint32_t)(g >> 32), kSampleStream, 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    if (c[0] >= threshold) continue;
    uint64_t key;
    if (cell_key(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], coarse, key)) atomicAdd(&counts[key], 1u);
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

// ------------------------------------------------------------------ MLP

// fp32 -> bf16, round to nearest even (finite inputs)
__device__ __forceinline__ short to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// C[i][j] = beta * C[i][j] + sum_k A(i, k) * B(k, j) for i < M, j < N, with
// A(i, k) = A[i * sai + k * sak], B(k, j) = B[k * sbk + j * sbj] read as fp32 and rounded
// to bf16, products accumulated in fp32 by v_mfma_f32_16x16x16_bf16.  One wave per 16x16
// tile of C; elements outside the matrices read as 0 and are not written.
// Lane l of the MFMA holds A rows l % 16, k = 4 (l / 16) .. +3; B columns l % 16 at the
// same k; the result rows 4 (l / 16) .. +3 of column l % 16.
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
  const uint32_t r = lane & 15u, kq = (lane >> 4) * 4;
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (uint32_t k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t k = k0 + kq + (uint32_t)e;
      const uint32_t ia = i0 + r, jb = j0 + r;
      a[e] = to_bf16((ia < M && k < K) ? A[ia * sai + k * sak] : 0.0f);
      b[e] = to_bf16((jb < N && k < K) ? B[k * sbk + jb * sbj] : 0.0f);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t i = i0 + kq + (uint32_t)e, j = j0 + r;
    if (i < M && j < N) {
      float* c = C + i * sci + j * scj;
      *c = (beta != 0.0f ? beta * *c : 0.0f) + acc[e];
    }
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

// Output layer and loss: z[i] = H2[i] . w3 + b3 (w3 rounded to bf16, fp32 sums); with
// labels y, dz[i] = (sigmoid(z) - y) / M and loss[0] += mean binary cross-entropy.
__global__ __launch_bounds__(256) void head_kernel(const float* __restrict__ H2, uint32_t M, const float* __restrict__ w3,
                                                   const float* __restrict__ b3, float* __restrict__ z,
                                                   const float* __restrict__ y, float* __restrict__ dz,
                                                   float* __restrict__ loss) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < M; i += gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int j = 0; j < kHidden; ++j) {
      const float wj = __uint_as_float((uint32_t)(uint16_t)to_bf16(w3[j]) << 16);
      const float hj = __uint_as_float((uint32_t)(uint16_t)to_bf16(H2[(uint64_t)i * kHidden + j]) << 16);
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

// Every in-domain particle whose coarse parent (fine index / factor on each axis) is in
// the sorted list `admitted` adds 1 to its fine key's entry of the exact table; every
// other in-domain particle is appended to rest_pos (count in *rest_count).  Particles
// outside the domain latch kErrDomain in *err and go nowhere.
__global__ __launch_bounds__(256) void route_split_kernel(const float* __restrict__ pos, uint64_t n, Mesh mesh,
                                                          uint32_t factor, const uint64_t* __restrict__ admitted,
                                                          uint32_t na, uint64_t* __restrict__ tkeys,
                                                          uint32_t* __restrict__ tcounts, uint32_t tmask,
                                                          float* __restrict__ rest_pos,
                                                          unsigned long long* __restrict__ rest_count,
                                                          uint32_t* __restrict__ err) {
  __shared__ uint64_t adm[kMaxAdmitted];
  for (uint32_t i = threadIdx.x; i < na; i += blockDim.x) adm[i] = admitted[i];
  __syncthreads();
  const uint64_t G = (uint64_t)mesh.G, Gc = G / factor;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t n_round = (n + blockDim.x - 1) / blockDim.x * blockDim.x;   // whole waves for the append
  for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x; i0 < n_round; i0 += stride) {
    const uint64_t i = i0 + threadIdx.x;
    bool rest = false;
    float x = 0.0f, y = 0.0f, z = 0.0f;
    if (i < n) {
      x = pos[3 * i];
      y = pos[3 * i + 1];
      z = pos[3 * i + 2];
      uint64_t key;
      if (!cell_key(x, y, z, mesh, key)) {
        atomicOr(err, 1u);
      } else {
        const uint64_t ix = key / (G * G), iy = (key / G) % G, iz = key % G;
        const uint64_t ckey = ((ix / factor) * Gc + iy / factor) * Gc + iz / factor;
        uint32_t lo = 0, hi = na;   // binary search in the sorted admitted list
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (adm[mid] < ckey) lo = mid + 1;
          else hi = mid;
        }
        if (lo < na && adm[lo] == ckey) {
          uint32_t sl = table_slot(key, tmask);
          for (uint32_t probe = 0; probe <= tmask; ++probe) {
            const unsigned long long old = atomicCAS((unsigned long long*)&tkeys[sl], ~0ull, (unsigned long long)key);
            if (old == ~0ull || old == key) {
              atomicAdd(&tcounts[sl], 1u);
              break;
            }
            sl = (sl + 1) & tmask;
            if (probe == tmask) atomicOr(err, 2u);   // table full (admission keeps it at most half full)
          }
        } else {
          rest = true;
        }
      }
    }
    // wave-aggregated append of the rest
    const uint64_t mask = __ballot(rest);
    if (mask) {
      const uint32_t lane = threadIdx.x & 63u;
      const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1u;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(rest_count, (unsigned long long)__popcll(mask));
      base = __shfl(base, (int)leader, 64);
      if (rest) {
        const uint64_t below = (lane == 0) ? 0ull : (mask & ((~0ull) >> (64 - lane)));
        const uint64_t o = base + (uint64_t)__popcll(below);
        rest_pos[3 * o] = x;
        rest_pos[3 * o + 1] = y;
        rest_pos[3 * o + 2] = z;
      }
    }
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
                                const Mesh& coarse, uint32_t* counts, hipStream_t s) {
  hipLaunchKernelGGL(sample_counts_kernel, dim3(grid_of(n, 256, 8192)), dim3(256), 0, s, pos, n, index0, seed,
                     threshold, coarse, counts);
  return hipGetLastError();
}

hipError_t launch_features(const uint32_t* counts, uint32_t Gc, const uint64_t* cells, uint64_t m, float* feat,
                           hipStream_t s) {
  hipLaunchKernelGGL(features_kernel, dim3(grid_of(m, 256, 8192)), dim3(256), 0, s, counts, Gc, cells, m, feat);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16(uint32_t M, uint32_t N, uint32_t K, const float* A, uint64_t sai, uint64_t sak,
                            const float* B, uint64_t sbk, uint64_t sbj, float* C, uint64_t sci, uint64_t scj,
                            float beta, hipStream_t s) {
  const uint64_t tiles = (uint64_t)((M + 15) / 16) * ((N + 15) / 16);
  hipLaunchKernelGGL(gemm_bf16_kernel, dim3((uint32_t)((tiles + 3) / 4)), dim3(256), 0, s, M, N, K, A, sai, sak, B,
                     sbk, sbj, C, sci, scj, beta);
  return hipGetLastError();
}

hipError_t launch_bias_act(float* Y, uint32_t M, uint32_t N, const float* bias, bool relu, hipStream_t s) {
  hipLaunchKernelGGL(bias_act_kernel, dim3(grid_of((uint64_t)M * N, 256, 4096)), dim3(256), 0, s, Y, M, N, bias,
                     relu ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_head(const float* H2, uint32_t M, const float* w3, const float* b3, float* z, const float* y,
                       float* dz, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(head_kernel, dim3(grid_of(M, 256, 4096)), dim3(256), 0, s, H2, M, w3, b3, z, y, dz, loss);
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

hipError_t launch_route_split(const float* pos, uint64_t n, const Mesh& mesh, uint32_t factor, const uint64_t* admitted,
                              uint32_t na, uint64_t* tkeys, uint32_t* tcounts, uint32_t tmask, float* rest_pos,
                              unsigned long long* rest_count, uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(route_split_kernel, dim3(grid_of(n, 256, 8192)), dim3(256), 0, s, pos, n, mesh, factor, admitted,
                     na, tkeys, tcounts, tmask, rest_pos, rest_count, err);
  return hipGetLastError();
}

}  // namespace csk
