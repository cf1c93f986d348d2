// plummer_gpu.hip — the mixture recipe of plummer.c on the GPU, for streams too large to
// generate on the host (2^34 particles in 2^27-particle chunks).  Same Philox4x32-10
// draws (key = seed, counter = (index, stream 1, draw)), same alias records (built on the
// host by wl_alias_records), same per-particle arithmetic in binary64.  The device's pow,
// sqrt and sincos may differ from the host libm in the last bit, so a float32 position
// may rarely differ from the host generator's; every comparison feeds both sides the
// bytes this generator wrote.
//
// Holds no arithmetic of the sketch method: it only writes positions.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

struct AliasRec {
  double own[3];
  double alt[3];
  double prob;
  double pad;
};

__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
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

__device__ __forceinline__ double u01(uint32_t x) { return ((double)x + 0.5) * (1.0 / 4294967296.0); }

__device__ __forceinline__ float wrap_to_float(double x, double L) {
  if (x >= L || x < 0.0) {
    x = fmod(x, L);
    if (x < 0.0) x += L;
  }
  return (float)x;
}

__global__ __launch_bounds__(256) void gen_mixture_kernel(uint64_t start, uint64_t n, double L, uint32_t n_halo,
                                                          double a, double f_bg, uint64_t seed, double u_max,
                                                          const AliasRec* __restrict__ rec, float* __restrict__ pos) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t jj = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; jj < n; jj += stride) {
    const uint64_t i = start + jj;
    uint32_t r[4] = {(uint32_t)i, (uint32_t)(i >> 32), 1u, 0u};
    philox(r, k0, k1);
    float* out = pos + 3 * jj;
    if (n_halo == 0 || u01(r[0]) < f_bg) {
      for (int c = 0; c < 3; ++c) out[c] = wrap_to_float(u01(r[1 + c]) * L, L);
    } else {
      uint32_t q[4] = {(uint32_t)i, (uint32_t)(i >> 32), 1u, 1u};
      philox(q, k0, k1);
      const uint32_t col = (uint32_t)(((uint64_t)r[1] * n_halo) >> 32);
      const AliasRec& rc = rec[col];
      const double* cc = (u01(r[2]) < rc.prob) ? rc.own : rc.alt;
      const double u = u01(r[3]) * u_max;
      const double rad = a / sqrt(pow(u, -2.0 / 3.0) - 1.0);
      const double ct = 2.0 * u01(q[0]) - 1.0;
      const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
      double sp, cp;
      sincos(2.0 * M_PI * u01(q[1]), &sp, &cp);
      out[0] = wrap_to_float(cc[0] + rad * st * cp, L);
      out[1] = wrap_to_float(cc[1] + rad * st * sp, L);
      out[2] = wrap_to_float(cc[2] + rad * ct, L);
    }
  }
}

}  // namespace

// Particles [start, start + n) of the mixture stream into pos (device, n x 3 float32), with
// the alias records rec (device, n_halo records of 8 doubles).  u_max = 1.01^(-3/2).
// Returns 0, or the HIP error code of the launch.
extern "C" int wl_gen_mixture_device(uint64_t start, uint64_t n, double L, uint32_t n_halo, double a, double f_bg,
                                     uint64_t seed, double u_max, const void* rec, float* pos, void* stream) {
  if (n == 0) return 0;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(gen_mixture_kernel, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream, start, n, L,
                     n_halo, a, f_bg, seed, u_max, (const AliasRec*)rec, pos);
  return (int)hipGetLastError();
}
