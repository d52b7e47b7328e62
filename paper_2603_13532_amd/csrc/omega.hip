// Seeded Gaussian test matrices Omega_k (Section 3.1: one standard Gaussian
// matrix per mode, reused by every sketch S_n with n != k).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) gives four 32-bit words
// per 128-bit counter; two 53-bit uniforms feed one Box-Muller pair in FP64;
// the pair fills two consecutive column-major entries.  Values are rounded
// to 8 significant bits (nearest even) on the FP64 bit pattern, so every
// precision form sketches with the same, BF16-exact matrix.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace tsk {

namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

__device__ __forceinline__ void philox_round(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
  const uint32_t hi0 = __umulhi(kPhiloxM0, c[0]);
  const uint32_t lo0 = kPhiloxM0 * c[0];
  const uint32_t hi1 = __umulhi(kPhiloxM1, c[2]);
  const uint32_t lo1 = kPhiloxM1 * c[2];
  const uint32_t n0 = hi1 ^ c[1] ^ k0;
  const uint32_t n2 = hi0 ^ c[3] ^ k1;
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

__device__ __forceinline__ double round_8bit_significand(double x) {
  uint64_t b = (uint64_t)__double_as_longlong(x);
  b = (b + ((1ull << 44) - 1ull) + ((b >> 45) & 1ull)) & ~((1ull << 45) - 1ull);
  return __longlong_as_double((long long)b);
}

__device__ __forceinline__ void omega_pair(uint64_t seed, uint32_t mode, int64_t p, double& z0,
                                           double& z1) {
  uint32_t c[4] = {(uint32_t)((uint64_t)p & 0xFFFFFFFFull), (uint32_t)((uint64_t)p >> 32), mode, 0u};
  uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFull), k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    philox_round(c, k0, k1);
  }
  const uint64_t w0 = ((uint64_t)c[1] << 32) | c[0];
  const uint64_t w1 = ((uint64_t)c[3] << 32) | c[2];
  const double u1 = (double)((w0 >> 11) + 1ull) * 0x1.0p-53;
  const double u2 = (double)(w1 >> 11) * 0x1.0p-53;
  const double rho = sqrt(-2.0 * log(u1));
  const double ang = (2.0 * 3.141592653589793) * u2;
  z0 = round_8bit_significand(rho * cos(ang));
  z1 = round_8bit_significand(rho * sin(ang));
}

template <typename T>
__device__ __forceinline__ void omega_fill(uint64_t seed, uint32_t mode, int64_t count, T* out,
                                           int64_t first, int64_t stride) {
  const int64_t pairs = (count + 1) / 2;
  for (int64_t p = first; p < pairs; p += stride) {
    double z0, z1;
    omega_pair(seed, mode, p, z0, z1);
    const int64_t e = 2 * p;
    out[e] = (T)z0;
    if (e + 1 < count) out[e + 1] = (T)z1;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void omega_kernel(uint64_t seed, uint32_t mode, int64_t count,
                                                    T* __restrict__ out) {
  omega_fill<T>(seed, mode, count, out, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                (int64_t)gridDim.x * blockDim.x);
}

// Many matrices in one launch: blockIdx.y selects the job.
__global__ __launch_bounds__(256) void omega_jobs_kernel(const OmegaJobDev* __restrict__ jobs) {
  const OmegaJobDev J = jobs[blockIdx.y];
  const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (J.f64) omega_fill<double>(J.seed, (uint32_t)J.mode, J.count, (double*)J.out, first, stride);
  else omega_fill<float>(J.seed, (uint32_t)J.mode, J.count, (float*)J.out, first, stride);
}

}  // namespace

hipError_t launch_omega_jobs(const OmegaJobDev* jobs, int count, int64_t max_count,
                             hipStream_t stream) {
  if (count <= 0 || max_count <= 0) return hipSuccess;
  int64_t blocks = ((max_count + 1) / 2 + 255) / 256;
  if (blocks > 64) blocks = 64;
  omega_jobs_kernel<<<dim3((unsigned)blocks, (unsigned)count), dim3(256), 0, stream>>>(jobs);
  return hipGetLastError();
}

hipError_t launch_omega(uint64_t seed, int mode, int64_t rows, int64_t cols, void* out, bool f64,
                        hipStream_t stream) {
  const int64_t count = rows * cols;
  if (count <= 0) return hipSuccess;
  const int64_t pairs = (count + 1) / 2;
  int64_t blocks = (pairs + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (f64)
    omega_kernel<double><<<dim3((unsigned)blocks), dim3(256), 0, stream>>>(seed, (uint32_t)mode,
                                                                            count, (double*)out);
  else
    omega_kernel<float><<<dim3((unsigned)blocks), dim3(256), 0, stream>>>(seed, (uint32_t)mode,
                                                                           count, (float*)out);
  return hipGetLastError();
}

}  // namespace tsk
