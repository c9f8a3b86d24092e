// Counter-based standard normal noise for the Brownian terms (W^(r), W^(w) of
// Sections 3.1 and 3.3, W and W~ of the EM-RFD step, Section 4.4).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter (c0, c1, c2, c3),
// key (k0, k1); each of ten rounds forms the 64-bit products M0 c0 and M1 c2 and
// returns (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the
// key advances by the Weyl constants between rounds.  Two 53-bit uniforms per
// output give two normals by the Box-Muller transform.  Every element is a pure
// function of (seed, stream, draw counter, index): no state on the device, any
// thread count, bit-reproducible.
#include "kernels.h"

namespace fbim {
namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c.x;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return c;
}

__device__ __forceinline__ uint4 philox_at(uint64_t seed, uint32_t stream, uint64_t counter, uint32_t j) {
  return philox4x32_10(make_uint4(j, stream, (uint32_t)counter, (uint32_t)(counter >> 32)), (uint32_t)seed,
                       (uint32_t)(seed >> 32));
}

// pair j -> elements 2j, 2j + 1
__global__ __launch_bounds__(256) void k_normals(uint64_t seed, uint32_t stream, uint64_t counter, size_t n,
                                                 double *__restrict__ out) {
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (2 * j >= n) return;
  const uint4 x = philox_at(seed, stream, counter, (uint32_t)j);
  const uint64_t a = (((uint64_t)x.x << 32) | x.y) >> 11;
  const uint64_t b = (((uint64_t)x.z << 32) | x.w) >> 11;
  const double u1 = ((double)a + 1.0) * 0x1p-53;  // (0, 1]
  const double u2 = (double)b * 0x1p-53;          // [0, 1)
  const double r = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincos(2.0 * M_PI * u2, &sn, &cs);
  out[2 * j] = r * cs;
  if (2 * j + 1 < n) out[2 * j + 1] = r * sn;
}

__global__ __launch_bounds__(256) void k_philox_words(uint64_t seed, uint32_t stream, uint64_t counter,
                                                      size_t npairs, uint4 *__restrict__ out) {
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= npairs) return;
  out[j] = philox_at(seed, stream, counter, (uint32_t)j);
}

}  // namespace

hipError_t launch_normals(uint64_t seed, uint32_t stream, uint64_t counter, size_t n, double *out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t pairs = (n + 1) / 2;
  if (pairs > 0xFFFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_normals, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, seed, stream, counter, n,
                     out);
  return hipGetLastError();
}

hipError_t launch_philox_words(uint64_t seed, uint32_t stream, uint64_t counter, size_t npairs, uint32_t *out,
                               hipStream_t s) {
  if (npairs == 0) return hipSuccess;
  if (npairs > 0xFFFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_philox_words, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, s, seed, stream, counter,
                     npairs, reinterpret_cast<uint4 *>(out));
  return hipGetLastError();
}

}  // namespace fbim
