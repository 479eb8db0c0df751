// Device helpers shared by the fast-summation and CG kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "nld_internal.h"

namespace nld {

// Scaled Kaiser-Bessel spreading weight at distance delta (grid cells, |delta| <= m):
//   psi(delta) = m sinh(b z) / (z sinh(b m)),  z = sqrt(m^2 - delta^2),
// evaluated as (m/z) exp(b (z - m)) (1 - exp(-2 b z)) / (1 - exp(-2 b m)), which does not
// overflow; psi(0) = 1 and the z -> 0 limit is 2 b m exp(-b m) / (1 - exp(-2 b m)).
__device__ __forceinline__ float kb_psi(float delta, float m, float b, float den) {
  const float z2 = fmaxf(m * m - delta * delta, 0.0f);
  const float z = sqrtf(z2);
  if (z > 0.0f) return (m / z) * expf(b * (z - m)) * (-expm1f(-2.0f * b * z)) * den;
  return 2.0f * b * m * expf(-b * m) * den;
}
__device__ __forceinline__ double kb_psi(double delta, double m, double b, double den) {
  const double z2 = fmax(m * m - delta * delta, 0.0);
  const double z = sqrt(z2);
  if (z > 0.0) return (m / z) * exp(b * (z - m)) * (-expm1(-2.0 * b * z)) * den;
  return 2.0 * b * m * exp(-b * m) * den;
}

// Sum of NS values over a block of kRedThreads threads, the same bits in every thread: an XOR
// butterfly within each wavefront (each step adds symmetric pairs, so all lanes agree), then
// the wavefronts' partials in order.
template <int NS>
__device__ __forceinline__ void block_sum(double (&v)[NS]) {
  constexpr int kWaves = kRedThreads / 64;
  __shared__ double sh[NS][kWaves];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < NS; ++k) v[k] += __shfl_xor(v[k], off);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < NS; ++k) sh[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    double s = sh[k][0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += sh[k][w];
    v[k] = s;
  }
  __syncthreads();
}

// Deterministic FP64 reduction of NS values over the whole grid: every block sums its threads'
// values in a fixed order, writes one partial per value, and the last block to finish
// (agent-scope ticket) sums the partials in block order.  Returns true in the last block, with
// the totals in out[] for every thread of that block.  Block size must be kRedThreads;
// nblocks blocks (blockIdx.x < nblocks) take part; the ticket is reset by the last block.
template <int NS>
__device__ bool grid_reduce(const double (&v)[NS], double* red, unsigned* ticket,
                            double (&out)[NS], unsigned nblocks) {
  __shared__ int last;
  const int t = threadIdx.x;
  double bs[NS];
  for (int k = 0; k < NS; ++k) bs[k] = v[k];
  block_sum<NS>(bs);
  if (t == 0) {
    for (int k = 0; k < NS; ++k) red[(size_t)blockIdx.x * 8 + k] = bs[k];
    __threadfence();
    const unsigned prev = atomicAdd(ticket, 1u);
    last = (prev == nblocks - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double acc[NS];
  for (int k = 0; k < NS; ++k) acc[k] = 0.0;
  for (unsigned b = t; b < nblocks; b += kRedThreads)
    for (int k = 0; k < NS; ++k)
      acc[k] += __hip_atomic_load(&red[(size_t)b * 8 + k], __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  block_sum<NS>(acc);
  for (int k = 0; k < NS; ++k) out[k] = acc[k];
  if (t == 0) atomicExch(ticket, 0u);
  return true;
}

template <typename T>
__device__ __forceinline__ const T* vin(const ImgDev& im, VecArg a) {
  return a.ext ? reinterpret_cast<const T*>(a.ext) : reinterpret_cast<const T*>(im.vec[a.sel]);
}
template <typename T>
__device__ __forceinline__ T* vout(const ImgDev& im, VecArg a) {
  return a.ext ? reinterpret_cast<T*>(const_cast<void*>(a.ext)) : reinterpret_cast<T*>(im.vec[a.sel]);
}

}  // namespace nld
