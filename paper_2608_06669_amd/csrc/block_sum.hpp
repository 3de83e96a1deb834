// Fixed-order workgroup sums.
#pragma once

#include <hip/hip_runtime.h>

namespace pnk {

// Sums NV per-thread values over the workgroup: a butterfly inside each
// 64-lane wave, then the four wave totals in wave order. At every butterfly
// level the two lanes of a pair add the same two numbers (in either order),
// so all lanes end with the same bits, and any workgroup that sums the same
// per-thread values gets the same totals. Every thread receives the totals
// in v. sm is workgroup LDS of at least NV x 4 doubles; it can be reused
// once the call returns.
template <int NV>
__device__ inline void block_sum256(double (&v)[NV], double (*sm)[4]) {
#pragma unroll
  for (int c = 0; c < NV; ++c)
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v[c] += __shfl_xor(v[c], m, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int c = 0; c < NV; ++c) sm[c][w] = v[c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; ++c) v[c] = (sm[c][0] + sm[c][1]) + (sm[c][2] + sm[c][3]);
  __syncthreads();
}

// The same for workgroups of NW waves: wave totals summed in wave order,
// pairwise. sm holds at least NV x NW doubles.
template <int NV, int NW>
__device__ inline void block_sum_waves(double (&v)[NV], double (*sm)[NW]) {
#pragma unroll
  for (int c = 0; c < NV; ++c)
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v[c] += __shfl_xor(v[c], m, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int c = 0; c < NV; ++c) sm[c][w] = v[c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    double t[NW];
#pragma unroll
    for (int q = 0; q < NW; ++q) t[q] = sm[c][q];
#pragma unroll
    for (int h = 1; h < NW; h *= 2)
#pragma unroll
      for (int q = 0; q + h < NW; q += 2 * h) t[q] += t[q + h];
    v[c] = t[0];
  }
  __syncthreads();
}

}  // namespace pnk
