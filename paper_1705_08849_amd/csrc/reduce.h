// Deterministic block / grid reductions.
//
// Every reduction in the library follows one pattern: each thread
// accumulates in a fixed order, a wavefront folds its 64 lanes with
// shuffles, the block sums its wavefronts in order and publishes one partial
// per block; the last block to arrive (atomic ticket) sums the partials in
// block order.  Results are therefore bitwise reproducible for a fixed launch
// configuration, which the solver tests rely on.
#pragma once

#include "fit_internal.h"

namespace fit {

template <int N>
__device__ __forceinline__ void wave_reduce(double (&v)[N]) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += __shfl_down(v[q], off, 64);
  }
}

// Sum v over the block; the result is valid in thread 0.  lds must hold
// N * blockDim.x / 64 doubles.
template <int N>
__device__ __forceinline__ void block_reduce(double (&v)[N], double* lds) {
  wave_reduce<N>(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) lds[wid * N + q] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = 0.0;
    for (int w = 0; w < nw; ++w) {
#pragma unroll
      for (int q = 0; q < N; ++q) v[q] += lds[w * N + q];
    }
  }
  __syncthreads();
}

// Publish this block's partial and, in the last block to finish, sum all
// partials in block order.  Returns true in every thread of that last block;
// the grid-wide sums are then in `out` of thread 0.  The ticket counter is
// reset by the last block so the next launch (or graph replay) starts at 0.
template <int N>
__device__ __forceinline__ bool grid_reduce(double (&v)[N], double* partials, unsigned* counter,
                                            double* lds, double (&out)[N]) {
  __shared__ int s_last;
  block_reduce<N>(v, lds);
  const int nblk = gridDim.x * gridDim.y * gridDim.z;
  const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) partials[(int64_t)bid * N + q] = v[q];
    __threadfence();
    unsigned t = atomicAdd(counter, 1u);
    s_last = (t == (unsigned)(nblk - 1));
  }
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  double s[N];
#pragma unroll
  for (int q = 0; q < N; ++q) s[q] = 0.0;
  const volatile double* vp = partials;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
#pragma unroll
    for (int q = 0; q < N; ++q) s[q] += vp[(int64_t)b * N + q];
  }
  block_reduce<N>(s, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) out[q] = s[q];
    atomicExch(counter, 0u);
  }
  return true;
}

}  // namespace fit
