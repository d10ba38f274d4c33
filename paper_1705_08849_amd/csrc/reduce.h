// Deterministic block / grid reductions.
//
// Every reduction in the library follows one pattern: each thread
// accumulates in a fixed order, a wavefront folds its 64 lanes with
// shuffles, the block sums its wavefronts in order and stores one partial
// per block with plain stores.  A one-block finish kernel launched right
// after on the same stream sums the partials in block order and runs the
// scalar update.  The kernel boundary makes the partials visible; no
// device-scope fence or atomic ticket is used (on a multi-XCD part a
// device-scope release fence writes back the XCD's L2, which made a ticket
// per block cost more than the streaming work itself).  Results are bitwise
// reproducible for a fixed launch configuration.
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

// Store this block's partial sums at partials[block * N + q].
template <int N>
__device__ __forceinline__ void block_partial(double (&v)[N], double* partials, double* lds) {
  block_reduce<N>(v, lds);
  if (threadIdx.x == 0) {
    const int64_t bid = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
#pragma unroll
    for (int q = 0; q < N; ++q) partials[bid * N + q] = v[q];
  }
}

// Store this block's partial sums at partials[bid * N + q].
template <int N>
__device__ __forceinline__ void block_partial_at(double (&v)[N], double* partials, double* lds,
                                                 int64_t bid) {
  block_reduce<N>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) partials[bid * N + q] = v[q];
  }
}

// Finish kernel: one block sums nblk partials in block order and hands the
// totals to f (thread 0).  F provides skip() (nothing was reduced) and
// operator()(const double* sums).
template <int N, class F>
__global__ void __launch_bounds__(1024) finish_kernel(const double* partials, int nblk, F f) {
  // 1024 threads with four independent loads in flight each: the finish sits
  // on the critical path of every Krylov iteration, so its latency counts
  constexpr int NT = 1024, U = 4;
  __shared__ double lds[N * (NT / 64)];
  if (f.skip()) return;
  double s[N];
#pragma unroll
  for (int q = 0; q < N; ++q) s[q] = 0.0;
  int b = threadIdx.x;
  for (; b + (U - 1) * NT < nblk; b += U * NT) {
    double v[U][N];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < N; ++q) v[u][q] = partials[(int64_t)(b + u * NT) * N + q];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < N; ++q) s[q] += v[u][q];
  }
  for (; b < nblk; b += NT) {
#pragma unroll
    for (int q = 0; q < N; ++q) s[q] += partials[(int64_t)b * N + q];
  }
  block_reduce<N>(s, lds);
  if (threadIdx.x == 0) f(s);
}

// Several finishes in one launch: block s sums items[s]'s partials.
template <class F>
struct FinishItem {
  const double* partials;
  int nblk;
  F f;
};
template <int N, class F>
__global__ void __launch_bounds__(256) finish_multi_kernel(const FinishItem<F>* items) {
  __shared__ double lds[N * 4];
  const FinishItem<F>& it = items[blockIdx.x];
  if (it.f.skip()) return;
  double s[N];
#pragma unroll
  for (int q = 0; q < N; ++q) s[q] = 0.0;
  for (int b = threadIdx.x; b < it.nblk; b += blockDim.x) {
#pragma unroll
    for (int q = 0; q < N; ++q) s[q] += it.partials[(int64_t)b * N + q];
  }
  block_reduce<N>(s, lds);
  if (threadIdx.x == 0) it.f(s);
}

template <int N, class F>
inline hipError_t launch_finish(const double* partials, int nblk, const F& f, hipStream_t s) {
  hipLaunchKernelGGL((finish_kernel<N, F>), dim3(1), dim3(1024), 0, s, partials, nblk, f);
  return hipGetLastError();
}

}  // namespace fit
