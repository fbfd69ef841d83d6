// Shared pieces of the BLAS-1 kernels: complex loads/stores in double or
// float storage, the block reduction into per-block partials, and the grid
// sizes (which depend only on the vector length, so results are bitwise
// reproducible run to run).
#pragma once

#include <algorithm>

#include "kernels.h"

namespace wcmg {
namespace blas_detail {

constexpr int kThreads = 256;
constexpr int kMaxK = 16;

template <typename T>
struct C2;
template <>
struct C2<double> {
  using V = double2;
};
template <>
struct C2<float> {
  using V = float2;
};

template <typename T>
__device__ __forceinline__ cpx<double> ld(const void* p, size_t i) {
  auto v = reinterpret_cast<const typename C2<T>::V*>(p)[i];
  return mk((double)v.x, (double)v.y);
}
template <typename T>
__device__ __forceinline__ void st(void* p, size_t i, cpx<double> c) {
  using V = typename C2<T>::V;
  V v;
  v.x = (T)c.r;
  v.y = (T)c.i;
  reinterpret_cast<V*>(p)[i] = v;
}

// Reduce NR doubles over the block into partial[blockIdx.x*NR + k].
template <int NR>
__device__ __forceinline__ void block_reduce_to(double (&v)[NR], double* partial) {
  __shared__ double sh[NR][kThreads / 64];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NR; ++k) sh[k][wave] = v[k];
  }
  __syncthreads();
  if ((int)threadIdx.x < NR) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) s += sh[threadIdx.x][w];
    partial[(size_t)blockIdx.x * NR + threadIdx.x] = s;
  }
}
// Grid-wide sum of NR doubles in one launch: every block stores its partials
// (device-coherent), counts itself in o.counter, and the last block to
// arrive adds the partials in block order (TPV threads per value over fixed
// strided subsets of the blocks, then a fixed shuffle tree) and writes the
// first nvalid sums to o.res (and o.hres); it then rearms the counter.  The
// order of the additions never depends on which block finishes last.
template <int NR>
__device__ __forceinline__ void block_reduce(double (&v)[NR], const RedOut& o, int nvalid = NR) {
  __shared__ double sh[NR][kThreads / 64];
  __shared__ double shw[kThreads / 64];
  __shared__ int last_s;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NR; ++k) sh[k][wave] = v[k];
  }
  __syncthreads();
  if ((int)threadIdx.x < NR) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) s += sh[threadIdx.x][w];
    __hip_atomic_store(o.partial + (size_t)blockIdx.x * NR + threadIdx.x, s, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  // the partial stores are complete (and coherent) before the block counts itself
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0)
    last_s = __hip_atomic_fetch_add(o.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
  __syncthreads();
  if (!last_s) return;
  const int nb = gridDim.x;
  int tpv = 1;
  while (tpv * 2 * nvalid <= kThreads && tpv < nb) tpv *= 2;
  const int t = threadIdx.x, vv = t / tpv, j = t - vv * tpv;
  double s = 0.0;
  if (vv < nvalid) {
    // eight loads in flight, then added in block order
    int b = j;
    for (; b + 7 * tpv < nb; b += 8 * tpv) {
      double p[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        p[u] = __hip_atomic_load(o.partial + (size_t)(b + u * tpv) * NR + vv, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
      for (int u = 0; u < 8; ++u) s += p[u];
    }
    for (; b < nb; b += tpv)
      s += __hip_atomic_load(o.partial + (size_t)b * NR + vv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  const int width = tpv < 64 ? tpv : 64;
  for (int off = width >> 1; off > 0; off >>= 1) s += __shfl_down(s, off, width);
  if (tpv > 64) {
    if (lane == 0) shw[wave] = s;
    __syncthreads();
    if (j == 0 && vv < nvalid) {
      double u = 0.0;
      for (int q = 0; q < tpv / 64; ++q) u += shw[wave + q];
      s = u;
    }
  }
  if (j == 0 && vv < nvalid) {
    o.res[vv] = s;
    if (o.hres) o.hres[vv] = s;
  }
  if (threadIdx.x == 0) __hip_atomic_store(o.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// enough blocks that every thread handles about 8 elements, at most
// kRedBlocks; short vectors (the coarse levels) spread over up to 64 blocks
// with at least one element per thread, so that a pass is not limited by the
// latency of a handful of compute units
inline dim3 red_grid(size_t n) {
  size_t b = (n + 8 * kThreads - 1) / (8 * kThreads);
  const size_t spread = std::min<size_t>((n + kThreads - 1) / kThreads, 64);
  if (b < spread) b = spread;
  if (b < 1) b = 1;
  if (b > (size_t)kRedBlocks) b = kRedBlocks;
  return dim3((unsigned)b);
}
inline dim3 ew_grid(size_t n) {
  size_t b = (n + kThreads - 1) / kThreads;
  if (b > 65536) b = 65536;
  if (b == 0) b = 1;
  return dim3((unsigned)b);
}

#define GRID_STRIDE(i, n) \
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (size_t)gridDim.x * blockDim.x)


}  // namespace blas_detail
}  // namespace wcmg
