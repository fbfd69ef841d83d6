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
template <int NR>
__device__ __forceinline__ void block_reduce(double (&v)[NR], const RedOut& o) {
  block_reduce_to<NR>(v, o.partial);
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
