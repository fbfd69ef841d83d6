// Kernels for levels below the first coarse level ("Implementation"
// paragraph: the recursion of the coarse construction, and the coarsest
// solve).
//
// A level-l vector (l >= 1) is [site][n_f] complex in the level's internal
// site order, n_f = 2 Nv_l with component a of chirality a >= Nv_l.  The
// transfer to level l+1 uses Nv_{l+1} such vectors V_k, orthonormalised per
// (level-(l+1) block, chirality):
//   restrict  c(b, s, k) = (+1|-1)_s sum_{i in b} sum_{chi(a) = s} conj(V_k(i, a)) r(i, a)
//   prolong   e(i, a)    = sum_k V_k(i, a) c(b(i), chi(a), k)
// (R = P^dag Gamma5 with the coarse Gamma5 = diag(+1_Nv, -1_Nv)).  The
// level-(l+1) operator R D_p P is assembled column by column from the
// direction-split hop of the level-l stencil, exactly as on the fine level.
//
// The coarsest level can be solved directly: its full stencil is expanded
// into a dense matrix and inverted in FP64 by Gauss-Jordan elimination with
// partial pivoting; the solve is then one dense matrix-vector product.
#include "kernels.h"

namespace wcmg {

namespace {

template <typename T>
struct CVec;
template <>
struct CVec<double> {
  using V = double2;
};
template <>
struct CVec<float> {
  using V = float2;
};

template <typename T>
__device__ __forceinline__ cpx<double> cld(const void* p, size_t i) {
  auto v = reinterpret_cast<const typename CVec<T>::V*>(p)[i];
  return mk((double)v.x, (double)v.y);
}
template <typename T>
__device__ __forceinline__ void cst(void* p, size_t i, cpx<double> c) {
  typename CVec<T>::V v;
  v.x = (T)c.r;
  v.y = (T)c.i;
  reinterpret_cast<typename CVec<T>::V*>(p)[i] = v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// one wave per (coarse site c, vector k, right-hand side)
template <typename T>
__global__ void __launch_bounds__(64) k_ctr_restrict(void* out, size_t out_site_stride, size_t out_rhs_stride,
                                                     const void* in, size_t in_rhs_stride, const void* V,
                                                     size_t vstride, const int* members, int bvol, int nf,
                                                     int nvec) {
  const int c = blockIdx.x, k = blockIdx.y, r = blockIdx.z;
  const int lane = threadIdx.x;
  const int nh = nf / 2;
  const char* inr = reinterpret_cast<const char*>(in) + (size_t)r * in_rhs_stride * sizeof(typename CVec<T>::V);
  const void* vk = reinterpret_cast<const char*>(V) + (size_t)k * vstride * sizeof(typename CVec<T>::V);
  double a0r = 0, a0i = 0, a1r = 0, a1i = 0;
  for (int e = lane; e < bvol * nf; e += 64) {
    const int m = e / nf, a = e - m * nf;
    const size_t idx = (size_t)members[(size_t)c * bvol + m] * nf + a;
    cpx<double> v = cld<T>(vk, idx), x = cld<T>(inr, idx);
    const double pr = v.r * x.r + v.i * x.i, pi = v.r * x.i - v.i * x.r;
    if (a < nh) {
      a0r += pr;
      a0i += pi;
    } else {
      a1r += pr;
      a1i += pi;
    }
  }
  a0r = wave_sum(a0r);
  a0i = wave_sum(a0i);
  a1r = wave_sum(a1r);
  a1i = wave_sum(a1i);
  if (lane == 0) {
    char* o = reinterpret_cast<char*>(out) + (size_t)r * out_rhs_stride * sizeof(typename CVec<T>::V);
    cst<T>(o, (size_t)c * out_site_stride + k, mk(a0r, a0i));
    cst<T>(o, (size_t)c * out_site_stride + nvec + k, mk(-a1r, -a1i));
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_ctr_prolong(void* out, size_t out_rhs_stride, const void* in,
                                                     size_t in_rhs_stride, const void* V, size_t vstride,
                                                     const int* blk, int nsites, int nf, int nvec) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)nsites * nf) return;
  const int r = blockIdx.y;
  const int i = (int)(t / nf), a = (int)(t - (size_t)i * nf);
  const int s = a >= nf / 2;
  const int n2 = 2 * nvec;
  const char* inr = reinterpret_cast<const char*>(in) + (size_t)r * in_rhs_stride * sizeof(typename CVec<T>::V);
  const size_t cbase = (size_t)blk[i] * n2 + (size_t)s * nvec;
  cpx<double> acc = mk(0.0, 0.0);
  for (int k = 0; k < nvec; ++k) {
    const cpx<double> v = cld<T>(V, (size_t)k * vstride + t);
    cfma(acc, v, cld<T>(inr, cbase + k));
  }
  cst<T>(reinterpret_cast<char*>(out) + (size_t)r * out_rhs_stride * sizeof(typename CVec<T>::V), t, acc);
}

// block reduction of a complex double over 256 threads
__device__ cpx<double> block_csum(double re, double im) {
  __shared__ double sh[2][4];
  re = wave_sum(re);
  im = wave_sum(im);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sh[0][w] = re;
    sh[1][w] = im;
  }
  __syncthreads();
  return mk(sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3], sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3]);
}

// classical Gram-Schmidt, twice, over the rows of one (block, chirality)
__global__ void __launch_bounds__(256) k_ctr_block_ortho(double2* V, size_t vstride, const int* members, int bvol,
                                                         int nf, int nvec, int* flag) {
  const int c = blockIdx.x, s = blockIdx.y;
  const int nh = nf / 2;
  const int rows = bvol * nh;
  auto addr = [&](int k, int row) -> size_t {
    const int m = row / nh, a = s * nh + (row - m * nh);
    return (size_t)k * vstride + (size_t)members[(size_t)c * bvol + m] * nf + a;
  };
  for (int k = 0; k < nvec; ++k) {
    double n0 = 0.0;
    for (int row = threadIdx.x; row < rows; row += blockDim.x) {
      const double2 v = V[addr(k, row)];
      n0 += v.x * v.x + v.y * v.y;
    }
    n0 = block_csum(n0, 0.0).r;
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = 0; j < k; ++j) {
        double re = 0.0, im = 0.0;
        for (int row = threadIdx.x; row < rows; row += blockDim.x) {
          const double2 q = V[addr(j, row)], v = V[addr(k, row)];
          re += q.x * v.x + q.y * v.y;
          im += q.x * v.y - q.y * v.x;
        }
        const cpx<double> d = block_csum(re, im);
        for (int row = threadIdx.x; row < rows; row += blockDim.x) {
          const double2 q = V[addr(j, row)];
          double2& v = V[addr(k, row)];
          v.x -= d.r * q.x - d.i * q.y;
          v.y -= d.r * q.y + d.i * q.x;
        }
      }
    }
    double nk = 0.0;
    for (int row = threadIdx.x; row < rows; row += blockDim.x) {
      const double2 v = V[addr(k, row)];
      nk += v.x * v.x + v.y * v.y;
    }
    nk = block_csum(nk, 0.0).r;
    if (!(nk > 1e-24 * n0) || !(nk > 0.0)) {
      if (threadIdx.x == 0) flag[0] = 1;  // rank loss: every writer stores 1
      return;
    }
    const double inv = 1.0 / sqrt(nk);
    for (int row = threadIdx.x; row < rows; row += blockDim.x) {
      double2& v = V[addr(k, row)];
      v.x *= inv;
      v.y *= inv;
    }
  }
}

struct Buckets9 {
  double2* b[9];
};

// direction-split hop of u on level l: bucket 1+d receives Y_d(i) u(i+d) when
// i+d lies in another level-(l+1) block, bucket 0 the rest plus v
__global__ void __launch_bounds__(256) k_chop_split(Buckets9 bk, const double2* v, const double2* u,
                                                    const double2* Yhop, const int* nbr, const int* blk, int nsites,
                                                    int n) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)nsites * n) return;
  const int i = (int)(t / n), r = (int)(t - (size_t)i * n);
  cpx<double> b0 = mk(v[t].x, v[t].y);
  for (int d = 0; d < 8; ++d) {
    const int j = nbr[(size_t)i * 8 + d];
    const double2* Y = Yhop + ((size_t)i * 8 + d) * n * n;
    cpx<double> acc = mk(0.0, 0.0);
    for (int col = 0; col < n; ++col) {
      const double2 y = Y[(size_t)col * n + r], x = u[(size_t)j * n + col];
      cfma(acc, mk(y.x, y.y), mk(x.x, x.y));
    }
    if (blk[j] == blk[i]) {
      b0 = b0 + acc;
      bk.b[1 + d][t] = make_double2(0.0, 0.0);
    } else {
      bk.b[1 + d][t] = make_double2(acc.r, acc.i);
    }
  }
  bk.b[0][t] = make_double2(b0.r, b0.i);
}

__global__ void k_unit_fill(double2* e, int nsites, int n, int j) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)nsites * n) return;
  const int a = (int)(t % n);
  e[t] = make_double2(a == j ? 1.0 : 0.0, 0.0);
}

// augmented [M | 1], row-major N x 2N, from the stencil Y9 [site][9][n][n] (column-major blocks)
__global__ void __launch_bounds__(256) k_dense_from_stencil(double2* M, const double2* Y9, const int* nbr,
                                                            int nsites, int n) {
  const int R = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = nsites * n;
  if (R >= N) return;
  const int c = R / n, r = R - c * n;
  double2* row = M + (size_t)R * 2 * N;
  for (int j = 0; j < 2 * N; ++j) row[j] = make_double2(0.0, 0.0);
  const size_t nn = (size_t)n * n;
  for (int slot = 0; slot < 9; ++slot) {
    const int cc = slot == 0 ? c : nbr[(size_t)c * 8 + slot - 1];
    const double2* Y = Y9 + ((size_t)c * 9 + slot) * nn;
    for (int col = 0; col < n; ++col) {
      double2& m = row[(size_t)cc * n + col];
      const double2 y = Y[(size_t)col * n + r];
      m.x += y.x;
      m.y += y.y;
    }
  }
  row[N + R] = make_double2(1.0, 0.0);
}

// pivot of column k among rows k..N-1 (largest modulus, first on ties)
__global__ void __launch_bounds__(256) k_gj_pivot(const double2* M, int N, int k, int* piv, double2* pval) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  const size_t ld = 2 * (size_t)N;
  double best = -1.0;
  int idx = k;
  for (int i = k + threadIdx.x; i < N; i += blockDim.x) {
    const double2 m = M[(size_t)i * ld + k];
    const double a = m.x * m.x + m.y * m.y;
    if (a > best) {
      best = a;
      idx = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double o = bv[threadIdx.x + w];
      const int oi = bi[threadIdx.x + w];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    piv[0] = bi[0];
    pval[0] = M[(size_t)bi[0] * ld + k];
  }
}

// swap rows k and p, then divide row k by the pivot value (columns k..N+k)
__global__ void __launch_bounds__(256) k_gj_swap_scale(double2* M, int N, int k, const int* piv,
                                                       const double2* pval, int* flag) {
  const int j = k + blockIdx.x * blockDim.x + threadIdx.x;
  if (j > N + k) return;
  const size_t ld = 2 * (size_t)N;
  const int p = piv[0];
  const double2 pv = pval[0];
  const double d = pv.x * pv.x + pv.y * pv.y;
  if (!(d > 0.0)) {
    if (j == k) flag[0] = 1;  // singular
    return;
  }
  const double2 a = M[(size_t)k * ld + j], b = M[(size_t)p * ld + j];
  // b / pv
  M[(size_t)k * ld + j] = make_double2((b.x * pv.x + b.y * pv.y) / d, (b.y * pv.x - b.x * pv.y) / d);
  if (p != k) M[(size_t)p * ld + j] = a;
}

__global__ void k_gj_colcopy(const double2* M, int N, int k, double2* f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  f[i] = i == k ? make_double2(0.0, 0.0) : M[(size_t)i * 2 * N + k];
}

// M[i][j] -= f[i] M[k][j] for columns k..N+k (the only nonzero ones of row k)
__global__ void __launch_bounds__(256) k_gj_elim(double2* M, int N, int k, const double2* f) {
  const int j = k + blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j > N + k) return;
  const double2 fi = f[i];
  if (fi.x == 0.0 && fi.y == 0.0) return;
  const size_t ld = 2 * (size_t)N;
  const double2 mk_ = M[(size_t)k * ld + j];
  double2& m = M[(size_t)i * ld + j];
  m.x -= fi.x * mk_.x - fi.y * mk_.y;
  m.y -= fi.x * mk_.y + fi.y * mk_.x;
}

// x = Minv b with Minv the right half of the augmented matrix; one wave per row
template <typename T>
__global__ void __launch_bounds__(256) k_dense_gemv(const double2* M, int N, const void* b, void* x) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= N) return;
  const double2* m = M + (size_t)row * 2 * N + N;
  double re = 0.0, im = 0.0;
  for (int j = lane; j < N; j += 64) {
    const double2 a = m[j];
    const cpx<double> v = cld<T>(b, j);
    re += a.x * v.r - a.y * v.i;
    im += a.x * v.i + a.y * v.r;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) cst<T>(x, row, mk(re, im));
}

inline unsigned nblk(size_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void launch_ctr_restrict(int prec, void* out, size_t out_site_stride, size_t out_rhs_stride, const void* in,
                         size_t in_rhs_stride, const void* V, size_t vstride, const int* members, int nblocks,
                         int bvol, int nf, int nvec, int nrhs, hipStream_t st) {
  dim3 grid(nblocks, nvec, nrhs);
  if (prec == WCMG_F64)
    hipLaunchKernelGGL(k_ctr_restrict<double>, grid, dim3(64), 0, st, out, out_site_stride, out_rhs_stride, in,
                       in_rhs_stride, V, vstride, members, bvol, nf, nvec);
  else
    hipLaunchKernelGGL(k_ctr_restrict<float>, grid, dim3(64), 0, st, out, out_site_stride, out_rhs_stride, in,
                       in_rhs_stride, V, vstride, members, bvol, nf, nvec);
  HIPCHK(hipGetLastError());
}

void launch_ctr_prolong(int prec, void* out, size_t out_rhs_stride, const void* in, size_t in_rhs_stride,
                        const void* V, size_t vstride, const int* blk, int nsites, int nf, int nvec, int nrhs,
                        hipStream_t st) {
  dim3 grid(nblk((size_t)nsites * nf), nrhs);
  if (prec == WCMG_F64)
    hipLaunchKernelGGL(k_ctr_prolong<double>, grid, dim3(256), 0, st, out, out_rhs_stride, in, in_rhs_stride, V,
                       vstride, blk, nsites, nf, nvec);
  else
    hipLaunchKernelGGL(k_ctr_prolong<float>, grid, dim3(256), 0, st, out, out_rhs_stride, in, in_rhs_stride, V,
                       vstride, blk, nsites, nf, nvec);
  HIPCHK(hipGetLastError());
}

void launch_ctr_block_ortho(void* V, size_t vstride, const int* members, int nblocks, int bvol, int nf, int nvec,
                            int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_ctr_block_ortho, dim3(nblocks, 2), dim3(256), 0, st, reinterpret_cast<double2*>(V), vstride,
                     members, bvol, nf, nvec, flag);
  HIPCHK(hipGetLastError());
}

void launch_chop_split(void* const* buckets, const void* v, const void* u, const void* Yhop, const int* nbr,
                       const int* blk, int nsites, int n, hipStream_t st) {
  Buckets9 bk;
  for (int s = 0; s < 9; ++s) bk.b[s] = reinterpret_cast<double2*>(buckets[s]);
  hipLaunchKernelGGL(k_chop_split, dim3(nblk((size_t)nsites * n)), dim3(256), 0, st, bk,
                     reinterpret_cast<const double2*>(v), reinterpret_cast<const double2*>(u),
                     reinterpret_cast<const double2*>(Yhop), nbr, blk, nsites, n);
  HIPCHK(hipGetLastError());
}

void launch_unit_fill(void* e, int nsites, int n, int j, hipStream_t st) {
  hipLaunchKernelGGL(k_unit_fill, dim3(nblk((size_t)nsites * n)), dim3(256), 0, st, reinterpret_cast<double2*>(e),
                     nsites, n, j);
  HIPCHK(hipGetLastError());
}

void dense_inverse_build(void* M, const void* Y9, const int* nbr, int nsites, int n, int* piv, void* pval, void* f,
                         int* flag, hipStream_t st) {
  const int N = nsites * n;
  double2* A = reinterpret_cast<double2*>(M);
  hipLaunchKernelGGL(k_dense_from_stencil, dim3(nblk(N)), dim3(256), 0, st, A,
                     reinterpret_cast<const double2*>(Y9), nbr, nsites, n);
  HIPCHK(hipGetLastError());
  double2* pv = reinterpret_cast<double2*>(pval);
  double2* fv = reinterpret_cast<double2*>(f);
  for (int k = 0; k < N; ++k) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, st, A, N, k, piv, pv);
    hipLaunchKernelGGL(k_gj_swap_scale, dim3(nblk(N + 1)), dim3(256), 0, st, A, N, k, piv, pv, flag);
    hipLaunchKernelGGL(k_gj_colcopy, dim3(nblk(N)), dim3(256), 0, st, A, N, k, fv);
    hipLaunchKernelGGL(k_gj_elim, dim3(nblk(N + 1), N), dim3(256), 0, st, A, N, k, fv);
  }
  HIPCHK(hipGetLastError());
}

void dense_inverse_apply(int prec, const void* M, int N, const void* b, void* x, hipStream_t st) {
  const double2* A = reinterpret_cast<const double2*>(M);
  if (prec == WCMG_F64)
    hipLaunchKernelGGL(k_dense_gemv<double>, dim3((N + 3) / 4), dim3(256), 0, st, A, N, b, x);
  else
    hipLaunchKernelGGL(k_dense_gemv<float>, dim3((N + 3) / 4), dim3(256), 0, st, A, N, b, x);
  HIPCHK(hipGetLastError());
}

}  // namespace wcmg
