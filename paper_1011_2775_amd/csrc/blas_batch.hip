// Batched BLAS-1 kernels for the lockstep multi-right-hand-side solvers.
//
// A batch holds nrhs vectors of n complex elements, vstride elements apart.
// Grid row blockIdx.y is the right-hand side; every reduction of a batch
// writes its per-block partials to part[rhs][block][NR] and a second pass
// (one block per result and right-hand side, fixed tree, as in the
// single-vector kernels) writes res[rhs * rs + k].  The GCR coefficients of right-hand
// side r live at beta + r * bs and qa + r * qs (device memory), so no
// right-hand side shares a scalar with another.
#include "blas_common.h"

namespace wcmg {

namespace {

using namespace blas_detail;

__device__ __forceinline__ double* part_row(const RedB& o, int nr) {
  return o.part + (size_t)blockIdx.y * gridDim.x * nr;
}
template <typename T>
__device__ __forceinline__ const void* row(const void* p, size_t vs) {
  return reinterpret_cast<const char*>(p) + (size_t)blockIdx.y * vs * sizeof(typename C2<T>::V);
}
template <typename T>
__device__ __forceinline__ void* row(void* p, size_t vs) {
  return reinterpret_cast<char*>(p) + (size_t)blockIdx.y * vs * sizeof(typename C2<T>::V);
}

// one block per (output k, right-hand side r), fixed-order tree as in the single-vector kernels
__global__ void __launch_bounds__(kThreads) k_finalize_b(RedB o, int nr, int stride, int nblocks) {
  const int k = blockIdx.x, r = blockIdx.y;
  const double* p = o.part + (size_t)r * nblocks * stride;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kThreads) s += p[(size_t)b * stride + k];
  __shared__ double sh[kThreads];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) o.res[(size_t)r * o.rs + k] = sh[0];
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_norm2_b(const void* x, size_t vs, size_t n, RedB o) {
  double v[1] = {0.0};
  const void* xr = row<T>(x, vs);
  GRID_STRIDE(i, n) {
    cpx<double> a = ld<T>(xr, i);
    v[0] += a.r * a.r + a.i * a.i;
  }
  block_reduce_to<1>(v, part_row(o, 1));
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_cdot_norm_b(const void* x, const void* y, size_t vs, size_t n, RedB o) {
  double v[3] = {0.0, 0.0, 0.0};
  const void* xr = row<T>(x, vs);
  const void* yr = row<T>(y, vs);
  GRID_STRIDE(i, n) {
    cpx<double> a = ld<T>(xr, i), b = ld<T>(yr, i);
    v[0] += a.r * b.r + a.i * b.i;
    v[1] += a.r * b.i - a.i * b.r;
    v[2] += a.r * a.r + a.i * a.i;
  }
  block_reduce_to<3>(v, part_row(o, 3));
}

struct MultiB {
  const void* v[kMaxK];
  const void* w[kMaxK];
};

template <typename T>
__global__ void __launch_bounds__(kThreads) k_multi_cdot_b(MultiB m, int k, const void* y, size_t vs, size_t n,
                                                           RedB o) {
  double v[2 * kMaxK];
#pragma unroll
  for (int j = 0; j < 2 * kMaxK; ++j) v[j] = 0.0;
  const void* yr = row<T>(y, vs);
  GRID_STRIDE(i, n) {
    cpx<double> b = ld<T>(yr, i);
#pragma unroll
    for (int j = 0; j < kMaxK; ++j) {
      if (j < k) {
        cpx<double> a = ld<T>(row<T>(m.v[j], vs), i);
        v[2 * j] += a.r * b.r + a.i * b.i;
        v[2 * j + 1] += a.r * b.i - a.i * b.r;
      }
    }
  }
  block_reduce_to<2 * kMaxK>(v, part_row(o, 2 * kMaxK));
}

__device__ __forceinline__ cpx<double> alpha_of(const double* qa) {
  const double d = qa[0];
  return d > 0.0 ? mk(qa[1] / d, qa[2] / d) : mk(0.0, 0.0);
}

// The single-vector GCR step (k_gcr_step_dev) for every right-hand side (row
// r of beta, qa and cj at beta + r bs, qa + r qs, cj + r cjs); the last
// launch of a step leaves the partials of ||r||^2
template <typename T>
__global__ void __launch_bounds__(kThreads) k_gcr_step_b(MultiB m, int j0, int k, int ktot, void* y, void* r,
                                                         size_t vs, size_t n, const double* beta, size_t bs,
                                                         double* qa, size_t qs, double* cj, size_t cjs, int last,
                                                         RedB o) {
  const double* be = beta + (size_t)blockIdx.y * bs;
  double* q4 = qa + (size_t)blockIdx.y * qs;
  cpx<double> c[kMaxK];
#pragma unroll
  for (int j = 0; j < kMaxK; ++j) {
    const double d = j < k ? q4[4 * (j0 + j)] : 0.0;
    c[j] = (j < k && d > 0.0) ? mk(be[2 * (j0 + j)] / d, be[2 * (j0 + j) + 1] / d) : mk(0.0, 0.0);
  }
  cpx<double> alpha = mk(0.0, 0.0);
  if (last) {
    double qq = be[2 * ktot];
    for (int j = 0; j < ktot; ++j) {
      const double d = q4[4 * j];
      if (d > 0.0) {
        const double br = be[2 * j], bi = be[2 * j + 1];
        qq -= (br * br + bi * bi) / d;
      }
    }
    const cpx<double> qr = mk(be[2 * ktot + 2], -be[2 * ktot + 3]);
    if (qq > 0.0) alpha = mk(qr.r / qq, qr.i / qq);
    if (blockIdx.x == 0) {
      if (threadIdx.x == 0) {
        q4[4 * ktot] = qq;
        q4[4 * ktot + 1] = qr.r;
        q4[4 * ktot + 2] = qr.i;
      }
      double* cr = cj + (size_t)blockIdx.y * cjs;
      for (int j = threadIdx.x; j < ktot; j += blockDim.x) {
        const double d = q4[4 * j];
        cr[2 * j] = d > 0.0 ? be[2 * j] / d : 0.0;
        cr[2 * j + 1] = d > 0.0 ? be[2 * j + 1] / d : 0.0;
      }
    }
  }
  double v[1] = {0.0};
  void* yr = row<T>(y, vs);
  void* rr = row<T>(r, vs);
  GRID_STRIDE(i, n) {
    cpx<double> a = ld<T>(yr, i);
#pragma unroll
    for (int j = 0; j < kMaxK; ++j)
      if (j < k) a = a - c[j] * ld<T>(row<T>(m.v[j], vs), i);
    st<T>(yr, i, a);
    if (last) {
      const cpx<double> as = mk((double)(T)a.r, (double)(T)a.i);
      const cpx<double> b = ld<T>(rr, i) - alpha * as;
      st<T>(rr, i, b);
      const cpx<double> bs2 = mk((double)(T)b.r, (double)(T)b.i);
      v[0] += bs2.r * bs2.r + bs2.i * bs2.i;
    }
  }
  if (last) block_reduce_to<1>(v, part_row(o, 1));
}

// per right-hand side (one thread each): (I + C) y = alpha by back
// substitution, C from cmat row r (cmat + r cms, column j at 2 j ldc), alpha
// from qa row r; y row r at y + r ys
__global__ void k_gcr_coef_solve_b(const double* qa, size_t qs, const double* cmat, size_t cms, int ldc, double* y,
                                   size_t ys, int kt, int nrhs) {
  const int rr = blockIdx.x * blockDim.x + threadIdx.x;
  if (rr >= nrhs) return;
  const double* q4 = qa + (size_t)rr * qs;
  const double* cm = cmat + (size_t)rr * cms;
  double* yv = y + (size_t)rr * ys;
  for (int i = kt - 1; i >= 0; --i) {
    cpx<double> s = alpha_of(q4 + 4 * i);
    for (int j = i + 1; j < kt; ++j) {
      const cpx<double> cij = mk(cm[2 * ((size_t)j * ldc + i)], cm[2 * ((size_t)j * ldc + i) + 1]);
      s = s - cij * mk(yv[2 * j], yv[2 * j + 1]);
    }
    yv[2 * i] = s.r;
    yv[2 * i + 1] = s.i;
  }
}

// x += sum_j coef_j z_j per right-hand side (coef row r at coef + r cs)
template <typename T>
__global__ void k_multi_axpy_b(MultiB m, int k, void* x, size_t vs, size_t n, const double* coef, size_t cs) {
  const double* cf = coef + (size_t)blockIdx.y * cs;
  cpx<double> c[kMaxK];
#pragma unroll
  for (int j = 0; j < kMaxK; ++j) c[j] = j < k ? mk(cf[2 * j], cf[2 * j + 1]) : mk(0.0, 0.0);
  void* xr = row<T>(x, vs);
  GRID_STRIDE(i, n) {
    cpx<double> acc = ld<T>(xr, i);
#pragma unroll
    for (int j = 0; j < kMaxK; ++j)
      if (j < k) acc = acc + c[j] * ld<T>(row<T>(m.v[j], vs), i);
    st<T>(xr, i, acc);
  }
}

// MR step of every right-hand side with alpha = coef[0..1] / coef[2] (row r at coef + r * cs)
template <typename T>
__global__ void k_mr_update_b(const double* coef, size_t cs, void* x, void* r, const void* Ar, size_t vs, size_t n) {
  const double* cf = coef + (size_t)blockIdx.y * cs;
  const double d = cf[2];
  const cpx<double> a = d > 0.0 ? mk(cf[0] / d, cf[1] / d) : mk(0.0, 0.0);
  void* xr = row<T>(x, vs);
  void* rr = row<T>(r, vs);
  const void* ar = row<T>(Ar, vs);
  GRID_STRIDE(i, n) {
    st<T>(xr, i, ld<T>(xr, i) + a * ld<T>(rr, i));
    st<T>(rr, i, ld<T>(rr, i) - a * ld<T>(ar, i));
  }
}

}  // namespace

#define DISPATCH_B(prec, KERNEL, grid, ...)                                                 \
  do {                                                                                      \
    if ((prec) == WCMG_F64)                                                                 \
      hipLaunchKernelGGL(KERNEL<double>, grid, dim3(kThreads), 0, st, __VA_ARGS__);         \
    else                                                                                    \
      hipLaunchKernelGGL(KERNEL<float>, grid, dim3(kThreads), 0, st, __VA_ARGS__);          \
    HIPCHK(hipGetLastError());                                                              \
  } while (0)

static dim3 red_grid_b(size_t n, int nrhs) { return dim3(red_grid(n).x, nrhs); }
static dim3 ew_grid_b(size_t n, int nrhs) { return dim3(ew_grid(n).x, nrhs); }

static void finalize_b(const RedB& o, int nr, int stride, size_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_b, dim3(nr, nrhs), dim3(kThreads), 0, st, o, nr, stride, (int)red_grid(n).x);
  HIPCHK(hipGetLastError());
}

static void check_batch(int nrhs) {
  if (nrhs < 1 || nrhs > kMaxBatch) fail(WCMG_EINVAL, "batch size out of range");
}

void blas_norm2_b(int prec, const void* x, size_t vs, size_t n, int nrhs, const RedB& o, hipStream_t st) {
  check_batch(nrhs);
  DISPATCH_B(prec, k_norm2_b, red_grid_b(n, nrhs), x, vs, n, o);
  finalize_b(o, 1, 1, n, nrhs, st);
}

void blas_cdot_norm_b(int prec, const void* x, const void* y, size_t vs, size_t n, int nrhs, const RedB& o,
                      hipStream_t st) {
  check_batch(nrhs);
  DISPATCH_B(prec, k_cdot_norm_b, red_grid_b(n, nrhs), x, y, vs, n, o);
  finalize_b(o, 3, 3, n, nrhs, st);
}

void blas_multi_cdot_b(int prec, const void* const* v, int k, const void* y, size_t vs, size_t n, int nrhs,
                       const RedB& o, hipStream_t st) {
  check_batch(nrhs);
  for (int j0 = 0; j0 < k; j0 += kMaxK) {
    const int kk = std::min(kMaxK, k - j0);
    MultiB m{};
    for (int j = 0; j < kk; ++j) m.v[j] = v[j0 + j];
    RedB oo{o.res + 2 * j0, o.rs, o.part};
    DISPATCH_B(prec, k_multi_cdot_b, red_grid_b(n, nrhs), m, kk, y, vs, n, oo);
    finalize_b(oo, 2 * kk, 2 * kMaxK, n, nrhs, st);
  }
}

void blas_gcr_step_b(int prec, const void* const* q, int k, void* y, void* r, size_t vs, size_t n, int nrhs,
                     const double* beta, size_t bs, double* qa, size_t qs, double* cj, size_t cjs, const RedB& o,
                     hipStream_t st) {
  check_batch(nrhs);
  if (k == 0) {
    MultiB m{};
    DISPATCH_B(prec, k_gcr_step_b, red_grid_b(n, nrhs), m, 0, 0, 0, y, r, vs, n, beta, bs, qa, qs, cj, cjs, 1, o);
    finalize_b(o, 1, 1, n, nrhs, st);
    return;
  }
  for (int j0 = 0; j0 < k; j0 += kMaxK) {
    const int kk = std::min(kMaxK, k - j0);
    MultiB m{};
    for (int j = 0; j < kk; ++j) m.v[j] = q[j0 + j];
    const int last = j0 + kk == k;
    DISPATCH_B(prec, k_gcr_step_b, red_grid_b(n, nrhs), m, j0, kk, k, y, r, vs, n, beta, bs, qa, qs, cj, cjs, last,
               o);
    if (last) finalize_b(o, 1, 1, n, nrhs, st);
  }
}

void blas_gcr_update_x_raw_b(int prec, const void* const* z, int kt, void* x, size_t vs, size_t n, int nrhs,
                             const double* qa, size_t qs, const double* cmat, size_t cms, int ldc, double* y,
                             size_t ys, hipStream_t st) {
  check_batch(nrhs);
  if (kt <= 0) return;
  hipLaunchKernelGGL(k_gcr_coef_solve_b, dim3(1), dim3(64), 0, st, qa, qs, cmat, cms, ldc, y, ys, kt, nrhs);
  HIPCHK(hipGetLastError());
  for (int j0 = 0; j0 < kt; j0 += kMaxK) {
    const int kk = std::min(kMaxK, kt - j0);
    MultiB m{};
    for (int j = 0; j < kk; ++j) m.v[j] = z[j0 + j];
    DISPATCH_B(prec, k_multi_axpy_b, ew_grid_b(n, nrhs), m, kk, x, vs, n, y + 2 * j0, ys);
  }
}

void blas_mr_update_b(int prec, const double* coef, size_t cs, void* x, void* r, const void* Ar, size_t vs, size_t n,
                      int nrhs, hipStream_t st) {
  check_batch(nrhs);
  DISPATCH_B(prec, k_mr_update_b, ew_grid_b(n, nrhs), coef, cs, x, r, Ar, vs, n);
}

}  // namespace wcmg
