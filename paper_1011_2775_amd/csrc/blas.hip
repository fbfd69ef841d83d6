// BLAS-1 kernels for the Krylov solvers (GCR, BiCGStab, MR).
//
// Vectors are flat arrays of complex numbers in double or float storage;
// every reduction accumulates in double, first per wavefront with lane
// shuffles, then across the 4 wavefronts of a block in LDS; the last block
// of the grid to finish then sums the per-block partials in a fixed tree and
// writes the result to device memory, all in the one launch.  The grids
// depend only on the vector length, so results are bitwise reproducible run
// to run.
#include "blas_common.h"

namespace wcmg {

namespace {

using namespace blas_detail;

// complex vector in storage D from storage T (rounding to nearest)
template <typename D, typename T>
__global__ void k_convert(void* y, const void* x, size_t n) {
  GRID_STRIDE(i, n) st<D>(y, i, ld<T>(x, i));
}

__global__ void k_defl_coefs(const double* dots, double* qa, int K) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < K) {
    qa[4 * j] = 1.0;
    qa[4 * j + 1] = dots[2 * j];
    qa[4 * j + 2] = dots[2 * j + 1];
    qa[4 * j + 3] = 0.0;
  }
}

template <typename T>
__global__ void k_zero(void* x, size_t n) {
  GRID_STRIDE(i, n) st<T>(x, i, mk(0.0, 0.0));
}
template <typename T>
__global__ void k_copy(void* y, const void* x, size_t n) {
  GRID_STRIDE(i, n) st<T>(y, i, ld<T>(x, i));
}
template <typename T>
__global__ void k_axpby(double ar, double ai, const void* x, double br, double bi, void* y, size_t n) {
  cpx<double> a = mk(ar, ai), b = mk(br, bi);
  GRID_STRIDE(i, n) st<T>(y, i, a * ld<T>(x, i) + b * ld<T>(y, i));
}
template <typename T>
__global__ void __launch_bounds__(kThreads) k_norm2(const void* x, size_t n, const RedOut o) {
  double v[1] = {0.0};
  GRID_STRIDE(i, n) {
    cpx<double> a = ld<T>(x, i);
    v[0] += a.r * a.r + a.i * a.i;
  }
  block_reduce<1>(v, o);
}
template <typename T>
__global__ void __launch_bounds__(kThreads) k_cdot(const void* x, const void* y, size_t n, const RedOut o) {
  double v[2] = {0.0, 0.0};
  GRID_STRIDE(i, n) {
    cpx<double> a = ld<T>(x, i), b = ld<T>(y, i);
    v[0] += a.r * b.r + a.i * b.i;
    v[1] += a.r * b.i - a.i * b.r;
  }
  block_reduce<2>(v, o);
}
template <typename T>
__global__ void __launch_bounds__(kThreads) k_cdot_norm(const void* x, const void* y, size_t n, const RedOut o) {
  double v[3] = {0.0, 0.0, 0.0};
  GRID_STRIDE(i, n) {
    cpx<double> a = ld<T>(x, i), b = ld<T>(y, i);
    v[0] += a.r * b.r + a.i * b.i;
    v[1] += a.r * b.i - a.i * b.r;
    v[2] += a.r * a.r + a.i * a.i;
  }
  block_reduce<3>(v, o);
}

struct MultiArgs {
  const void* v[kMaxK];
  const void* w[kMaxK];
  double c[2 * kMaxK];
};

template <typename T>
__global__ void __launch_bounds__(kThreads) k_multi_cdot(MultiArgs m, int k, const void* y, size_t n,
                                                         const RedOut o) {
  double v[2 * kMaxK];
#pragma unroll
  for (int j = 0; j < 2 * kMaxK; ++j) v[j] = 0.0;
  GRID_STRIDE(i, n) {
    cpx<double> b = ld<T>(y, i);
#pragma unroll
    for (int j = 0; j < kMaxK; ++j) {
      if (j < k) {
        cpx<double> a = ld<T>(m.v[j], i);
        v[2 * j] += a.r * b.r + a.i * b.i;
        v[2 * j + 1] += a.r * b.i - a.i * b.r;
      }
    }
  }
  block_reduce<2 * kMaxK>(v, o, 2 * k);
}

template <typename T>
__global__ void k_multi_axpy(MultiArgs m, int k, void* y, size_t n) {
  GRID_STRIDE(i, n) {
    cpx<double> acc = ld<T>(y, i);
#pragma unroll
    for (int j = 0; j < kMaxK; ++j)
      if (j < k) acc = acc + mk(m.c[2 * j], m.c[2 * j + 1]) * ld<T>(m.v[j], i);
    st<T>(y, i, acc);
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_axpy_norm(double ar, double ai, const void* x, void* y, size_t n,
                                                        const RedOut o) {
  double v[1] = {0.0};
  cpx<double> a = mk(ar, ai);
  GRID_STRIDE(i, n) {
    cpx<double> b = ld<T>(y, i) + a * ld<T>(x, i);
    st<T>(y, i, b);
    cpx<double> bs = ld<T>(y, i);
    v[0] += bs.r * bs.r + bs.i * bs.i;
  }
  block_reduce<1>(v, o);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_bicg_update(double ar, double ai, double wr, double wi, const void* p,
                                                          const void* s, const void* t, void* x, void* r,
                                                          const void* rhat, size_t n, const RedOut o) {
  double v[3] = {0.0, 0.0, 0.0};
  cpx<double> a = mk(ar, ai), w = mk(wr, wi);
  GRID_STRIDE(i, n) {
    cpx<double> sv = ld<T>(s, i);
    st<T>(x, i, ld<T>(x, i) + a * ld<T>(p, i) + w * sv);
    st<T>(r, i, sv - w * ld<T>(t, i));
    cpx<double> rv = ld<T>(r, i), h = ld<T>(rhat, i);
    v[0] += rv.r * rv.r + rv.i * rv.i;
    v[1] += h.r * rv.r + h.i * rv.i;
    v[2] += h.r * rv.i - h.i * rv.r;
  }
  block_reduce<3>(v, o);
}

template <typename T>
__global__ void k_bicg_p(double br, double bi, double wr, double wi, const void* r, const void* v, void* p,
                         size_t n) {
  cpx<double> b = mk(br, bi), w = mk(wr, wi);
  GRID_STRIDE(i, n) st<T>(p, i, ld<T>(r, i) + b * (ld<T>(p, i) - w * ld<T>(v, i)));
}

// ---- device-resident coefficients (no host round trip between kernels) ----
// GCR basis slot j keeps qa[4j..4j+3] = { ||q_j||^2, re <q_j,r>, im <q_j,r>, ||r||^2 after step j };
// beta[2j..2j+1] = <q_j, q_new> from the multi-dot.
__device__ __forceinline__ cpx<double> gcr_alpha(const double* qa) {
  double d = qa[0];
  return d > 0.0 ? mk(qa[1] / d, qa[2] / d) : mk(0.0, 0.0);
}

template <typename T>
__global__ void k_gcr_update_x_dev(MultiArgs m, int k, void* x, size_t n, const double* qa) {
  cpx<double> c[kMaxK];
#pragma unroll
  for (int j = 0; j < kMaxK; ++j) c[j] = j < k ? gcr_alpha(qa + 4 * j) : mk(0.0, 0.0);
  GRID_STRIDE(i, n) {
    cpx<double> acc = ld<T>(x, i);
#pragma unroll
    for (int j = 0; j < kMaxK; ++j)
      if (j < k) acc = acc + c[j] * ld<T>(m.v[j], i);
    st<T>(x, i, acc);
  }
}

// value of c after a store in T and a load back (rounding to T)
template <typename T>
__device__ __forceinline__ cpx<double> rnd(cpx<double> c) {
  return mk((double)(T)c.r, (double)(T)c.i);
}

// One GCR step after the multi-dot: beta[2j] = <q_j, y> for the ktot basis
// slots, beta[2 ktot] = <y, y>, beta[2 ktot + 2] = <r, y>.  This launch takes
// the slots j0 .. j0 + k - 1 (m.v): y -= sum_j c_j q_j, c_j = <q_j, y> /
// ||q_j||^2.  The last launch of the step (last = 1) also forms
//   ||y_orth||^2 = <y, y> - sum_j |<q_j, y>|^2 / ||q_j||^2   (in order of j),
//   <y_orth, r>  = <y, r>                                    (r is orthogonal to every q_j),
// applies r -= alpha y_orth with alpha = <y_orth, r> / ||y_orth||^2, reduces
// ||r||^2 into o, and (block 0) writes {||y_orth||^2, <y_orth, r>} to
// qa[4 ktot ..] and the c_j to cj[0 .. ktot).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_gcr_step_dev(MultiArgs m, int j0, int k, int ktot, void* y, void* r,
                                                           size_t n, const double* beta, double* qa, double* cj,
                                                           int last, const RedOut o) {
  cpx<double> c[kMaxK];
#pragma unroll
  for (int j = 0; j < kMaxK; ++j) {
    const double d = j < k ? qa[4 * (j0 + j)] : 0.0;
    c[j] = (j < k && d > 0.0) ? mk(beta[2 * (j0 + j)] / d, beta[2 * (j0 + j) + 1] / d) : mk(0.0, 0.0);
  }
  cpx<double> alpha = mk(0.0, 0.0);
  double qq = 0.0;
  cpx<double> qr = mk(0.0, 0.0);
  if (last) {
    qq = beta[2 * ktot];
    for (int j = 0; j < ktot; ++j) {
      const double d = qa[4 * j];
      if (d > 0.0) {
        const double br = beta[2 * j], bi = beta[2 * j + 1];
        qq -= (br * br + bi * bi) / d;
      }
    }
    qr = mk(beta[2 * ktot + 2], -beta[2 * ktot + 3]);
    if (qq > 0.0) alpha = mk(qr.r / qq, qr.i / qq);
    if (blockIdx.x == 0) {
      if (threadIdx.x == 0) {
        qa[4 * ktot] = qq;
        qa[4 * ktot + 1] = qr.r;
        qa[4 * ktot + 2] = qr.i;
      }
      for (int j = threadIdx.x; j < ktot; j += blockDim.x) {
        const double d = qa[4 * j];
        cj[2 * j] = d > 0.0 ? beta[2 * j] / d : 0.0;
        cj[2 * j + 1] = d > 0.0 ? beta[2 * j + 1] / d : 0.0;
      }
    }
  }
  double v[1] = {0.0};
  GRID_STRIDE(i, n) {
    cpx<double> a = ld<T>(y, i);
#pragma unroll
    for (int j = 0; j < kMaxK; ++j)
      if (j < k) a = a - c[j] * ld<T>(m.v[j], i);
    st<T>(y, i, a);
    if (last) {
      const cpx<double> b = ld<T>(r, i) - alpha * rnd<T>(a);
      st<T>(r, i, b);
      const cpx<double> bs = rnd<T>(b);
      v[0] += bs.r * bs.r + bs.i * bs.i;
    }
  }
  if (last) block_reduce<1>(v, o);
}

// Coefficients of the solution update of a GCR cycle whose directions are kept
// as the raw preconditioned vectors z_j: with z~_j = z_j - sum_{i<j} c_ij z~_i
// (c_ij in cmat[j][i], complex) and x += sum_j alpha_j z~_j, x += sum_j y_j z_j
// where y solves (I + C) y = alpha by back substitution (alpha_j = 0 for the
// nf fixed slots, whose vectors are not orthogonalised).  One thread.
__global__ void k_gcr_coef_solve(const double* qa, const double* cmat, int ldc, double* y, int nf, int kt) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = kt - 1; i >= 0; --i) {
    cpx<double> s = i < nf ? mk(0.0, 0.0) : gcr_alpha(qa + 4 * i);
    for (int j = (i + 1 > nf ? i + 1 : nf); j < kt; ++j) {
      const cpx<double> cij = mk(cmat[2 * ((size_t)j * ldc + i)], cmat[2 * ((size_t)j * ldc + i) + 1]);
      s = s - cij * mk(y[2 * j], y[2 * j + 1]);
    }
    y[2 * i] = s.r;
    y[2 * i + 1] = s.i;
  }
}

// x += sum_j coef_j v_j (coef: complex, device)
template <typename T>
__global__ void k_multi_axpy_dev(MultiArgs m, int k, void* x, size_t n, const double* coef) {
  cpx<double> c[kMaxK];
#pragma unroll
  for (int j = 0; j < kMaxK; ++j) c[j] = j < k ? mk(coef[2 * j], coef[2 * j + 1]) : mk(0.0, 0.0);
  GRID_STRIDE(i, n) {
    cpx<double> acc = ld<T>(x, i);
#pragma unroll
    for (int j = 0; j < kMaxK; ++j)
      if (j < k) acc = acc + c[j] * ld<T>(m.v[j], i);
    st<T>(x, i, acc);
  }
}

// MR step with alpha = <Ar, r> / ||Ar||^2 read from coef = [re, im, ||Ar||^2]
template <typename T>
__global__ void k_mr_update_dev(const double* coef, void* x, void* r, const void* Ar, size_t n) {
  const double d = coef[2];
  cpx<double> a = d > 0.0 ? mk(coef[0] / d, coef[1] / d) : mk(0.0, 0.0);
  GRID_STRIDE(i, n) {
    st<T>(x, i, ld<T>(x, i) + a * ld<T>(r, i));
    st<T>(r, i, ld<T>(r, i) - a * ld<T>(Ar, i));
  }
}

template <typename T>
__global__ void k_mr_update(double ar, double ai, void* x, void* r, const void* Ar, size_t n) {
  cpx<double> a = mk(ar, ai);
  GRID_STRIDE(i, n) {
    st<T>(x, i, ld<T>(x, i) + a * ld<T>(r, i));
    st<T>(r, i, ld<T>(r, i) - a * ld<T>(Ar, i));
  }
}

}  // namespace

#define DISPATCH(prec, KERNEL, grid, ...)                                                       \
  do {                                                                                          \
    if ((prec) == WCMG_F64)                                                                     \
      hipLaunchKernelGGL(KERNEL<double>, grid, dim3(kThreads), 0, st, __VA_ARGS__);             \
    else                                                                                        \
      hipLaunchKernelGGL(KERNEL<float>, grid, dim3(kThreads), 0, st, __VA_ARGS__);              \
    HIPCHK(hipGetLastError());                                                                  \
  } while (0)


void blas_zero(int prec, void* x, size_t n, hipStream_t st) { DISPATCH(prec, k_zero, ew_grid(n), x, n); }
void blas_defl_coefs(const double* dots, double* qa, int K, hipStream_t st) {
  hipLaunchKernelGGL(k_defl_coefs, dim3((K + 63) / 64), dim3(64), 0, st, dots, qa, K);
  HIPCHK(hipGetLastError());
}
void blas_convert(int prec_dst, void* y, int prec_src, const void* x, size_t n, hipStream_t st) {
  const dim3 g = ew_grid(n);
  if (prec_dst == WCMG_F64 && prec_src == WCMG_F64)
    hipLaunchKernelGGL((k_convert<double, double>), g, dim3(kThreads), 0, st, y, x, n);
  else if (prec_dst == WCMG_F64)
    hipLaunchKernelGGL((k_convert<double, float>), g, dim3(kThreads), 0, st, y, x, n);
  else if (prec_src == WCMG_F64)
    hipLaunchKernelGGL((k_convert<float, double>), g, dim3(kThreads), 0, st, y, x, n);
  else
    hipLaunchKernelGGL((k_convert<float, float>), g, dim3(kThreads), 0, st, y, x, n);
  HIPCHK(hipGetLastError());
}
void blas_copy(int prec, void* y, const void* x, size_t n, hipStream_t st) {
  DISPATCH(prec, k_copy, ew_grid(n), y, x, n);
}
void blas_axpby(int prec, double ar, double ai, const void* x, double br, double bi, void* y, size_t n,
                hipStream_t st) {
  DISPATCH(prec, k_axpby, ew_grid(n), ar, ai, x, br, bi, y, n);
}
void blas_norm2(int prec, const void* x, size_t n, const RedOut& o, hipStream_t st) {
  DISPATCH(prec, k_norm2, red_grid(n), x, n, o);
}
void blas_cdot(int prec, const void* x, const void* y, size_t n, const RedOut& o, hipStream_t st) {
  DISPATCH(prec, k_cdot, red_grid(n), x, y, n, o);
}
void blas_cdot_norm(int prec, const void* x, const void* y, size_t n, const RedOut& o, hipStream_t st) {
  DISPATCH(prec, k_cdot_norm, red_grid(n), x, y, n, o);
}
void blas_multi_cdot(int prec, const void* const* v, int k, const void* y, size_t n, const RedOut& o,
                     hipStream_t st) {
  for (int j0 = 0; j0 < k; j0 += kMaxK) {
    int kk = std::min(kMaxK, k - j0);
    MultiArgs m{};
    for (int j = 0; j < kk; ++j) m.v[j] = v[j0 + j];
    // all 2*kMaxK slots are written; only the first 2*kk are meaningful
    DISPATCH(prec, k_multi_cdot, red_grid(n), m, kk, y, n, o.at(2 * j0));
  }
}
void blas_multi_axpy(int prec, const double* c, const void* const* v, int k, void* y, size_t n, hipStream_t st) {
  for (int j0 = 0; j0 < k; j0 += kMaxK) {
    int kk = std::min(kMaxK, k - j0);
    MultiArgs m{};
    for (int j = 0; j < kk; ++j) {
      m.v[j] = v[j0 + j];
      m.c[2 * j] = c[2 * (j0 + j)];
      m.c[2 * j + 1] = c[2 * (j0 + j) + 1];
    }
    DISPATCH(prec, k_multi_axpy, ew_grid(n), m, kk, y, n);
  }
}
void blas_axpy_norm(int prec, double ar, double ai, const void* x, void* y, size_t n, const RedOut& o,
                    hipStream_t st) {
  DISPATCH(prec, k_axpy_norm, red_grid(n), ar, ai, x, y, n, o);
}
void blas_bicg_update(int prec, double ar, double ai, double wr, double wi, const void* p, const void* s,
                      const void* t, void* x, void* r, const void* rhat, size_t n, const RedOut& o, hipStream_t st) {
  DISPATCH(prec, k_bicg_update, red_grid(n), ar, ai, wr, wi, p, s, t, x, r, rhat, n, o);
}
void blas_bicg_p(int prec, double br, double bi, double wr, double wi, const void* r, const void* v, void* p,
                 size_t n, hipStream_t st) {
  DISPATCH(prec, k_bicg_p, ew_grid(n), br, bi, wr, wi, r, v, p, n);
}
void blas_mr_update(int prec, double ar, double ai, void* x, void* r, const void* Ar, size_t n, hipStream_t st) {
  DISPATCH(prec, k_mr_update, ew_grid(n), ar, ai, x, r, Ar, n);
}

void blas_gcr_update_x_dev(int prec, const void* const* z, int k, void* x, size_t n, const double* qa,
                           hipStream_t st) {
  for (int j0 = 0; j0 < k; j0 += kMaxK) {
    int kk = std::min(kMaxK, k - j0);
    MultiArgs m{};
    for (int j = 0; j < kk; ++j) m.v[j] = z[j0 + j];
    DISPATCH(prec, k_gcr_update_x_dev, ew_grid(n), m, kk, x, n, qa + 4 * j0);
  }
}

void blas_gcr_step_dev(int prec, const void* const* q, int k, void* y, void* r, size_t n, const double* beta,
                       double* qa, double* cj, const RedOut& o, hipStream_t st) {
  if (k == 0) {
    MultiArgs m{};
    DISPATCH(prec, k_gcr_step_dev, red_grid(n), m, 0, 0, 0, y, r, n, beta, qa, cj, 1, o);
    return;
  }
  for (int j0 = 0; j0 < k; j0 += kMaxK) {
    const int kk = std::min(kMaxK, k - j0);
    MultiArgs m{};
    for (int j = 0; j < kk; ++j) m.v[j] = q[j0 + j];
    const int last = j0 + kk == k;
    DISPATCH(prec, k_gcr_step_dev, red_grid(n), m, j0, kk, k, y, r, n, beta, qa, cj, last, o);
  }
}

void blas_gcr_update_x_raw(int prec, const void* const* z, int nf, int kt, void* x, size_t n, const double* qa,
                           const double* cmat, int ldc, double* y, hipStream_t st) {
  if (kt <= 0) return;
  hipLaunchKernelGGL(k_gcr_coef_solve, dim3(1), dim3(64), 0, st, qa, cmat, ldc, y, nf, kt);
  HIPCHK(hipGetLastError());
  for (int j0 = 0; j0 < kt; j0 += kMaxK) {
    const int kk = std::min(kMaxK, kt - j0);
    MultiArgs m{};
    for (int j = 0; j < kk; ++j) m.v[j] = z[j0 + j];
    DISPATCH(prec, k_multi_axpy_dev, ew_grid(n), m, kk, x, n, y + 2 * j0);
  }
}

void blas_mr_update_dev(int prec, const double* coef, void* x, void* r, const void* Ar, size_t n, hipStream_t st) {
  DISPATCH(prec, k_mr_update_dev, ew_grid(n), coef, x, r, Ar, n);
}

}  // namespace wcmg
