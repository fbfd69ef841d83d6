// Coarse-level stencil (red-black paragraph and Implementation paragraph):
//
//   (Yhat v)(c) = X(c) v(c) + sum_d Y_d(c) v(c + d),   d = +-x, +-y, +-z, +-t
//
// stored per coarse site as 8 hop blocks of 2Nv x 2Nv complex, column-major
// (entry (i, j) at j*n + i), so that the lanes that own consecutive rows
// read consecutive addresses.  The red-black solver uses the hops
// Ytilde_d(c) = Y_d(c) X(c+d)^-1, which are exactly the hops of the coarse
// D_p = Yhat X^-1, so that
//   D_r_hat = 1 - Ytilde_eo Ytilde_oe        (two launches)
//   b_r_hat = b_e - Ytilde_eo b_o
//   c_e = X_ee^-1 y_e,  c_o = X_oo^-1 (b_o - Ytilde_oe y_e).
//
// A coarse site is computed by `split` workgroups (1, 2 or 4), each owning
// n/split consecutive rows, so that small coarse lattices still occupy every
// CU: the 8 neighbour vectors are gathered into LDS, G column groups of
// n/(2 split) lanes (two rows per lane) split the 8n columns, and the
// partial rows are summed in LDS.
#include "kernels.h"

namespace wcmg {

namespace {

// two consecutive complex entries (rows 2r, 2r+1 of one column)
__device__ __forceinline__ void load2(const float2* p, cpx<float>& e0, cpx<float>& e1) {
  float4 t = *reinterpret_cast<const float4*>(p);
  e0 = mk(t.x, t.y);
  e1 = mk(t.z, t.w);
}
__device__ __forceinline__ void load2(const double2* p, cpx<double>& e0, cpx<double>& e1) {
  double2 t0 = p[0], t1 = p[1];
  e0 = mk(t0.x, t0.y);
  e1 = mk(t1.x, t1.y);
}

// Thread t owns the row pair (2r, 2r+1), r = t mod n/2, and the column
// group g = t div n/2; the G groups stride over the 8n hop columns (and the
// n columns of X for DIAG 2), so each lane keeps several 16-byte loads in
// flight.  Up to 1024 lanes (16 wavefronts) work on one coarse site.
// RB = 1 marks the launches of the red-black reduced operator (the solver's
// hot path), so that profiles separate them from the other uses
template <typename S, int RB>
__global__ void __launch_bounds__(1024) k_coarse_hop(void* out, const void* in, const void* x, const void* M,
                                                     const void* Xm, int diag, double coeff, int site0, int n,
                                                     const int* nbr, size_t vs, int split, int G) {
  using C = typename Compute<S>::T;
  using V2 = typename Vec2<S>::T;
  extern __shared__ char smem[];
  cpx<C>* vin = reinterpret_cast<cpx<C>*>(smem);  // 9n: 8 neighbour vectors, then x(c)
  cpx<C>* part = vin + 9 * n;                       // G * rows partial rows
  const int c = site0 + blockIdx.x / split;
  const int rows = n / split, row0 = (blockIdx.x % split) * rows;
  const int R2 = rows >> 1;  // lanes g * R2 .. g * R2 + R2 - 1 form column group g < G
  // right-hand side blockIdx.y of a batch, vs elements apart
  const size_t ro = (size_t)blockIdx.y * vs;
  const V2* vi = reinterpret_cast<const V2*>(in) + (in ? ro : 0);
  const V2* vx = reinterpret_cast<const V2*>(x) + (x ? ro : 0);
  out = reinterpret_cast<V2*>(out) + ro;
  if (M) {
    for (int t = threadIdx.x; t < 8 * n; t += blockDim.x) {
      int d = t / n, j = t - d * n;
      V2 w = vi[(size_t)nbr[(size_t)c * 8 + d] * n + j];
      vin[t] = mk((C)w.x, (C)w.y);
    }
  }
  if (diag == 2) {
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      V2 w = vx[(size_t)c * n + t];
      vin[8 * n + t] = mk((C)w.x, (C)w.y);
    }
  }
  __syncthreads();
  const int g = threadIdx.x / R2, rp = threadIdx.x - g * R2;
  if (g < G) {
    cpx<C> a0 = mk((C)0, (C)0), a1 = a0, d0 = a0, d1 = a0;
    if (M) {
      const V2* m = reinterpret_cast<const V2*>(M) + (size_t)c * 8 * n * n + row0 + 2 * rp;
#pragma unroll 4
      for (int col = g; col < 8 * n; col += G) {
        cpx<C> e0, e1;
        load2(m + (size_t)col * n, e0, e1);
        const cpx<C> v = vin[col];
        cfma(a0, e0, v);
        cfma(a1, e1, v);
      }
    }
    if (diag == 2) {
      const V2* m = reinterpret_cast<const V2*>(Xm) + (size_t)c * n * n + row0 + 2 * rp;
      for (int col = g; col < n; col += G) {
        cpx<C> e0, e1;
        load2(m + (size_t)col * n, e0, e1);
        const cpx<C> v = vin[8 * n + col];
        cfma(d0, e0, v);
        cfma(d1, e1, v);
      }
    }
    part[g * rows + 2 * rp] = (C)coeff * a0 + d0;
    part[g * rows + 2 * rp + 1] = (C)coeff * a1 + d1;
  }
  // fixed-order tree over the G (a power of two) column groups
  for (int h = G >> 1; h > 0; h >>= 1) {
    __syncthreads();
    if (g < h) {
      part[g * rows + 2 * rp] = part[g * rows + 2 * rp] + part[(g + h) * rows + 2 * rp];
      part[g * rows + 2 * rp + 1] = part[g * rows + 2 * rp + 1] + part[(g + h) * rows + 2 * rp + 1];
    }
  }
  if (g == 0) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int i = row0 + 2 * rp + k;
      cpx<C> s = part[2 * rp + k];
      if (diag == 1) {
        V2 w = vx[(size_t)c * n + i];
        s = s + mk((C)w.x, (C)w.y);
      }
      V2 o;
      o.x = (S)s.r;
      o.y = (S)s.i;
      reinterpret_cast<V2*>(out)[(size_t)c * n + i] = o;
    }
  }
}

// in-place Gauss-Jordan inversion with partial (row) pivoting, one workgroup
// per matrix; the storage order does not matter (inverse of the transpose is
// the transpose of the inverse)
__global__ void __launch_bounds__(256) k_inverse(double2* Mall, int n, int* flag) {
  double2* A = Mall + (size_t)blockIdx.x * n * n;
  __shared__ int piv[128];
  __shared__ double2 f[128];
  __shared__ double2 pinv;
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      int p = k;
      double best = -1.0;
      for (int r = k; r < n; ++r) {
        double2 v = A[(size_t)r * n + k];
        double m = v.x * v.x + v.y * v.y;
        if (m > best) {
          best = m;
          p = r;
        }
      }
      piv[k] = p;
      if (!(best > 0.0)) *flag = 1;
    }
    __syncthreads();
    const int p = piv[k];
    if (p != k) {
      for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double2 t = A[(size_t)k * n + j];
        A[(size_t)k * n + j] = A[(size_t)p * n + j];
        A[(size_t)p * n + j] = t;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double2 v = A[(size_t)k * n + k];
      double d = v.x * v.x + v.y * v.y;
      pinv = d > 0.0 ? make_double2(v.x / d, -v.y / d) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    // row k: A[k][k] = 1 then scale the row by 1/pivot
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      double2 v = (j == k) ? make_double2(1.0, 0.0) : A[(size_t)k * n + j];
      A[(size_t)k * n + j] = make_double2(v.x * pinv.x - v.y * pinv.y, v.x * pinv.y + v.y * pinv.x);
    }
    for (int r = threadIdx.x; r < n; r += blockDim.x) f[r] = A[(size_t)r * n + k];
    __syncthreads();
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
      int r = t / n, j = t - r * n;
      if (r == k) continue;
      double2 a = (j == k) ? make_double2(0.0, 0.0) : A[(size_t)r * n + j];
      double2 b = A[(size_t)k * n + j], fr = f[r];
      A[(size_t)r * n + j] = make_double2(a.x - (fr.x * b.x - fr.y * b.y), a.y - (fr.x * b.y + fr.y * b.x));
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k) {
      for (int r = threadIdx.x; r < n; r += blockDim.x) {
        double2 t = A[(size_t)r * n + k];
        A[(size_t)r * n + k] = A[(size_t)r * n + p];
        A[(size_t)r * n + p] = t;
      }
    }
    __syncthreads();
  }
}

// Yt[c][d] = Y[c][d] * Xinv[nb(c,d)], column-major n x n
__global__ void __launch_bounds__(256) k_right_mul(double2* Yt, const double2* Y, const double2* Xinv,
                                                   const int* nbr, int n) {
  const int c = blockIdx.x, d = blockIdx.y;
  const double2* y = Y + ((size_t)c * 8 + d) * n * n;
  const double2* xi = Xinv + (size_t)nbr[(size_t)c * 8 + d] * n * n;
  double2* o = Yt + ((size_t)c * 8 + d) * n * n;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int j = t / n, i = t - j * n;  // column-major element (i, j)
    cpx<double> s = mk(0.0, 0.0);
    for (int k = 0; k < n; ++k) {
      double2 a = y[(size_t)k * n + i], b = xi[(size_t)j * n + k];
      cfma(s, mk(a.x, a.y), mk(b.x, b.y));
    }
    o[t] = make_double2(s.r, s.i);
  }
}

// canonical complex128 [lex][n] <-> internal [perm[lex]][n] in double or float
template <typename S>
__global__ void k_coarse_canon(void* internal, double2* canon, const int* perm, int V, int n, int to_internal) {
  using V2 = typename Vec2<S>::T;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= V * n) return;
  int lex = t / n, a = t - lex * n;
  V2* in = reinterpret_cast<V2*>(internal) + (size_t)perm[lex] * n + a;
  if (to_internal) {
    double2 v = canon[t];
    V2 w;
    w.x = (S)v.x;
    w.y = (S)v.y;
    *in = w;
  } else {
    V2 w = *in;
    canon[t] = make_double2((double)w.x, (double)w.y);
  }
}

}  // namespace

void launch_coarse_canon(int prec, void* internal, void* canon, const int* perm, int V, int n, bool to_internal,
                         hipStream_t st) {
  dim3 grid((V * n + 255) / 256), block(256);
  if (prec == WCMG_F64)
    hipLaunchKernelGGL(k_coarse_canon<double>, grid, block, 0, st, internal, reinterpret_cast<double2*>(canon), perm,
                       V, n, (int)to_internal);
  else
    hipLaunchKernelGGL(k_coarse_canon<float>, grid, block, 0, st, internal, reinterpret_cast<double2*>(canon), perm,
                       V, n, (int)to_internal);
  HIPCHK(hipGetLastError());
}

void launch_coarse_hop(int prec, void* out, const void* in, const void* x, const void* M, const void* Xmat,
                       int diag, double coeff, int parity, const CoarseGeom& cg, const int* nbr, hipStream_t st,
                       int nrhs, size_t vs, bool rb) {
  const int n = cg.n;
  if (n % 2 || n > 256) fail(WCMG_EDIM, "coarse block size must be even and <= 256");
  int site0 = 0, nsites = cg.V;
  if (parity >= 0) {
    site0 = parity * cg.Vh;
    nsites = cg.Vh;
  }
  // rows per workgroup: split small lattices until about 1024 workgroups are in flight
  int split = 1;
  while (split < 4 && nsites * nrhs * split < 1024 && n % (4 * split) == 0) split *= 2;
  const int rows = n / split;
  const int R2 = rows / 2;
  // G column groups: the largest power of two with G * R2 <= 1024 and G <= 64
  int G = 1;
  while (G < 64 && 2 * G * R2 <= 1024) G *= 2;
  const int threads = ((G * R2 + 63) / 64) * 64;  // lanes beyond G * R2 idle
  const size_t cb = (prec == WCMG_F64) ? 16 : 8;
  const size_t shm = (size_t)(9 * n + G * rows) * cb;
  if (nsites == 0) return;
#define WCMG_CH(S, R)                                                                                          \
  hipLaunchKernelGGL((k_coarse_hop<S, R>), dim3(nsites * split, nrhs), dim3(threads), shm, st, out, in, x, M, Xmat, \
                     diag, coeff, site0, n, nbr, vs, split, G)
  if (prec == WCMG_F64) {
    if (rb) WCMG_CH(double, 1);
    else WCMG_CH(double, 0);
  } else {
    if (rb) WCMG_CH(float, 1);
    else WCMG_CH(float, 0);
  }
#undef WCMG_CH
  HIPCHK(hipGetLastError());
}

void launch_coarse_local(int prec, void* out, const void* in, const void* M, int parity, const CoarseGeom& cg,
                         hipStream_t st, int nrhs, size_t vs) {
  launch_coarse_hop(prec, out, nullptr, in, nullptr, M, 2, 0.0, parity, cg, nullptr, st, nrhs, vs);
}

void launch_batched_inverse(double* M, int nmat, int n, int* flag, hipStream_t st) {
  if (n > 128) fail(WCMG_EDIM, "coarse block too large to invert");
  hipLaunchKernelGGL(k_inverse, dim3(nmat), dim3(256), 0, st, reinterpret_cast<double2*>(M), n, flag);
  HIPCHK(hipGetLastError());
}

void launch_coarse_right_mul(double* Yt, const double* Y, const double* Xinv, const int* nbr, int V, int n,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_right_mul, dim3(V, 8), dim3(256), 0, st, reinterpret_cast<double2*>(Yt),
                     reinterpret_cast<const double2*>(Y), reinterpret_cast<const double2*>(Xinv), nbr, n);
  HIPCHK(hipGetLastError());
}

}  // namespace wcmg
