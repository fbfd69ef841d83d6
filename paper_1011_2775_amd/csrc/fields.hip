// Field layout conversion and the clover term (site-diagonal D_ee, D_oo of
// the red-black paragraph).
//
// The clover kernel builds, per site, Fhat_mu_nu = (Q_mu_nu - Q_mu_nu^dag)/8
// from the four plaquette leaves, then the two chirality blocks
//   A_s = (4 + m0) 1_6 + sum_{mu<nu} S_s(mu,nu) (x) Fhat_mu_nu,
//   S_s(mu,nu) = csw (i/2) sigma_mu_nu restricted to chirality s,
// (equal to csw (i/4) sum_{mu != nu} sigma (x) Fhat) and their inverses by a
// Cholesky factorisation, all in FP64.
#include "kernels.h"
#include "su3.h"

namespace wcmg {

namespace {
constexpr int kT = 256;

template <typename S>
__device__ __forceinline__ typename Vec2<S>::T from_c(double r, double i);
template <>
__device__ __forceinline__ double2 from_c<double>(double r, double i) { return make_double2(r, i); }
template <>
__device__ __forceinline__ float2 from_c<float>(double r, double i) { return make_float2((float)r, (float)i); }
template <>
__device__ __forceinline__ __half2 from_c<__half>(double r, double i) {
  return __floats2half2_rn((float)r, (float)i);
}

template <typename S>
__global__ void k_gauge_to_internal(void* dst, const double2* canon, DGeom g, int V) {
  using V2 = typename Vec2<S>::T;
  int lex = blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= V) return;
  int c[4];
  coords_of(g.L, lex, c);
  int p = (c[0] + c[1] + c[2] + c[3]) & 1;
  int cb = lex >> 1;
  V2* d = reinterpret_cast<V2*>(dst);
  for (int mu = 0; mu < 4; ++mu)
    for (int k = 0; k < 9; ++k) {
      double2 u = canon[((size_t)lex * 4 + mu) * 9 + k];
      d[((size_t)(p * 4 + mu) * 9 + k) * g.Vh + cb] = from_c<S>(u.x, u.y);
    }
}

template <typename S>
__global__ void k_spinor_to_internal(void* even, void* odd, const double2* canon, DGeom g, int V, int g5) {
  using C = typename Compute<S>::T;
  int lex = blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= V) return;
  int c[4];
  coords_of(g.L, lex, c);
  int p = (c[0] + c[1] + c[2] + c[3]) & 1;
  cpx<C> v[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    double2 t = canon[(size_t)lex * 12 + k];
    C sg = (g5 && k >= 6) ? (C)-1 : (C)1;
    v[k] = mk((C)(sg * t.x), (C)(sg * t.y));
  }
  SpinorIO<S>::store(p ? odd : even, g.Vh, lex >> 1, v);
}

template <typename S>
__global__ void k_spinor_from_internal(double2* canon, const void* even, const void* odd, DGeom g, int V, int g5) {
  using C = typename Compute<S>::T;
  int lex = blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= V) return;
  int c[4];
  coords_of(g.L, lex, c);
  int p = (c[0] + c[1] + c[2] + c[3]) & 1;
  const void* src = p ? odd : even;
  cpx<C> v[12];
  if (src) {
    SpinorIO<S>::load(src, g.Vh, lex >> 1, v);
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = mk((C)0, (C)0);
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    double sg = (g5 && k >= 6) ? -1.0 : 1.0;
    canon[(size_t)lex * 12 + k] = make_double2(sg * (double)v[k].r, sg * (double)v[k].i);
  }
}

template <typename SD, typename SS>
__global__ void k_spinor_convert(void* dst, const void* src, int Vh) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vh) return;
  using CS = typename Compute<SS>::T;
  using CD = typename Compute<SD>::T;
  cpx<CS> v[12];
  SpinorIO<SS>::load(src, Vh, i, v);
  cpx<CD> w[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) w[k] = mk((CD)v[k].r, (CD)v[k].i);
  SpinorIO<SD>::store(dst, Vh, i, w);
}

template <typename S>
__global__ void k_spinor_chiral(void* dst, const void* src, int Vh, int chi, int flip_lower) {
  using C = typename Compute<S>::T;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vh) return;
  cpx<C> v[12];
  SpinorIO<S>::load(src, Vh, i, v);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    int s = k >= 6;
    if (flip_lower) {
      if (s) v[k] = mk(-v[k].r, -v[k].i);
    } else if (s != chi) {
      v[k] = mk((C)0, (C)0);
    }
  }
  SpinorIO<S>::store(dst, Vh, i, v);
}

// ---------------------------------------------------------------- clover
// Fhat_mu_nu(x) = (Q - Q^dag)/8, Q = sum of the four leaves
__device__ C3 fhat(const double2* gauge, const DGeom& g, const int x[4], int mu, int nu) {
  int xpm[4], xpn[4], xmm[4], xmn[4], xmm_pn[4], xmm_mn[4], xpm_mn[4];
  shift(g.L, x, mu, 1, xpm);
  shift(g.L, x, nu, 1, xpn);
  shift(g.L, x, mu, -1, xmm);
  shift(g.L, x, nu, -1, xmn);
  shift(g.L, xmm, nu, 1, xmm_pn);
  shift(g.L, xmm, nu, -1, xmm_mn);
  shift(g.L, xpm, nu, -1, xpm_mn);
  C3 q1 = mul(mul(load_u(gauge, g, x, mu), load_u(gauge, g, xpm, nu)),
              mul(dagm(load_u(gauge, g, xpn, mu)), dagm(load_u(gauge, g, x, nu))));
  C3 q2 = mul(mul(load_u(gauge, g, x, nu), dagm(load_u(gauge, g, xmm_pn, mu))),
              mul(dagm(load_u(gauge, g, xmm, nu)), load_u(gauge, g, xmm, mu)));
  C3 q3 = mul(mul(dagm(load_u(gauge, g, xmm, mu)), dagm(load_u(gauge, g, xmm_mn, nu))),
              mul(load_u(gauge, g, xmm_mn, mu), load_u(gauge, g, xmn, nu)));
  C3 q4 = mul(mul(dagm(load_u(gauge, g, xmn, nu)), load_u(gauge, g, xmn, mu)),
              mul(load_u(gauge, g, xpm_mn, nu), dagm(load_u(gauge, g, x, mu))));
  C3 f;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cpx<double> q = q1.m[i * 3 + j] + q2.m[i * 3 + j] + q3.m[i * 3 + j] + q4.m[i * 3 + j];
      cpx<double> qt = q1.m[j * 3 + i] + q2.m[j * 3 + i] + q3.m[j * 3 + i] + q4.m[j * 3 + i];
      f.m[i * 3 + j] = 0.125 * (q - cconj(qt));
    }
  return f;
}

// Hermitian 6x6 in packed lower form: d[6] real diagonal, l[15] strictly lower
struct Herm6 {
  double d[6];
  cpx<double> l[15];
};
__device__ __forceinline__ int tri(int r, int s) { return r * (r - 1) / 2 + s; }

// inverse through Cholesky; returns false if not positive definite
__device__ bool herm6_inverse(const Herm6& A, Herm6& Ainv) {
  double Ld[6];
  cpx<double> Ll[15];
  for (int j = 0; j < 6; ++j) {
    double s = A.d[j];
    for (int k = 0; k < j; ++k) {
      cpx<double> v = Ll[tri(j, k)];
      s -= v.r * v.r + v.i * v.i;
    }
    if (!(s > 0.0)) return false;
    Ld[j] = sqrt(s);
    for (int i = j + 1; i < 6; ++i) {
      cpx<double> t = A.l[tri(i, j)];
      for (int k = 0; k < j; ++k) {
        // t -= L[i][k] conj(L[j][k])
        cpx<double> a = Ll[tri(i, k)], b = Ll[tri(j, k)];
        t = t - mk(a.r * b.r + a.i * b.i, a.i * b.r - a.r * b.i);
      }
      Ll[tri(i, j)] = (1.0 / Ld[j]) * t;
    }
  }
  // M = L^-1 (lower)
  double Md[6];
  cpx<double> Ml[15];
  for (int i = 0; i < 6; ++i) Md[i] = 1.0 / Ld[i];
  for (int j = 0; j < 6; ++j) {
    for (int i = j + 1; i < 6; ++i) {
      // M[i][j] = -(sum_{k=j}^{i-1} L[i][k] M[k][j]) / L[i][i]
      cpx<double> s = Ll[tri(i, j)] * mk(Md[j], 0.0);
      for (int k = j + 1; k < i; ++k) s = s + Ll[tri(i, k)] * Ml[tri(k, j)];
      Ml[tri(i, j)] = (-Md[i]) * s;
    }
  }
  // Ainv[i][j] = sum_{k>=i} conj(M[k][i]) M[k][j], i >= j
  for (int i = 0; i < 6; ++i) {
    double s = 0.0;
    for (int k = i; k < 6; ++k) {
      cpx<double> m = (k == i) ? mk(Md[i], 0.0) : Ml[tri(k, i)];
      s += m.r * m.r + m.i * m.i;
    }
    Ainv.d[i] = s;
    for (int j = 0; j < i; ++j) {
      cpx<double> t = mk(0.0, 0.0);
      for (int k = i; k < 6; ++k) {
        cpx<double> mi = (k == i) ? mk(Md[i], 0.0) : Ml[tri(k, i)];
        cpx<double> mj = Ml[tri(k, j)];
        cfmac(t, mi, mj);
      }
      Ainv.l[tri(i, j)] = t;
    }
  }
  return true;
}

// Packed clover record of a site: 72 reals per (parity, kind), chirality
// block chi at reals chi*36 .. chi*36+35 (6 diagonal, then the 15 strictly
// lower complex entries), stored as 16-byte chunks [p][kind][chunk][Vh]
// holding E = 16 / sizeof(real) consecutive reals (FP64 2, FP32 4, FP16 8).
__device__ __forceinline__ size_t clover_real_index(int pk, int K, int Vh, int i, int E) {
  return (((size_t)pk * (72 / E) + K / E) * Vh + i) * E + K % E;
}

__device__ void store_herm6(double* clov, const DGeom& g, int p, int kind, int chi, int i, const Herm6& h) {
  const int pk = p * 2 + kind, o = chi * 36;
  for (int k = 0; k < 6; ++k) clov[clover_real_index(pk, o + k, g.Vh, i, 2)] = h.d[k];
  for (int t = 0; t < 15; ++t) {
    clov[clover_real_index(pk, o + 6 + 2 * t, g.Vh, i, 2)] = h.l[t].r;
    clov[clover_real_index(pk, o + 7 + 2 * t, g.Vh, i, 2)] = h.l[t].i;
  }
}

// FP64 chunked clover -> the chunked layout of precision S
template <typename S>
__global__ void k_clover_relayout(S* dst, const double* src, int Vh) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)4 * 72 * Vh) return;
  const int i = (int)(t % Vh);
  const int K = (int)((t / Vh) % 72);
  const int pk = (int)(t / ((size_t)Vh * 72));
  dst[clover_real_index(pk, K, Vh, i, 16 / sizeof(S))] = (S)src[clover_real_index(pk, K, Vh, i, 2)];
}

__global__ void __launch_bounds__(128) k_clover(double* clov, const double2* gauge, DGeom g, int V, double diag,
                                                CloverCoef cc, int* flag) {
  int lex = blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= V) return;
  int x[4];
  coords_of(g.L, lex, x);
  int p = (x[0] + x[1] + x[2] + x[3]) & 1;
  int cb = lex >> 1;
  for (int chi = 0; chi < 2; ++chi) {
    Herm6 A;
    for (int k = 0; k < 6; ++k) A.d[k] = diag;
    for (int t = 0; t < 15; ++t) A.l[t] = mk(0.0, 0.0);
    int plane = 0;
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = mu + 1; nu < 4; ++nu, ++plane) {
        C3 F = fhat(gauge, g, x, mu, nu);
        // entry (s1*3+a, s2*3+b) += S[s1][s2] * F[a][b]
        for (int s1 = 0; s1 < 2; ++s1)
          for (int s2 = 0; s2 < 2; ++s2) {
            cpx<double> sv = mk(cc.s[plane][chi][s1 * 2 + s2][0], cc.s[plane][chi][s1 * 2 + s2][1]);
            for (int a = 0; a < 3; ++a)
              for (int b = 0; b < 3; ++b) {
                int r = s1 * 3 + a, q = s2 * 3 + b;
                cpx<double> v = sv * F.m[a * 3 + b];
                if (r == q) A.d[r] += v.r;
                else if (r > q) A.l[tri(r, q)] = A.l[tri(r, q)] + v;
              }
          }
      }
    Herm6 Ai;
    bool ok = herm6_inverse(A, Ai);
    if (!ok) {
      *flag = 1;  // benign race: every writer stores 1
      for (int k = 0; k < 6; ++k) Ai.d[k] = 0.0;
      for (int t = 0; t < 15; ++t) Ai.l[t] = mk(0.0, 0.0);
    }
    store_herm6(clov, g, p, 0, chi, cb, A);
    store_herm6(clov, g, p, 1, chi, cb, Ai);
  }
}

__global__ void __launch_bounds__(128) k_clover_from_matrix(double* clov, const double2* Amat, DGeom g, int V,
                                                            int* flag) {
  int lex = blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= V) return;
  int x[4];
  coords_of(g.L, lex, x);
  int p = (x[0] + x[1] + x[2] + x[3]) & 1;
  const double2* M = Amat + (size_t)lex * 144;
  for (int chi = 0; chi < 2; ++chi) {
    Herm6 A;
    int o = chi * 6;
    for (int r = 0; r < 6; ++r) {
      A.d[r] = M[(o + r) * 12 + o + r].x;
      for (int q = 0; q < r; ++q) {
        double2 v = M[(o + r) * 12 + o + q];
        A.l[tri(r, q)] = mk(v.x, v.y);
      }
    }
    Herm6 Ai;
    if (!herm6_inverse(A, Ai)) {
      *flag = 1;  // benign race: every writer stores 1
      for (int k = 0; k < 6; ++k) Ai.d[k] = 0.0;
      for (int t = 0; t < 15; ++t) Ai.l[t] = mk(0.0, 0.0);
    }
    store_herm6(clov, g, p, 0, chi, lex >> 1, A);
    store_herm6(clov, g, p, 1, chi, lex >> 1, Ai);
  }
}

template <typename S>
__global__ void k_reals_convert(S* dst, const double* src, size_t n);
template <>
__global__ void k_reals_convert<double>(double* dst, const double* src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
template <>
__global__ void k_reals_convert<float>(float* dst, const double* src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}
template <>
__global__ void k_reals_convert<__half>(__half* dst, const double* src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = __float2half_rn((float)src[i]);
}

inline dim3 grid_for(size_t n, int t = kT) { return dim3((unsigned)((n + t - 1) / t)); }

}  // namespace

void gauge_to_internal(int prec, void* dst, const void* canon, const Geom& g, hipStream_t st) {
  DGeom d = dgeom(g);
  auto c = reinterpret_cast<const double2*>(canon);
  if (prec == WCMG_F64)
    hipLaunchKernelGGL(k_gauge_to_internal<double>, grid_for(g.V), dim3(kT), 0, st, dst, c, d, g.V);
  else if (prec == WCMG_F32)
    hipLaunchKernelGGL(k_gauge_to_internal<float>, grid_for(g.V), dim3(kT), 0, st, dst, c, d, g.V);
  else
    hipLaunchKernelGGL(k_gauge_to_internal<__half>, grid_for(g.V), dim3(kT), 0, st, dst, c, d, g.V);
  HIPCHK(hipGetLastError());
}

void spinor_to_internal(int prec, void* even, void* odd, const void* canon, const Geom& g, bool g5,
                        hipStream_t st) {
  DGeom d = dgeom(g);
  auto c = reinterpret_cast<const double2*>(canon);
  if (prec == WCMG_F64)
    hipLaunchKernelGGL(k_spinor_to_internal<double>, grid_for(g.V), dim3(kT), 0, st, even, odd, c, d, g.V, (int)g5);
  else if (prec == WCMG_F32)
    hipLaunchKernelGGL(k_spinor_to_internal<float>, grid_for(g.V), dim3(kT), 0, st, even, odd, c, d, g.V, (int)g5);
  else
    hipLaunchKernelGGL(k_spinor_to_internal<__half>, grid_for(g.V), dim3(kT), 0, st, even, odd, c, d, g.V,
                       (int)g5);
  HIPCHK(hipGetLastError());
}

void spinor_from_internal(int prec, void* canon, const void* even, const void* odd, const Geom& g, bool g5,
                          hipStream_t st) {
  DGeom d = dgeom(g);
  auto c = reinterpret_cast<double2*>(canon);
  if (prec == WCMG_F64)
    hipLaunchKernelGGL(k_spinor_from_internal<double>, grid_for(g.V), dim3(kT), 0, st, c, even, odd, d, g.V,
                       (int)g5);
  else if (prec == WCMG_F32)
    hipLaunchKernelGGL(k_spinor_from_internal<float>, grid_for(g.V), dim3(kT), 0, st, c, even, odd, d, g.V,
                       (int)g5);
  else
    hipLaunchKernelGGL(k_spinor_from_internal<__half>, grid_for(g.V), dim3(kT), 0, st, c, even, odd, d, g.V,
                       (int)g5);
  HIPCHK(hipGetLastError());
}

void spinor_convert(int pd, void* dst, int ps, const void* src, int Vh, hipStream_t st) {
  dim3 gr = grid_for(Vh), bl(kT);
#define CV(SD, SS) hipLaunchKernelGGL((k_spinor_convert<SD, SS>), gr, bl, 0, st, dst, src, Vh)
  if (pd == WCMG_F64 && ps == WCMG_F64) CV(double, double);
  else if (pd == WCMG_F64 && ps == WCMG_F32) CV(double, float);
  else if (pd == WCMG_F64 && ps == WCMG_F16) CV(double, __half);
  else if (pd == WCMG_F32 && ps == WCMG_F64) CV(float, double);
  else if (pd == WCMG_F32 && ps == WCMG_F32) CV(float, float);
  else if (pd == WCMG_F32 && ps == WCMG_F16) CV(float, __half);
  else if (pd == WCMG_F16 && ps == WCMG_F64) CV(__half, double);
  else if (pd == WCMG_F16 && ps == WCMG_F32) CV(__half, float);
  else CV(__half, __half);
#undef CV
  HIPCHK(hipGetLastError());
}

void spinor_gamma5(int prec, void* v, int Vh, hipStream_t st) {
  if (prec == WCMG_F64)
    hipLaunchKernelGGL(k_spinor_chiral<double>, grid_for(Vh), dim3(kT), 0, st, v, v, Vh, 0, 1);
  else if (prec == WCMG_F32)
    hipLaunchKernelGGL(k_spinor_chiral<float>, grid_for(Vh), dim3(kT), 0, st, v, v, Vh, 0, 1);
  else
    hipLaunchKernelGGL(k_spinor_chiral<__half>, grid_for(Vh), dim3(kT), 0, st, v, v, Vh, 0, 1);
  HIPCHK(hipGetLastError());
}

void spinor_chiral_project(int prec, void* dst, const void* src, int Vh, int chi, hipStream_t st) {
  if (prec == WCMG_F64)
    hipLaunchKernelGGL(k_spinor_chiral<double>, grid_for(Vh), dim3(kT), 0, st, dst, src, Vh, chi, 0);
  else if (prec == WCMG_F32)
    hipLaunchKernelGGL(k_spinor_chiral<float>, grid_for(Vh), dim3(kT), 0, st, dst, src, Vh, chi, 0);
  else
    hipLaunchKernelGGL(k_spinor_chiral<__half>, grid_for(Vh), dim3(kT), 0, st, dst, src, Vh, chi, 0);
  HIPCHK(hipGetLastError());
}

void clover_compute(void* clov64, const void* gauge64, const Geom& g, double m0, const CloverCoef& cc, int* flag,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_clover, grid_for(g.V, 128), dim3(128), 0, st, reinterpret_cast<double*>(clov64),
                     reinterpret_cast<const double2*>(gauge64), dgeom(g), g.V,
                     g.hs == 1.0 ? 4.0 + m0 : m0 + 1.0 + 3.0 * g.hs, cc, flag);
  HIPCHK(hipGetLastError());
}

void clover_from_matrix(void* clov64, const void* A, const Geom& g, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_clover_from_matrix, grid_for(g.V, 128), dim3(128), 0, st, reinterpret_cast<double*>(clov64),
                     reinterpret_cast<const double2*>(A), dgeom(g), g.V, flag);
  HIPCHK(hipGetLastError());
}

void reals_convert(int prec, void* dst, const double* src, size_t n, hipStream_t st) {
  size_t b = std::min<size_t>((n + kT - 1) / kT, 65536);
  if (prec == WCMG_F64)
    hipLaunchKernelGGL(k_reals_convert<double>, dim3(b), dim3(kT), 0, st, (double*)dst, src, n);
  else if (prec == WCMG_F32)
    hipLaunchKernelGGL(k_reals_convert<float>, dim3(b), dim3(kT), 0, st, (float*)dst, src, n);
  else
    hipLaunchKernelGGL(k_reals_convert<__half>, dim3(b), dim3(kT), 0, st, (__half*)dst, src, n);
  HIPCHK(hipGetLastError());
}

void clover_relayout(int prec, void* dst, const double* src, int Vh, hipStream_t st) {
  const size_t n = (size_t)4 * 72 * Vh;
  const dim3 gr((unsigned)((n + kT - 1) / kT));
  if (prec == WCMG_F32)
    hipLaunchKernelGGL(k_clover_relayout<float>, gr, dim3(kT), 0, st, (float*)dst, src, Vh);
  else if (prec == WCMG_F16)
    hipLaunchKernelGGL(k_clover_relayout<__half>, gr, dim3(kT), 0, st, (__half*)dst, src, Vh);
  else
    fail(WCMG_EINVAL, "clover relayout targets F32 or F16");
  HIPCHK(hipGetLastError());
}

void launch_reals_convert(int prec, void* dst, const double* src, size_t n, hipStream_t st) {
  reals_convert(prec, dst, src, n, st);
}

}  // namespace wcmg
