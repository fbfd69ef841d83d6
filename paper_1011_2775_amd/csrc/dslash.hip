// Fine Wilson-clover hopping kernels (red-black paragraph, Eqs.(2)-(3)).
//
// One thread computes one output site of parity p for a group of NR
// right-hand sides (the links and clover blocks of the site are loaded once
// and applied to every right-hand side of the group):
//
//   out(x) = DIAG(x) + coeff * POST[ -1/2 sum_mu (1-gamma_mu) U_mu(x) in(x+mu)
//                                     + (1+gamma_mu) U_mu(x-mu)^dag in(x-mu) ]
//
// DIAG = 0 (none), 1 (xin(x)), 2 (A_p(x) xin(x));  POST = identity or the
// clover inverse A_p(x)^-1.  With these, the three pieces of the reduced
// operator D_r = 1 - D_eo D_oo^-1 D_oe D_ee^-1 are single launches:
//   w   = A_oo^-1 H_oe z            (DIAG 0, POST inverse, coeff 1)
//   out = y - H_eo w                (DIAG 1, coeff -1)
// and the full operator of Eq.(1) on one parity is DIAG 2, coeff 1.
//
// Spin projection in the chiral basis, gamma_mu = [[0, B],[B^dag, 0]]:
//   (1 - gamma) psi = [h ; -B^dag h],  h = psi_up - B psi_down
//   (1 + gamma) psi = [h ;  B^dag h],  h = psi_up + B psi_down
// so each direction multiplies only a half spinor (2 spins x 3 colours) by
// the link.  B_x = -i sigma_1, B_y = -i sigma_2, B_z = -i sigma_3, B_t = 1.
#include "wcmg_internal.h"
#include "kernels.h"
#include "hop_core.h"
#include "blas_common.h"

namespace wcmg {

// The direction terms are pure arithmetic, so the compiler is free to sink
// them all below the last load, which keeps every direction's spinor and
// link live at once (hundreds of registers, one wave per SIMD).  An empty
// asm that reads and redefines the accumulator after each direction forces
// that direction's arithmetic to complete there, so its operands die; loads
// of the next direction may still be issued early.  The arithmetic and its
// order are unchanged.
template <typename C>
__device__ __forceinline__ void pin_acc(cpx<C> acc[12]) {
#pragma unroll
  for (int k = 0; k < 12; ++k) asm volatile("" : "+v"(acc[k].r), "+v"(acc[k].i));
}

template <typename S, typename C>
__device__ __forceinline__ C to_f_or_d(S v) {
  return (C)v;
}
template <>
__device__ __forceinline__ float to_f_or_d<__half, float>(__half v) {
  return __half2float(v);
}

template <typename S>
__device__ __forceinline__ const void* rhs_ptr(const void* base, size_t stride, int r) {
  return reinterpret_cast<const char*>(base) + (size_t)r * stride;
}

template <typename S, typename G, int MU, int NR, bool STREAM, bool PIN = true>
__device__ __forceinline__ void hop_mu(const DslashArgs& a, int p, int i, const int c[4], int g0, int nr,
                                       cpx<typename Compute<S>::T> (&acc)[NR][12]) {
  using C = typename Compute<S>::T;
  const DGeom& g = a.g;
  cpx<C> psi[12], h[6], hu[6], U[9];
  // forward: (1 - gamma_mu) U_mu(x) in(x + mu)
  {
    int n[4] = {c[0], c[1], c[2], c[3]};
    n[MU] = (n[MU] + 1 == g.L[MU]) ? 0 : n[MU] + 1;
    const int nb = cb_index(g, n);
    load_link<G, C, STREAM>(a.gauge, g.Vh, p, MU, i, U);
    const bool edge = MU == 3 && c[3] == g.L[3] - 1;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r < nr) {
        SpinorIO<S>::load(rhs_ptr<S>(a.in, a.rstride, g0 + r), g.Vh, nb, psi);
        project<C, MU, false>(psi, h);
        link_mul<C, false>(U, h, hu);
        if (edge) {
          const C ph = (C)g.t_bc;
#pragma unroll
          for (int k = 0; k < 6; ++k) hu[k] = ph * hu[k];
        }
        if (MU < 3 && g.hs != 1.0) {  // spatial hop coefficient (anisotropic lattices only)
          const C hs = (C)g.hs;
#pragma unroll
          for (int k = 0; k < 6; ++k) hu[k] = hs * hu[k];
        }
        accumulate<C, MU, false>(acc[r], hu);
        if constexpr (PIN) pin_acc(acc[r]);
      }
    }
  }
  // backward: (1 + gamma_mu) U_mu(x - mu)^dag in(x - mu)
  {
    int n[4] = {c[0], c[1], c[2], c[3]};
    n[MU] = (n[MU] == 0) ? g.L[MU] - 1 : n[MU] - 1;
    const int nb = cb_index(g, n);
    load_link<G, C, STREAM>(a.gauge, g.Vh, 1 - p, MU, nb, U);
    const bool edge = MU == 3 && c[3] == 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r < nr) {
        SpinorIO<S>::load(rhs_ptr<S>(a.in, a.rstride, g0 + r), g.Vh, nb, psi);
        project<C, MU, true>(psi, h);
        link_mul<C, true>(U, h, hu);
        if (edge) {
          const C ph = (C)g.t_bc;
#pragma unroll
          for (int k = 0; k < 6; ++k) hu[k] = ph * hu[k];
        }
        if (MU < 3 && g.hs != 1.0) {
          const C hs = (C)g.hs;
#pragma unroll
          for (int k = 0; k < 6; ++k) hu[k] = hs * hu[k];
        }
        accumulate<C, MU, true>(acc[r], hu);
        if constexpr (PIN) pin_acc(acc[r]);
      }
    }
  }
}

// Packed clover (kind 0 = A, 1 = A^-1) of one site: per chirality 6 real
// diagonal entries then 15 strictly lower complex entries (36 reals), both
// chiralities in 72 reals stored as 16-byte chunks [p][kind][chunk][Vh].
template <typename G>
struct CloverChunk;
template <>
struct CloverChunk<double> {
  using V = double2;
  static constexpr int E = 2;
};
template <>
struct CloverChunk<float> {
  using V = float4;
  static constexpr int E = 4;
};
template <>
struct CloverChunk<__half> {
  using V = uint4;
  static constexpr int E = 8;
};

template <typename G, typename C>
__device__ __forceinline__ void unpack_chunk(const typename CloverChunk<G>::V& v, C* d);
template <>
__device__ __forceinline__ void unpack_chunk<double, double>(const double2& v, double* d) {
  d[0] = v.x;
  d[1] = v.y;
}
template <>
__device__ __forceinline__ void unpack_chunk<float, float>(const float4& v, float* d) {
  d[0] = v.x;
  d[1] = v.y;
  d[2] = v.z;
  d[3] = v.w;
}
template <>
__device__ __forceinline__ void unpack_chunk<__half, float>(const uint4& v, float* d) {
  const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float2 f = __half22float2(*reinterpret_cast<const __half2*>(&w[k]));
    d[2 * k] = f.x;
    d[2 * k + 1] = f.y;
  }
}

// apply one chirality block (36 reals in d) to NR vectors
template <typename C, int NR>
__device__ __forceinline__ void clover_block_apply_d(const C* d, int chi, int nr, const cpx<C> (&in)[NR][12],
                                                     cpx<C> (&out)[NR][12]) {
  const int o = 6 * chi;
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (r < nr)
#pragma unroll
      for (int k = 0; k < 6; ++k) out[r][o + k] = mk(d[k] * in[r][o + k].r, d[k] * in[r][o + k].i);
  int t = 0;
#pragma unroll
  for (int rr = 1; rr < 6; ++rr) {
#pragma unroll
    for (int s = 0; s < rr; ++s) {
      const cpx<C> L = mk(d[6 + 2 * t], d[7 + 2 * t]);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r < nr) {
          cfma(out[r][o + rr], L, in[r][o + s]);   // lower entry (rr,s)
          cfmac(out[r][o + s], L, in[r][o + rr]);  // upper entry (s,rr) = conj(L)
        }
      }
      ++t;
    }
  }
}

template <typename G, typename C, int NR, bool STREAM = false>
__device__ __forceinline__ void clover_multi(const void* clov, int Vh, int p, int kind, int i, int nr,
                                             const cpx<C> (&in)[NR][12], cpx<C> (&out)[NR][12]) {
  using V = typename CloverChunk<G>::V;
  constexpr int E = CloverChunk<G>::E;
  constexpr int NCH = 72 / E;
  const V* base = reinterpret_cast<const V*>(clov) + (size_t)(p * 2 + kind) * NCH * Vh + i;
  if constexpr (E == 8) {
    // FP16: the two chirality blocks share a chunk, load all 72 reals at once
    C d[72];
#pragma unroll
    for (int c = 0; c < NCH; ++c) unpack_chunk<G, C>(ld_maybe<STREAM>(base + (size_t)c * Vh), d + E * c);
    clover_block_apply_d<C, NR>(d, 0, nr, in, out);
    clover_block_apply_d<C, NR>(d + 36, 1, nr, in, out);
  } else {
#pragma unroll
    for (int chi = 0; chi < 2; ++chi) {
      C d[36];
#pragma unroll
      for (int c = 0; c < 36 / E; ++c)
        unpack_chunk<G, C>(ld_maybe<STREAM>(base + (size_t)(chi * (36 / E) + c) * Vh), d + E * c);
      clover_block_apply_d<C, NR>(d, chi, nr, in, out);
    }
  }
}

// S: spinor storage, G: link and clover storage (G = S, or FP16 fields with
// FP32 spinors); lb: the lattice's logical block
// RED (DIAG = 1, one right-hand side): also add <out, x> and ||out||^2 of the
// site, in FP64 from the stored values, to red[0..3)
// g0: first right-hand side of the thread's group (-1: blockIdx.y * NR)
template <typename S, typename G, int DIAG, bool POSTINV, int NR, bool STREAM = false, bool RED = false,
          bool PIN = true>
__device__ __forceinline__ void dslash_site(const DslashArgs& a, int lb, double* red = nullptr, int g0 = -1) {
  using C = typename Compute<S>::T;
  const int i = lb * blockDim.x + threadIdx.x;
  if (lb >= a.nblocks || i >= a.g.Vh) return;
  if (g0 < 0) g0 = blockIdx.y * NR;
  const int nr = min(NR, a.nrhs - g0);
  const int p = a.parity;
  int c[4];
  cb_coords(a.g, i, p, c);

  cpx<C> acc[NR][12];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[r][k] = mk((C)0, (C)0);
  hop_mu<S, G, 0, NR, STREAM, PIN>(a, p, i, c, g0, nr, acc);
  hop_mu<S, G, 1, NR, STREAM, PIN>(a, p, i, c, g0, nr, acc);
  hop_mu<S, G, 2, NR, STREAM, PIN>(a, p, i, c, g0, nr, acc);
  hop_mu<S, G, 3, NR, STREAM, PIN>(a, p, i, c, g0, nr, acc);

  const C f = (C)(-0.5 * a.coeff);
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[r][k] = f * acc[r][k];

  cpx<C> out[NR][12];
  if constexpr (POSTINV) {
    clover_multi<G, C, NR, STREAM>(a.clov, a.g.Vh, p, 1, i, nr, acc, out);
  } else {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int k = 0; k < 12; ++k) out[r][k] = acc[r][k];
  }
  if constexpr (DIAG != 0) {
    cpx<C> xv[NR][12];
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (r < nr) SpinorIO<S>::template load<STREAM>(rhs_ptr<S>(a.x, a.rstride, g0 + r), a.g.Vh, i, xv[r]);
    if constexpr (DIAG == 2) {
      cpx<C> ax[NR][12];
      clover_multi<G, C, NR, STREAM>(a.clov, a.g.Vh, p, 0, i, nr, xv, ax);
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < 12; ++k) out[r][k] = out[r][k] + ax[r][k];
    } else {
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < 12; ++k) out[r][k] = out[r][k] + xv[r][k];
      if constexpr (RED) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          const double orr = (double)(S)out[0][k].r, oi = (double)(S)out[0][k].i;
          const double xr = (double)xv[0][k].r, xi = (double)xv[0][k].i;
          red[0] += orr * xr + oi * xi;
          red[1] += orr * xi - oi * xr;
          red[2] += orr * orr + oi * oi;
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (r < nr)
      SpinorIO<S>::template store<STREAM>(const_cast<void*>(rhs_ptr<S>(a.out, a.rstride, g0 + r)), a.g.Vh, i, out[r]);
}

template <typename S, typename G, int DIAG, bool POSTINV, int NR, bool STREAM>
__global__ void __launch_bounds__(256) dslash_kernel(DslashArgs a) {
  dslash_site<S, G, DIAG, POSTINV, NR, STREAM>(a, xcd_block(a.nblocks));
}

// Small lattices (a few workgroups per compute unit, so one or two wavefronts
// per SIMD whatever the register count): the directions are not pinned, so
// the compiler may issue the loads of all eight hops before their arithmetic
// and more of the gather is in flight at once.  Same arithmetic, same order,
// same bits as dslash_kernel.
template <typename S, typename G, int DIAG, bool POSTINV, bool STREAM>
__global__ void __launch_bounds__(256) dslash_kernel_wide(DslashArgs a) {
  dslash_site<S, G, DIAG, POSTINV, 1, STREAM, false, false>(a, xcd_block(a.nblocks));
}

// Several right-hand sides, one per thread: logical workgroup L handles site
// block L / nrhs of right-hand side L % nrhs, so the nrhs workgroups of a site
// block are consecutive, land on one XCD (xcd_block) and run close together:
// the first to read a link or clover record brings it into that XCD's L2 and
// the others find it there, while every thread keeps the register budget of
// the single-right-hand-side kernel.
template <typename S, typename G, int DIAG, bool POSTINV, bool STREAM>
__global__ void __launch_bounds__(256) dslash_kernel_rhs(DslashArgs a) {
  const int L = xcd_block(a.nblocks * a.nrhs);
  dslash_site<S, G, DIAG, POSTINV, 1, STREAM>(a, L / a.nrhs, nullptr, L % a.nrhs);
}

// The DIAG = 1 hop of D_r with the minimal-residual sums of the smoother
// fused in: out = x + coeff H in, and <out, x>, ||out||^2 reduced into o in
// the same launch (every block, padding blocks included, takes part in the
// reduction; the last to arrive finishes it).
template <typename S, typename G, bool STREAM, bool PIN = true>
__global__ void __launch_bounds__(256) dslash_red_kernel(DslashArgs a, RedOut o) {
  double v[3] = {0.0, 0.0, 0.0};
  dslash_site<S, G, 1, false, 1, STREAM, true, PIN>(a, xcd_block(a.nblocks), v);
  blas_detail::block_reduce<3>(v, o);
}

// Several lattices of different volumes in one launch: a work list of block
// ranges, workgroup b serving lattice l with off[l] <= b < off[l+1].
template <typename S, typename G, int DIAG, bool POSTINV>
__global__ void __launch_bounds__(256) dslash_multi_kernel(DslashMulti m) {
  int l = 0;
  while (l + 1 < m.nl && (int)blockIdx.x >= m.off[l + 1]) ++l;
  dslash_site<S, G, DIAG, POSTINV, 1>(m.a[l], (int)blockIdx.x - m.off[l]);
}

// out_p = A_p^(kind) in_p   (site-local clover or clover inverse), NR right-hand sides per thread
template <typename S, typename G, int NR>
__global__ void __launch_bounds__(256) clover_kernel(void* out, const void* in, const void* clov, int Vh, int p,
                                                     int kind, int nrhs, size_t rstride) {
  using C = typename Compute<S>::T;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vh) return;
  const int g0 = blockIdx.y * NR;
  const int nr = min(NR, nrhs - g0);
  cpx<C> v[NR][12], o[NR][12];
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (r < nr) SpinorIO<S>::load(rhs_ptr<S>(in, rstride, g0 + r), Vh, i, v[r]);
  clover_multi<G, C, NR>(clov, Vh, p, kind, i, nr, v, o);
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (r < nr) SpinorIO<S>::store(const_cast<void*>(rhs_ptr<S>(out, rstride, g0 + r)), Vh, i, o[r]);
}

// Several right-hand sides, one per thread, in interleaved workgroups (as
// dslash_kernel_rhs): the nrhs workgroups of a site block are consecutive, so
// the clover records they share are read once from HBM and then from L2.
template <typename S, typename G>
__global__ void __launch_bounds__(256) clover_kernel_rhs(void* out, const void* in, const void* clov, int Vh, int p,
                                                         int kind, int nrhs, size_t rstride, int nblocks) {
  using C = typename Compute<S>::T;
  const int L = xcd_block(nblocks * nrhs);
  const int lb = L / nrhs, r = L - lb * nrhs;
  const int i = lb * blockDim.x + threadIdx.x;
  if (lb >= nblocks || i >= Vh) return;
  cpx<C> v[1][12], o[1][12];
  SpinorIO<S>::load(rhs_ptr<S>(in, rstride, r), Vh, i, v[0]);
  clover_multi<G, C, 1>(clov, Vh, p, kind, i, 1, v, o);
  SpinorIO<S>::store(const_cast<void*>(rhs_ptr<S>(out, rstride, r)), Vh, i, o[0]);
}

// The smoother's minimal-residual update of the previous step fused into the
// first kernel of the next D_r: with a = coef[0..2) / coef[2] (0 when
// coef[2] is not positive), per site e += a r, r -= a Ar (FP64 arithmetic on
// the stored values, rounded back to storage), then out = A_ee^-1 r.
template <typename S, typename G>
__global__ void __launch_bounds__(256) clover_mr_kernel(void* out, void* r, void* e, const void* Ar,
                                                        const double* coef, const void* clov, int Vh, int p) {
  using C = typename Compute<S>::T;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vh) return;
  const double d = coef[2];
  const cpx<double> a = d > 0.0 ? mk(coef[0] / d, coef[1] / d) : mk(0.0, 0.0);
  cpx<C> rv[1][12], ev[12], av[12], o[1][12];
  SpinorIO<S>::load(r, Vh, i, rv[0]);
  SpinorIO<S>::load(e, Vh, i, ev);
  SpinorIO<S>::load(Ar, Vh, i, av);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const cpx<double> rk = mk((double)rv[0][k].r, (double)rv[0][k].i);
    const cpx<double> ek = mk((double)ev[k].r, (double)ev[k].i) + a * rk;
    const cpx<double> rn = rk - a * mk((double)av[k].r, (double)av[k].i);
    ev[k] = mk((C)(S)ek.r, (C)(S)ek.i);
    rv[0][k] = mk((C)(S)rn.r, (C)(S)rn.i);
  }
  SpinorIO<S>::store(e, Vh, i, ev);
  SpinorIO<S>::store(r, Vh, i, rv[0]);
  clover_multi<G, C, 1>(clov, Vh, p, 1, i, 1, rv, o);
  SpinorIO<S>::store(out, Vh, i, o[0]);
}

bool launch_clover_mr(int prec, void* out, void* r, void* e, const void* Ar, const double* coef, const void* clov,
                      int Vh, int p, int fprec, hipStream_t st) {
  const int fp = fprec < 0 ? prec : fprec;
  const dim3 grid((Vh + 255) / 256);
  if (prec == WCMG_F64 && fp == WCMG_F64)
    hipLaunchKernelGGL((clover_mr_kernel<double, double>), grid, dim3(256), 0, st, out, r, e, Ar, coef, clov, Vh, p);
  else if (prec == WCMG_F32 && fp == WCMG_F32)
    hipLaunchKernelGGL((clover_mr_kernel<float, float>), grid, dim3(256), 0, st, out, r, e, Ar, coef, clov, Vh, p);
  else if (prec == WCMG_F32 && fp == WCMG_F16)
    hipLaunchKernelGGL((clover_mr_kernel<float, __half>), grid, dim3(256), 0, st, out, r, e, Ar, coef, clov, Vh, p);
  else
    return false;
  HIPCHK(hipGetLastError());
  return true;
}

// right-hand sides per thread: FP64 keeps at most 2 in registers, FP32/FP16 4
template <typename S>
constexpr int max_group() {
  return sizeof(S) == 8 ? 2 : 4;
}

// compute units of the current device (queried once)
static int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
    cus = n > 0 ? n : 1;
  }
  return cus;
}

// a single-right-hand-side grid of at most two 256-thread workgroups per compute unit
static bool small_grid(const DslashArgs& a) { return a.nrhs == 1 && (a.g.Vh + 255) / 256 <= 2 * device_cus(); }

template <typename S, typename G, int NR>
static void launch_dslash_nr(int diag, bool postinv, DslashArgs a, hipStream_t st) {
  const int threads = a.threads > 0 ? a.threads : 256;
  if (threads != 64 && threads != 128 && threads != 256) fail(WCMG_EINVAL, "unsupported Dslash block size");
  a.nblocks = (a.g.Vh + threads - 1) / threads;
  dim3 grid(xcd_grid(a.nblocks), (a.nrhs + NR - 1) / NR);
  if constexpr (NR == 1) {
    if (small_grid(a)) {
      const bool stream = a.stream > 0;
#define WCMG_DW(D, P)                                                                               \
  do {                                                                                            \
    if (stream)                                                                                   \
      hipLaunchKernelGGL((dslash_kernel_wide<S, G, D, P, true>), grid, dim3(threads), 0, st, a);  \
    else                                                                                          \
      hipLaunchKernelGGL((dslash_kernel_wide<S, G, D, P, false>), grid, dim3(threads), 0, st, a); \
  } while (0)
      if (diag == 0 && !postinv) WCMG_DW(0, false);
      else if (diag == 0 && postinv) WCMG_DW(0, true);
      else if (diag == 1 && !postinv) WCMG_DW(1, false);
      else if (diag == 1 && postinv) WCMG_DW(1, true);
      else if (diag == 2 && !postinv) WCMG_DW(2, false);
      else WCMG_DW(2, true);
#undef WCMG_DW
      HIPCHK(hipGetLastError());
      return;
    }
  }
  // stream the fields and the output past the caches when the fields (links and both
  // clover records, both parities) exceed three quarters of the 256 MB Infinity Cache
  const bool stream = a.stream >= 0 ? a.stream != 0 : (double)a.g.Vh * 432.0 * sizeof(G) > 192.0e6;
#define WCMG_DS(D, P)                                                                                  \
  do {                                                                                               \
    if (stream)                                                                                      \
      hipLaunchKernelGGL((dslash_kernel<S, G, D, P, NR, true>), grid, dim3(threads), 0, st, a);    \
    else                                                                                             \
      hipLaunchKernelGGL((dslash_kernel<S, G, D, P, NR, false>), grid, dim3(threads), 0, st, a);   \
  } while (0)
  if (diag == 0 && !postinv) WCMG_DS(0, false);
  else if (diag == 0 && postinv) WCMG_DS(0, true);
  else if (diag == 1 && !postinv) WCMG_DS(1, false);
  else if (diag == 1 && postinv) WCMG_DS(1, true);
  else if (diag == 2 && !postinv) WCMG_DS(2, false);
  else WCMG_DS(2, true);
#undef WCMG_DS
  HIPCHK(hipGetLastError());
}

template <typename S, typename G>
static void launch_dslash_rhs(int diag, bool postinv, DslashArgs a, hipStream_t st) {
  const int threads = a.threads > 0 ? a.threads : 256;
  if (threads != 64 && threads != 128 && threads != 256) fail(WCMG_EINVAL, "unsupported Dslash block size");
  a.nblocks = (a.g.Vh + threads - 1) / threads;
  if ((long)a.nblocks * a.nrhs > (1L << 30)) fail(WCMG_EINVAL, "too many workgroups");
  const dim3 grid(xcd_grid(a.nblocks * a.nrhs));
  // the right-hand sides of a site block reuse its links and clover records
  // from L2, so the fields are not streamed past the caches unless asked for
  const bool stream = a.stream > 0;
#define WCMG_DR(D, P)                                                                                 \
  do {                                                                                              \
    if (stream)                                                                                     \
      hipLaunchKernelGGL((dslash_kernel_rhs<S, G, D, P, true>), grid, dim3(threads), 0, st, a);     \
    else                                                                                            \
      hipLaunchKernelGGL((dslash_kernel_rhs<S, G, D, P, false>), grid, dim3(threads), 0, st, a);    \
  } while (0)
  if (diag == 0 && !postinv) WCMG_DR(0, false);
  else if (diag == 0 && postinv) WCMG_DR(0, true);
  else if (diag == 1 && !postinv) WCMG_DR(1, false);
  else if (diag == 1 && postinv) WCMG_DR(1, true);
  else if (diag == 2 && !postinv) WCMG_DR(2, false);
  else WCMG_DR(2, true);
#undef WCMG_DR
  HIPCHK(hipGetLastError());
}

template <typename S, typename G>
static void launch_dslash_t(int diag, bool postinv, const DslashArgs& a, hipStream_t st) {
  // several right-hand sides: one per thread, interleaved workgroups, unless a group size is asked for
  if (a.nrhs > 1 && (a.group == 0 || a.group == -1)) return launch_dslash_rhs<S, G>(diag, postinv, a, st);
  int g = a.nrhs >= max_group<S>() ? max_group<S>() : (a.nrhs >= 2 ? 2 : 1);
  if (a.group > 0) g = std::min(a.group, max_group<S>());
  if (g == 1) launch_dslash_nr<S, G, 1>(diag, postinv, a, st);
  else if (g == 2) launch_dslash_nr<S, G, 2>(diag, postinv, a, st);
  else launch_dslash_nr<S, G, max_group<S>()>(diag, postinv, a, st);
}

void launch_dslash(int prec, int diag, bool postinv, const DslashArgs& a, hipStream_t st) {
  if (a.nrhs < 1) fail(WCMG_EINVAL, "nrhs must be >= 1");
  const int fp = a.fprec < 0 ? prec : a.fprec;
  if (prec == WCMG_F64 && fp == WCMG_F64) launch_dslash_t<double, double>(diag, postinv, a, st);
  else if (prec == WCMG_F32 && fp == WCMG_F32) launch_dslash_t<float, float>(diag, postinv, a, st);
  else if (prec == WCMG_F32 && fp == WCMG_F16) launch_dslash_t<float, __half>(diag, postinv, a, st);
  else if (prec == WCMG_F16 && fp == WCMG_F16) launch_dslash_t<__half, __half>(diag, postinv, a, st);
  else fail(WCMG_EINVAL, "unsupported spinor / field precision pair");
}

template <typename S, typename G>
static void launch_dslash_red_t(DslashArgs a, const RedOut& o, hipStream_t st) {
  const bool stream = a.stream >= 0 ? a.stream != 0 : (double)a.g.Vh * 432.0 * sizeof(G) > 192.0e6;
  dim3 grid(xcd_grid(a.nblocks));
  if (small_grid(a)) {
    if (stream)
      hipLaunchKernelGGL((dslash_red_kernel<S, G, true, false>), grid, dim3(256), 0, st, a, o);
    else
      hipLaunchKernelGGL((dslash_red_kernel<S, G, false, false>), grid, dim3(256), 0, st, a, o);
  } else if (stream) {
    hipLaunchKernelGGL((dslash_red_kernel<S, G, true>), grid, dim3(256), 0, st, a, o);
  } else {
    hipLaunchKernelGGL((dslash_red_kernel<S, G, false>), grid, dim3(256), 0, st, a, o);
  }
  HIPCHK(hipGetLastError());
}

bool launch_dslash_red(int prec, const DslashArgs& a0, const RedOut& o, hipStream_t st) {
  if (a0.nrhs != 1) return false;
  DslashArgs a = a0;
  a.threads = 256;
  a.group = 1;
  a.nblocks = (a.g.Vh + 255) / 256;
  // per-block partials: three doubles per block of the padded grid
  if ((size_t)xcd_grid(a.nblocks) * 3 > (size_t)kRedBlocks * 64) return false;
  const int fp = a.fprec < 0 ? prec : a.fprec;
  if (prec == WCMG_F64 && fp == WCMG_F64) launch_dslash_red_t<double, double>(a, o, st);
  else if (prec == WCMG_F32 && fp == WCMG_F32) launch_dslash_red_t<float, float>(a, o, st);
  else if (prec == WCMG_F32 && fp == WCMG_F16) launch_dslash_red_t<float, __half>(a, o, st);
  else return false;
  return true;
}

template <typename S, typename G, int NR>
static void launch_clover_nr(void* out, const void* in, const void* clov, int Vh, int p, int kind, int nrhs,
                             size_t rstride, hipStream_t st) {
  dim3 grid((Vh + 255) / 256, (nrhs + NR - 1) / NR);
  hipLaunchKernelGGL((clover_kernel<S, G, NR>), grid, dim3(256), 0, st, out, in, clov, Vh, p, kind, nrhs, rstride);
}

template <typename S, typename G>
static void launch_clover_t(void* out, const void* in, const void* clov, int Vh, int p, int kind, int nrhs,
                            size_t rstride, hipStream_t st) {
  if (nrhs > 1) {
    const int nb = (Vh + 255) / 256;
    hipLaunchKernelGGL((clover_kernel_rhs<S, G>), dim3(xcd_grid(nb * nrhs)), dim3(256), 0, st, out, in, clov, Vh, p,
                       kind, nrhs, rstride, nb);
    return;
  }
  if (nrhs >= max_group<S>()) launch_clover_nr<S, G, max_group<S>()>(out, in, clov, Vh, p, kind, nrhs, rstride, st);
  else if (nrhs >= 2) launch_clover_nr<S, G, 2>(out, in, clov, Vh, p, kind, nrhs, rstride, st);
  else launch_clover_nr<S, G, 1>(out, in, clov, Vh, p, kind, nrhs, rstride, st);
}

void launch_clover(int prec, void* out, const void* in, const void* clov, int Vh, int p, int kind, hipStream_t st,
                   int nrhs, size_t rstride, int fprec) {
  if (nrhs < 1) fail(WCMG_EINVAL, "nrhs must be >= 1");
  const int fp = fprec < 0 ? prec : fprec;
  if (prec == WCMG_F64 && fp == WCMG_F64) launch_clover_t<double, double>(out, in, clov, Vh, p, kind, nrhs, rstride, st);
  else if (prec == WCMG_F32 && fp == WCMG_F32) launch_clover_t<float, float>(out, in, clov, Vh, p, kind, nrhs, rstride, st);
  else if (prec == WCMG_F32 && fp == WCMG_F16) launch_clover_t<float, __half>(out, in, clov, Vh, p, kind, nrhs, rstride, st);
  else if (prec == WCMG_F16 && fp == WCMG_F16) launch_clover_t<__half, __half>(out, in, clov, Vh, p, kind, nrhs, rstride, st);
  else fail(WCMG_EINVAL, "unsupported spinor / field precision pair");
  HIPCHK(hipGetLastError());
}

template <typename S, typename G>
__global__ void __launch_bounds__(256) clover_multi_kernel(CloverMulti m) {
  using C = typename Compute<S>::T;
  int l = 0;
  while (l + 1 < m.nl && (int)blockIdx.x >= m.off[l + 1]) ++l;
  const int i = ((int)blockIdx.x - m.off[l]) * blockDim.x + threadIdx.x;
  if (i >= m.Vh[l]) return;
  cpx<C> v[1][12], o[1][12];
  SpinorIO<S>::load(m.in[l], m.Vh[l], i, v[0]);
  clover_multi<G, C, 1>(m.clov[l], m.Vh[l], m.parity, m.kind, i, 1, v, o);
  SpinorIO<S>::store(m.out[l], m.Vh[l], i, o[0]);
}

template <typename S, typename G>
static void launch_multi_t(int diag, bool postinv, DslashMulti m, hipStream_t st) {
  int total = 0;
  for (int l = 0; l < m.nl; ++l) {
    m.a[l].nblocks = (m.a[l].g.Vh + 255) / 256;
    m.a[l].nrhs = 1;
    m.off[l] = total;
    total += m.a[l].nblocks;
  }
  m.off[m.nl] = total;
#define WCMG_DM(D, P) hipLaunchKernelGGL((dslash_multi_kernel<S, G, D, P>), dim3(total), dim3(256), 0, st, m)
  if (diag == 0 && !postinv) WCMG_DM(0, false);
  else if (diag == 0 && postinv) WCMG_DM(0, true);
  else if (diag == 1 && !postinv) WCMG_DM(1, false);
  else if (diag == 1 && postinv) WCMG_DM(1, true);
  else if (diag == 2 && !postinv) WCMG_DM(2, false);
  else WCMG_DM(2, true);
#undef WCMG_DM
  HIPCHK(hipGetLastError());
}

void launch_dslash_multi(int prec, int diag, bool postinv, const DslashMulti& m, hipStream_t st) {
  if (m.nl < 1 || m.nl > kMaxMulti) fail(WCMG_EINVAL, "lattice count out of range");
  if (prec == WCMG_F64) launch_multi_t<double, double>(diag, postinv, m, st);
  else if (prec == WCMG_F32) launch_multi_t<float, float>(diag, postinv, m, st);
  else launch_multi_t<__half, __half>(diag, postinv, m, st);
}

void launch_clover_multi(int prec, CloverMulti m, hipStream_t st) {
  if (m.nl < 1 || m.nl > kMaxMulti) fail(WCMG_EINVAL, "lattice count out of range");
  int total = 0;
  for (int l = 0; l < m.nl; ++l) {
    m.off[l] = total;
    total += (m.Vh[l] + 255) / 256;
  }
  m.off[m.nl] = total;
  if (prec == WCMG_F64)
    hipLaunchKernelGGL((clover_multi_kernel<double, double>), dim3(total), dim3(256), 0, st, m);
  else if (prec == WCMG_F32)
    hipLaunchKernelGGL((clover_multi_kernel<float, float>), dim3(total), dim3(256), 0, st, m);
  else
    hipLaunchKernelGGL((clover_multi_kernel<__half, __half>), dim3(total), dim3(256), 0, st, m);
  HIPCHK(hipGetLastError());
}

}  // namespace wcmg
