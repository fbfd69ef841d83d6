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

template <typename S, int MU, int NR>
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
    load_link<S, C>(a.gauge, g.Vh, p, MU, i, U);
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
        accumulate<C, MU, false>(acc[r], hu);
        pin_acc(acc[r]);
      }
    }
  }
  // backward: (1 + gamma_mu) U_mu(x - mu)^dag in(x - mu)
  {
    int n[4] = {c[0], c[1], c[2], c[3]};
    n[MU] = (n[MU] == 0) ? g.L[MU] - 1 : n[MU] - 1;
    const int nb = cb_index(g, n);
    load_link<S, C>(a.gauge, g.Vh, 1 - p, MU, nb, U);
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
        accumulate<C, MU, true>(acc[r], hu);
        pin_acc(acc[r]);
      }
    }
  }
}

// one 36-real chirality block of the packed clover, loaded once, applied to NR vectors
template <typename S, typename C, int NR>
__device__ __forceinline__ void clover_block_multi(const void* clov, int Vh, int p, int kind, int chi, int i,
                                                   int nr, const cpx<C> (&in)[NR][12], cpx<C> (&out)[NR][12]) {
  const S* c = reinterpret_cast<const S*>(clov) + ((size_t)(p * 2 + kind) * 72 + chi * 36) * Vh;
  const int o = 6 * chi;
  C d[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) d[k] = (C)to_f_or_d<S, C>(c[(size_t)k * Vh + i]);
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
      const cpx<C> L = mk((C)to_f_or_d<S, C>(c[(size_t)(6 + 2 * t) * Vh + i]),
                          (C)to_f_or_d<S, C>(c[(size_t)(7 + 2 * t) * Vh + i]));
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

template <typename S, typename C, int NR>
__device__ __forceinline__ void clover_multi(const void* clov, int Vh, int p, int kind, int i, int nr,
                                             const cpx<C> (&in)[NR][12], cpx<C> (&out)[NR][12]) {
  clover_block_multi<S, C, NR>(clov, Vh, p, kind, 0, i, nr, in, out);
  clover_block_multi<S, C, NR>(clov, Vh, p, kind, 1, i, nr, in, out);
}

template <typename S, int DIAG, bool POSTINV, int NR>
__global__ void __launch_bounds__(256) dslash_kernel(DslashArgs a) {
  using C = typename Compute<S>::T;
  const int lb = xcd_block(a.nblocks);
  const int i = lb * blockDim.x + threadIdx.x;
  if (lb >= a.nblocks || i >= a.g.Vh) return;
  const int g0 = blockIdx.y * NR;
  const int nr = min(NR, a.nrhs - g0);
  const int p = a.parity;
  int c[4];
  cb_coords(a.g, i, p, c);

  cpx<C> acc[NR][12];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[r][k] = mk((C)0, (C)0);
  hop_mu<S, 0, NR>(a, p, i, c, g0, nr, acc);
  hop_mu<S, 1, NR>(a, p, i, c, g0, nr, acc);
  hop_mu<S, 2, NR>(a, p, i, c, g0, nr, acc);
  hop_mu<S, 3, NR>(a, p, i, c, g0, nr, acc);

  const C f = (C)(-0.5 * a.coeff);
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[r][k] = f * acc[r][k];

  cpx<C> out[NR][12];
  if constexpr (POSTINV) {
    clover_multi<S, C, NR>(a.clov, a.g.Vh, p, 1, i, nr, acc, out);
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
      if (r < nr) SpinorIO<S>::load(rhs_ptr<S>(a.x, a.rstride, g0 + r), a.g.Vh, i, xv[r]);
    if constexpr (DIAG == 2) {
      cpx<C> ax[NR][12];
      clover_multi<S, C, NR>(a.clov, a.g.Vh, p, 0, i, nr, xv, ax);
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < 12; ++k) out[r][k] = out[r][k] + ax[r][k];
    } else {
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < 12; ++k) out[r][k] = out[r][k] + xv[r][k];
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (r < nr)
      SpinorIO<S>::store(const_cast<void*>(rhs_ptr<S>(a.out, a.rstride, g0 + r)), a.g.Vh, i, out[r]);
}

// out_p = A_p^(kind) in_p   (site-local clover or clover inverse), NR right-hand sides per thread
template <typename S, int NR>
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
  clover_multi<S, C, NR>(clov, Vh, p, kind, i, nr, v, o);
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (r < nr) SpinorIO<S>::store(const_cast<void*>(rhs_ptr<S>(out, rstride, g0 + r)), Vh, i, o[r]);
}

// right-hand sides per thread: FP64 keeps at most 2 in registers, FP32/FP16 4
template <typename S>
constexpr int max_group() {
  return sizeof(S) == 8 ? 2 : 4;
}

template <typename S, int NR>
static void launch_dslash_nr(int diag, bool postinv, DslashArgs a, hipStream_t st) {
  const int threads = a.threads > 0 ? a.threads : 256;
  if (threads != 64 && threads != 128 && threads != 256) fail(WCMG_EINVAL, "unsupported Dslash block size");
  a.nblocks = (a.g.Vh + threads - 1) / threads;
  dim3 grid(xcd_grid(a.nblocks), (a.nrhs + NR - 1) / NR);
#define WCMG_DS(D, P) hipLaunchKernelGGL((dslash_kernel<S, D, P, NR>), grid, dim3(threads), 0, st, a)
  if (diag == 0 && !postinv) WCMG_DS(0, false);
  else if (diag == 0 && postinv) WCMG_DS(0, true);
  else if (diag == 1 && !postinv) WCMG_DS(1, false);
  else if (diag == 1 && postinv) WCMG_DS(1, true);
  else if (diag == 2 && !postinv) WCMG_DS(2, false);
  else WCMG_DS(2, true);
#undef WCMG_DS
  HIPCHK(hipGetLastError());
}

template <typename S>
static void launch_dslash_t(int diag, bool postinv, const DslashArgs& a, hipStream_t st) {
  int g = a.nrhs >= max_group<S>() ? max_group<S>() : (a.nrhs >= 2 ? 2 : 1);
  if (a.group > 0) g = std::min(a.group, max_group<S>());
  if (g == 1) launch_dslash_nr<S, 1>(diag, postinv, a, st);
  else if (g == 2) launch_dslash_nr<S, 2>(diag, postinv, a, st);
  else launch_dslash_nr<S, max_group<S>()>(diag, postinv, a, st);
}

void launch_dslash(int prec, int diag, bool postinv, const DslashArgs& a, hipStream_t st) {
  if (a.nrhs < 1) fail(WCMG_EINVAL, "nrhs must be >= 1");
  if (prec == WCMG_F64) launch_dslash_t<double>(diag, postinv, a, st);
  else if (prec == WCMG_F32) launch_dslash_t<float>(diag, postinv, a, st);
  else launch_dslash_t<__half>(diag, postinv, a, st);
}

template <typename S, int NR>
static void launch_clover_nr(void* out, const void* in, const void* clov, int Vh, int p, int kind, int nrhs,
                             size_t rstride, hipStream_t st) {
  dim3 grid((Vh + 255) / 256, (nrhs + NR - 1) / NR);
  hipLaunchKernelGGL((clover_kernel<S, NR>), grid, dim3(256), 0, st, out, in, clov, Vh, p, kind, nrhs, rstride);
}

template <typename S>
static void launch_clover_t(void* out, const void* in, const void* clov, int Vh, int p, int kind, int nrhs,
                            size_t rstride, hipStream_t st) {
  if (nrhs >= max_group<S>()) launch_clover_nr<S, max_group<S>()>(out, in, clov, Vh, p, kind, nrhs, rstride, st);
  else if (nrhs >= 2) launch_clover_nr<S, 2>(out, in, clov, Vh, p, kind, nrhs, rstride, st);
  else launch_clover_nr<S, 1>(out, in, clov, Vh, p, kind, nrhs, rstride, st);
}

void launch_clover(int prec, void* out, const void* in, const void* clov, int Vh, int p, int kind, hipStream_t st,
                   int nrhs, size_t rstride) {
  if (nrhs < 1) fail(WCMG_EINVAL, "nrhs must be >= 1");
  if (prec == WCMG_F64) launch_clover_t<double>(out, in, clov, Vh, p, kind, nrhs, rstride, st);
  else if (prec == WCMG_F32) launch_clover_t<float>(out, in, clov, Vh, p, kind, nrhs, rstride, st);
  else launch_clover_t<__half>(out, in, clov, Vh, p, kind, nrhs, rstride, st);
  HIPCHK(hipGetLastError());
}

}  // namespace wcmg
