// Fine Wilson-clover hopping kernels (red-black paragraph, Eqs.(2)-(3)).
//
// One thread computes one output site of parity p:
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

template <typename S, int MU>
__device__ __forceinline__ void hop_mu(const DslashArgs& a, int p, int i, const int c[4],
                                       cpx<typename Compute<S>::T> acc[12]) {
  using C = typename Compute<S>::T;
  const DGeom& g = a.g;
  cpx<C> psi[12], h[6], hu[6], U[9];
  // forward: (1 - gamma_mu) U_mu(x) in(x + mu)
  {
    int n[4] = {c[0], c[1], c[2], c[3]};
    n[MU] = (n[MU] + 1 == g.L[MU]) ? 0 : n[MU] + 1;
    int nb = cb_index(g, n);
    SpinorIO<S>::load(a.in, g.Vh, nb, psi);
    load_link<S, C>(a.gauge, g.Vh, p, MU, i, U);
    project<C, MU, false>(psi, h);
    link_mul<C, false>(U, h, hu);
    if constexpr (MU == 3) {
      if (c[3] == g.L[3] - 1) {
        C ph = (C)g.t_bc;
#pragma unroll
        for (int k = 0; k < 6; ++k) hu[k] = ph * hu[k];
      }
    }
    accumulate<C, MU, false>(acc, hu);
    pin_acc(acc);
  }
  // backward: (1 + gamma_mu) U_mu(x - mu)^dag in(x - mu)
  {
    int n[4] = {c[0], c[1], c[2], c[3]};
    n[MU] = (n[MU] == 0) ? g.L[MU] - 1 : n[MU] - 1;
    int nb = cb_index(g, n);
    SpinorIO<S>::load(a.in, g.Vh, nb, psi);
    load_link<S, C>(a.gauge, g.Vh, 1 - p, MU, nb, U);
    project<C, MU, true>(psi, h);
    link_mul<C, true>(U, h, hu);
    if constexpr (MU == 3) {
      if (c[3] == 0) {
        C ph = (C)g.t_bc;
#pragma unroll
        for (int k = 0; k < 6; ++k) hu[k] = ph * hu[k];
      }
    }
    accumulate<C, MU, true>(acc, hu);
    pin_acc(acc);
  }
}

template <typename S, int DIAG, bool POSTINV>
__global__ void __launch_bounds__(256) dslash_kernel(DslashArgs a) {
  using C = typename Compute<S>::T;
  const int lb = xcd_block(a.nblocks);
  const int i = lb * blockDim.x + threadIdx.x;
  if (lb >= a.nblocks || i >= a.g.Vh) return;
  const int p = a.parity;
  int c[4];
  cb_coords(a.g, i, p, c);

  cpx<C> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mk((C)0, (C)0);
  hop_mu<S, 0>(a, p, i, c, acc);
  hop_mu<S, 1>(a, p, i, c, acc);
  hop_mu<S, 2>(a, p, i, c, acc);
  hop_mu<S, 3>(a, p, i, c, acc);

  const C f = (C)(-0.5 * a.coeff);
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = f * acc[k];

  cpx<C> out[12];
  if constexpr (POSTINV) {
    clover_apply<S, C>(a.clov, a.g.Vh, p, 1, i, acc, out);
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) out[k] = acc[k];
  }
  if constexpr (DIAG != 0) {
    cpx<C> xv[12];
    SpinorIO<S>::load(a.x, a.g.Vh, i, xv);
    if constexpr (DIAG == 2) {
      cpx<C> ax[12];
      clover_apply<S, C>(a.clov, a.g.Vh, p, 0, i, xv, ax);
#pragma unroll
      for (int k = 0; k < 12; ++k) out[k] = out[k] + ax[k];
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) out[k] = out[k] + xv[k];
    }
  }
  SpinorIO<S>::store(a.out, a.g.Vh, i, out);
}

// out_p = A_p^(kind) in_p   (site-local clover or clover inverse)
template <typename S>
__global__ void __launch_bounds__(256) clover_kernel(void* out, const void* in, const void* clov, int Vh, int p,
                                                     int kind) {
  using C = typename Compute<S>::T;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vh) return;
  cpx<C> v[12], o[12];
  SpinorIO<S>::load(in, Vh, i, v);
  clover_apply<S, C>(clov, Vh, p, kind, i, v, o);
  SpinorIO<S>::store(out, Vh, i, o);
}

template <typename S>
static void launch_dslash_t(int diag, bool postinv, DslashArgs a, hipStream_t st) {
  const int threads = 256;
  a.nblocks = (a.g.Vh + threads - 1) / threads;
  dim3 grid(xcd_grid(a.nblocks));
#define WCMG_DS(D, P) hipLaunchKernelGGL((dslash_kernel<S, D, P>), grid, dim3(threads), 0, st, a)
  if (diag == 0 && !postinv) WCMG_DS(0, false);
  else if (diag == 0 && postinv) WCMG_DS(0, true);
  else if (diag == 1 && !postinv) WCMG_DS(1, false);
  else if (diag == 1 && postinv) WCMG_DS(1, true);
  else if (diag == 2 && !postinv) WCMG_DS(2, false);
  else WCMG_DS(2, true);
#undef WCMG_DS
  HIPCHK(hipGetLastError());
}

void launch_dslash(int prec, int diag, bool postinv, const DslashArgs& a, hipStream_t st) {
  if (prec == WCMG_F64) launch_dslash_t<double>(diag, postinv, a, st);
  else if (prec == WCMG_F32) launch_dslash_t<float>(diag, postinv, a, st);
  else launch_dslash_t<__half>(diag, postinv, a, st);
}

void launch_clover(int prec, void* out, const void* in, const void* clov, int Vh, int p, int kind,
                   hipStream_t st) {
  const int threads = 256;
  dim3 grid((Vh + threads - 1) / threads);
  if (prec == WCMG_F64)
    hipLaunchKernelGGL(clover_kernel<double>, grid, dim3(threads), 0, st, out, in, clov, Vh, p, kind);
  else if (prec == WCMG_F32)
    hipLaunchKernelGGL(clover_kernel<float>, grid, dim3(threads), 0, st, out, in, clov, Vh, p, kind);
  else
    hipLaunchKernelGGL(clover_kernel<__half>, grid, dim3(threads), 0, st, out, in, clov, Vh, p, kind);
  HIPCHK(hipGetLastError());
}

}  // namespace wcmg
