// Spin projection, link multiplication and reconstruction of one hop
// direction of the Wilson term (chiral basis), shared by the Dslash and the
// coarse-operator construction.
//   (1 - gamma) psi = [h ; -B^dag h],  h = psi_up - B psi_down
//   (1 + gamma) psi = [h ;  B^dag h],  h = psi_up + B psi_down
// with gamma_mu = [[0, B],[B^dag, 0]], B_x = -i sigma_1, B_y = -i sigma_2,
// B_z = -i sigma_3, B_t = 1.
#pragma once

#include "wcmg_internal.h"

namespace wcmg {

template <typename C, int MU, bool BACK>
__device__ __forceinline__ void project(const cpx<C> psi[12], cpx<C> h[6]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cpx<C> d0 = psi[6 + a], d1 = psi[9 + a];
    cpx<C> b0, b1;  // B psi_down
    if constexpr (MU == 0) {
      b0 = cmi(d1);
      b1 = cmi(d0);
    } else if constexpr (MU == 1) {
      b0 = mk(-d1.r, -d1.i);
      b1 = d0;
    } else if constexpr (MU == 2) {
      b0 = cmi(d0);
      b1 = ci(d1);
    } else {
      b0 = d0;
      b1 = d1;
    }
    if constexpr (!BACK) {
      h[a] = psi[a] - b0;
      h[3 + a] = psi[3 + a] - b1;
    } else {
      h[a] = psi[a] + b0;
      h[3 + a] = psi[3 + a] + b1;
    }
  }
}

template <typename C, int MU, bool BACK>
__device__ __forceinline__ void accumulate(cpx<C> acc[12], const cpx<C> h[6]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cpx<C> h0 = h[a], h1 = h[3 + a];
    cpx<C> g0, g1;  // B^dag h
    if constexpr (MU == 0) {
      g0 = ci(h1);
      g1 = ci(h0);
    } else if constexpr (MU == 1) {
      g0 = h1;
      g1 = mk(-h0.r, -h0.i);
    } else if constexpr (MU == 2) {
      g0 = ci(h0);
      g1 = cmi(h1);
    } else {
      g0 = h0;
      g1 = h1;
    }
    acc[a] = acc[a] + h0;
    acc[3 + a] = acc[3 + a] + h1;
    if constexpr (!BACK) {
      acc[6 + a] = acc[6 + a] - g0;
      acc[9 + a] = acc[9 + a] - g1;
    } else {
      acc[6 + a] = acc[6 + a] + g0;
      acc[9 + a] = acc[9 + a] + g1;
    }
  }
}

// hu[s][a] = sum_b U[a][b] h[s][b]   (forward)
// hu[s][a] = sum_b conj(U[b][a]) h[s][b]   (backward)
template <typename C, bool DAG>
__device__ __forceinline__ void link_mul(const cpx<C> U[9], const cpx<C> h[6], cpx<C> hu[6]) {
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<C> t = mk((C)0, (C)0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if constexpr (!DAG)
          cfma(t, U[a * 3 + b], h[s * 3 + b]);
        else
          cfmac(t, U[b * 3 + a], h[s * 3 + b]);
      }
      hu[s * 3 + a] = t;
    }
  }
}

}  // namespace wcmg
