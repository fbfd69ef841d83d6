// Lexicographic site geometry and 3x3 complex (SU(3)) matrix helpers in FP64,
// shared by the clover construction and the gauge force.
#pragma once

#include "wcmg_internal.h"

namespace wcmg {

__device__ __forceinline__ int lex_of(const int L[4], const int c[4]) {
  return ((c[3] * L[2] + c[2]) * L[1] + c[1]) * L[0] + c[0];
}
__device__ __forceinline__ void coords_of(const int L[4], int lex, int c[4]) {
  c[0] = lex % L[0];
  lex /= L[0];
  c[1] = lex % L[1];
  lex /= L[1];
  c[2] = lex % L[2];
  c[3] = lex / L[2];
}

struct C3 {
  cpx<double> m[9];
};
__device__ __forceinline__ C3 load_u(const double2* gauge, const DGeom& g, const int c[4], int mu) {
  int lex = lex_of(g.L, c);
  int p = (c[0] + c[1] + c[2] + c[3]) & 1;
  const double2* b = gauge + ((size_t)(p * 4 + mu) * 9) * g.Vh + (lex >> 1);
  C3 u;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double2 t = b[(size_t)k * g.Vh];
    u.m[k] = mk(t.x, t.y);
  }
  return u;
}
__device__ __forceinline__ C3 mul(const C3& a, const C3& b) {
  C3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cpx<double> t = mk(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) cfma(t, a.m[i * 3 + k], b.m[k * 3 + j]);
      r.m[i * 3 + j] = t;
    }
  return r;
}
__device__ __forceinline__ C3 dagm(const C3& a) {
  C3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.m[i * 3 + j] = cconj(a.m[j * 3 + i]);
  return r;
}
__device__ __forceinline__ void shift(const int L[4], const int c[4], int mu, int d, int o[4]) {
  o[0] = c[0];
  o[1] = c[1];
  o[2] = c[2];
  o[3] = c[3];
  o[mu] = (o[mu] + d + L[mu]) % L[mu];
}

}  // namespace wcmg
