// Gauge-link gradient ("force") of a real loss through x = D(U)^-1 eta.
//
// With lambda = D^-dag g for the upstream gradient g of x, the loss changes by
// dL = -Re <lambda, dD x>.  Gradients follow PyTorch's convention for complex
// variables (dL = Re sum conj(G) dU).  Derivation from Eq.(1):
//
//  hop:    G_mu(y) = 1/2 ph sum_s [ lambda(y)_s chi_s^dag + phi_s lambda(y+mu)_s^dag ]
//          chi = (1 - gamma_mu) x(y+mu), phi = (1 + gamma_mu) x(y), ph the time
//          boundary phase of the link;
//  clover: with S_s(mu,nu) = csw (i/2) sigma_mu_nu on chirality s (mu < nu),
//          Xi(y)[i][j] = sum_s sum_{a,b} S_s[a][b] x(y)_{s,b,i} conj(lambda(y)_{s,a,j}),
//          Z = (Xi^dag - Xi)/8, the loss changes by Re sum_y tr(dQ_mu_nu(y) Z(y))
//          with Q the sum of the four plaquette leaves.  Every leaf of Q at y
//          is one elementary square of the plane read from its corner y, so
//          sum_y tr(Q(y) Z(y)) = sum_squares sum_corners tr(loop from corner c
//          times Z(c)).  For the square L1 L2 L3 L4 = U_a(z) U_b(z+a)
//          U_a(z+b)^dag U_b(z)^dag with corners c1..c4 = z, z+a, z+a+b, z+b,
//          the derivative with respect to factor k is
//          K_k = Z1 A B C + A Z2 B C + A B Z3 C + A B C Z0,
//          (A, B, C) = (L_k+1, L_k+2, L_k+3), Z1..Z3 at the corners before
//          them and Z0 at corner k; a plain link collects K^dag, an adjoint
//          link collects K.
//
// All arithmetic is FP64; fields use the canonical lexicographic layout.
#include "kernels.h"
#include "hop_core.h"
#include "su3.h"

namespace wcmg {

namespace {
constexpr int kT = 128;

__device__ __forceinline__ void load12(const double2* v, size_t site, cpx<double> o[12]) {
  const double2* p = v + site * 12;
#pragma unroll
  for (int k = 0; k < 12; ++k) o[k] = mk(p[k].x, p[k].y);
}

// out = (1 - gamma_mu) v (BACK = false) or (1 + gamma_mu) v (BACK = true)
template <int MU, bool BACK>
__device__ __forceinline__ void one_pm_gamma(const cpx<double> v[12], cpx<double> out[12]) {
  cpx<double> h[6];
  project<double, MU, BACK>(v, h);
#pragma unroll
  for (int k = 0; k < 12; ++k) out[k] = mk(0.0, 0.0);
  accumulate<double, MU, BACK>(out, h);
}

template <int MU>
__device__ __forceinline__ void hop_force_mu(const double2* x, const double2* lam, int nrhs, size_t V,
                                             size_t y, size_t yp, double ph, double2* G) {
  cpx<double> acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = mk(0.0, 0.0);
  for (int r = 0; r < nrhs; ++r) {
    const size_t off = (size_t)r * V;
    cpx<double> v[12], w[12], l[12];
    // lambda(y)_s chi_s^dag,  chi = (1 - gamma) x(y+mu)
    load12(x, off + yp, v);
    one_pm_gamma<MU, false>(v, w);
    load12(lam, off + y, l);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) cfmac(acc[a * 3 + b], w[s * 3 + b], l[s * 3 + a]);
    // phi_s lambda(y+mu)_s^dag,  phi = (1 + gamma) x(y)
    load12(x, off + y, v);
    one_pm_gamma<MU, true>(v, w);
    load12(lam, off + yp, l);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) cfmac(acc[a * 3 + b], l[s * 3 + b], w[s * 3 + a]);
  }
  double2* o = G + (y * 4 + MU) * 9;
#pragma unroll
  for (int k = 0; k < 9; ++k) o[k] = make_double2(0.5 * ph * acc[k].r, 0.5 * ph * acc[k].i);
}

__global__ void __launch_bounds__(kT) k_hop_force(double2* G, const double2* x, const double2* lam, int nrhs,
                                                  DGeom g, int V) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= V) return;
  int c[4], n[4];
  coords_of(g.L, y, c);
  const double pht = (c[3] == g.L[3] - 1) ? g.t_bc : 1.0;
  // spatial hops carry the coefficient g.hs (1 on isotropic lattices)
  shift(g.L, c, 0, 1, n);
  hop_force_mu<0>(x, lam, nrhs, V, y, lex_of(g.L, n), g.hs, G);
  shift(g.L, c, 1, 1, n);
  hop_force_mu<1>(x, lam, nrhs, V, y, lex_of(g.L, n), g.hs, G);
  shift(g.L, c, 2, 1, n);
  hop_force_mu<2>(x, lam, nrhs, V, y, lex_of(g.L, n), g.hs, G);
  shift(g.L, c, 3, 1, n);
  hop_force_mu<3>(x, lam, nrhs, V, y, lex_of(g.L, n), pht, G);
}

// Z[plane][9][V] = (Xi^dag - Xi) / 8 per site and plane mu < nu
__global__ void __launch_bounds__(kT) k_clover_insertion(double2* Z, const double2* x, const double2* lam,
                                                         int nrhs, CloverCoef cc, int V) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= V) return;
  for (int pl = 0; pl < 6; ++pl) {
    cpx<double> xi[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) xi[k] = mk(0.0, 0.0);
    for (int r = 0; r < nrhs; ++r) {
      cpx<double> v[12], l[12];
      load12(x, (size_t)r * V + y, v);
      load12(lam, (size_t)r * V + y, l);
#pragma unroll
      for (int chi = 0; chi < 2; ++chi)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const cpx<double> s = mk(cc.s[pl][chi][a * 2 + b][0], cc.s[pl][chi][a * 2 + b][1]);
            const int sa = 2 * chi + a, sb = 2 * chi + b;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int j = 0; j < 3; ++j) {
                // s * x_{sb,i} * conj(lambda_{sa,j})
                cpx<double> t = mk(0.0, 0.0);
                cfmac(t, l[sa * 3 + j], v[sb * 3 + i]);
                cfma(xi[i * 3 + j], s, t);
              }
          }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        cpx<double> z = 0.125 * (cconj(xi[j * 3 + i]) - xi[i * 3 + j]);
        Z[((size_t)pl * 9 + i * 3 + j) * V + y] = make_double2(z.r, z.i);
      }
  }
}

__device__ __forceinline__ int plane_index(int a, int b) {  // a < b
  return a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
}

__device__ __forceinline__ C3 load_z(const double2* Z, int pl, int V, const int L[4], const int c[4]) {
  const int y = lex_of(L, c);
  C3 m;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double2 t = Z[((size_t)pl * 9 + k) * V + y];
    m.m[k] = mk(t.x, t.y);
  }
  return m;
}

__device__ __forceinline__ C3 madd(const C3& a, const C3& b) {
  C3 r;
#pragma unroll
  for (int k = 0; k < 9; ++k) r.m[k] = a.m[k] + b.m[k];
  return r;
}

// derivative matrix K_k of square z in plane (a, b) with respect to its factor k (1..4)
__device__ C3 square_derivative(const double2* gauge, const double2* Z, const DGeom& g, int V, int a, int b,
                                const int z[4], int k) {
  const int pl = plane_index(a, b);
  int c[4][4];  // corners c1..c4 -> c[0..3]
#pragma unroll
  for (int d = 0; d < 4; ++d) c[0][d] = z[d];
  shift(g.L, z, a, 1, c[1]);
  shift(g.L, c[1], b, 1, c[2]);
  shift(g.L, z, b, 1, c[3]);
  // factor j (0-based) starts at corner j: L1 = U_a(c1), L2 = U_b(c2), L3 = U_a(c4)^dag, L4 = U_b(c1)^dag
  auto factor = [&](int j) -> C3 {
    switch (j) {
      case 0: return load_u(gauge, g, c[0], a);
      case 1: return load_u(gauge, g, c[1], b);
      case 2: return dagm(load_u(gauge, g, c[3], a));
      default: return dagm(load_u(gauge, g, c[0], b));
    }
  };
  const int k0 = k - 1;
  const int j1 = (k0 + 1) & 3, j2 = (k0 + 2) & 3, j3 = (k0 + 3) & 3;
  const C3 A = factor(j1), B = factor(j2), C = factor(j3);
  const C3 Z1 = load_z(Z, pl, V, g.L, c[j1]);
  const C3 Z2 = load_z(Z, pl, V, g.L, c[j2]);
  const C3 Z3 = load_z(Z, pl, V, g.L, c[j3]);
  const C3 Z0 = load_z(Z, pl, V, g.L, c[k0]);
  const C3 AB = mul(A, B);
  const C3 T1 = madd(mul(Z1, A), mul(A, Z2));
  const C3 T2 = madd(mul(T1, B), mul(AB, Z3));
  const C3 ABC = mul(AB, C);
  return madd(mul(T2, C), mul(ABC, Z0));
}

// G[(y*4+mu)*9 ..] += clover part, one thread per link
__global__ void __launch_bounds__(kT) k_clover_force(double2* G, const double2* Z, const double2* gauge, DGeom g,
                                                     int V) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * V) return;
  const int y = t >> 2, mu = t & 3;
  int x[4];
  coords_of(g.L, y, x);
  C3 acc;
#pragma unroll
  for (int k = 0; k < 9; ++k) acc.m[k] = mk(0.0, 0.0);
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    int z[4];
    if (mu < nu) {
      // U_mu(x) is factor 1 of square z = x and factor 3 (adjoint) of square z = x - nu
      acc = madd(acc, dagm(square_derivative(gauge, Z, g, V, mu, nu, x, 1)));
      shift(g.L, x, nu, -1, z);
      acc = madd(acc, square_derivative(gauge, Z, g, V, mu, nu, z, 3));
    } else {
      // U_mu(x) is factor 2 of square z = x - nu and factor 4 (adjoint) of square z = x
      shift(g.L, x, nu, -1, z);
      acc = madd(acc, dagm(square_derivative(gauge, Z, g, V, nu, mu, z, 2)));
      acc = madd(acc, square_derivative(gauge, Z, g, V, nu, mu, x, 4));
    }
  }
  double2* o = G + (size_t)t * 9;
#pragma unroll
  for (int k = 0; k < 9; ++k) o[k] = make_double2(o[k].x + acc.m[k].r, o[k].y + acc.m[k].i);
}
}  // namespace

void force_compute(void* G, const void* x, const void* lam, int nrhs, const void* gauge64, const Geom& g,
                   const CloverCoef* cc, void* zbuf, hipStream_t st) {
  const DGeom d = dgeom(g);
  const int V = g.V;
  hipLaunchKernelGGL(k_hop_force, dim3((V + kT - 1) / kT), dim3(kT), 0, st, reinterpret_cast<double2*>(G),
                     reinterpret_cast<const double2*>(x), reinterpret_cast<const double2*>(lam), nrhs, d, V);
  HIPCHK(hipGetLastError());
  if (!cc) return;
  hipLaunchKernelGGL(k_clover_insertion, dim3((V + kT - 1) / kT), dim3(kT), 0, st,
                     reinterpret_cast<double2*>(zbuf), reinterpret_cast<const double2*>(x),
                     reinterpret_cast<const double2*>(lam), nrhs, *cc, V);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_clover_force, dim3((4 * V + kT - 1) / kT), dim3(kT), 0, st, reinterpret_cast<double2*>(G),
                     reinterpret_cast<const double2*>(zbuf), reinterpret_cast<const double2*>(gauge64), d, V);
  HIPCHK(hipGetLastError());
}

}  // namespace wcmg
