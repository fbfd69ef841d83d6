// Random start vectors of the multigrid setup (Setup procedure section).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of
//   (c0,c1,c2,c3) -> (hi(M1*c2)^c1^k0, lo(M1*c2), hi(M0*c0)^c3^k1, lo(M0*c0))
// with the key bumped by (0x9E3779B9, 0xBB67AE85) before each round after
// the first.  Entry n = site*ncomp + component of vector `vec` on level
// `level` uses counter (n mod 2^32, n div 2^32, vec, level) and key
// (seed mod 2^32, seed div 2^32); the first two words give uniforms
// u = (w + 1/2)/2^32 and the complex Gaussian sqrt(-2 ln u0) exp(2 pi i u1).
#include "kernels.h"
#include "random.h"

namespace wcmg {

namespace {

__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t p0 = (uint64_t)M0 * c[0];
    uint64_t p1 = (uint64_t)M1 * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ double2 gauss(uint64_t seed, uint32_t vec, uint32_t level, uint64_t n) {
  uint32_t c[4] = {(uint32_t)n, (uint32_t)(n >> 32), vec, level};
  philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  double u0 = ((double)c[0] + 0.5) * (1.0 / 4294967296.0);
  double u1 = ((double)c[1] + 0.5) * (1.0 / 4294967296.0);
  double r = sqrt(-2.0 * log(u0));
  double s, co;
  sincospi(2.0 * u1, &s, &co);
  return make_double2(r * co, r * s);
}

// fine full-lattice FP64 spinor (both parity halves, internal layout)
__global__ void k_fine_gauss(double2* out, uint64_t seed, uint32_t vec, uint32_t level, DGeom g, int V) {
  int lex = blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= V) return;
  int r = lex;
  int x = r % g.L[0];
  r /= g.L[0];
  int y = r % g.L[1];
  r /= g.L[1];
  int z = r % g.L[2];
  int t = r / g.L[2];
  int p = (x + y + z + t) & 1;
  double2* half = out + (size_t)p * 12 * g.Vh;
  for (int a = 0; a < 12; ++a) half[(size_t)a * g.Vh + (lex >> 1)] = gauss(seed, vec, level, (uint64_t)lex * 12 + a);
}

// coarse FP64 vector [internal site][n]; perm[lex] = internal index
__global__ void k_coarse_gauss(double2* out, uint64_t seed, uint32_t vec, uint32_t level, const int* perm, int V,
                               int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= V * n) return;
  int lex = t / n, a = t - lex * n;
  out[(size_t)perm[lex] * n + a] = gauss(seed, vec, level, (uint64_t)t);
}

}  // namespace

void random_fine_vector(void* out, uint64_t seed, int vec, int level, const Geom& g, hipStream_t st) {
  hipLaunchKernelGGL(k_fine_gauss, dim3((g.V + 255) / 256), dim3(256), 0, st, reinterpret_cast<double2*>(out), seed,
                     (uint32_t)vec, (uint32_t)level, dgeom(g), g.V);
  HIPCHK(hipGetLastError());
}

void random_coarse_vector(void* out, uint64_t seed, int vec, int level, const int* perm, int V, int n,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_coarse_gauss, dim3((V * n + 255) / 256), dim3(256), 0, st, reinterpret_cast<double2*>(out),
                     seed, (uint32_t)vec, (uint32_t)level, perm, V, n);
  HIPCHK(hipGetLastError());
}

}  // namespace wcmg
