// Multi-right-hand-side coarse stencil on the matrix cores.
//
// For a batch of right-hand sides the red-black coarse hop
//   out(c) = DIAG + coeff sum_d Yt_d(c) in(c + d)
// is, per coarse site, a dense product of the n x 8n complex block row with
// the 8n x k block of neighbour vectors (k right-hand sides).  Here it runs on
// v_mfma_f32_16x16x16f16: the matrices are stored once in FP16, already in
// the operand (fragment) order of the instruction, real and imaginary parts
// separately (no duplication); each neighbour block of the FP32 input is
// scaled per right-hand side to its largest entry and converted to FP16,
// multiplied with FP32 accumulation, and scaled back before the sum over the
// eight directions.  Complex arithmetic from real products:
//   Re = A_r B_r + A_i (-B_i),  Im = A_r B_i + A_i B_r.
//
// Operand layouts of the 16x16x16 instruction (lane l of 64):
//   A (M x K): A[l % 16][4 (l / 16) + j],  B (K x N): B[4 (l / 16) + j][l % 16],
//   D (M x N): D[4 (l / 16) + j][l % 16],  j = 0..3.
// One workgroup per coarse site, one wave per 16-row tile of the n rows; the
// 16 columns are 16 right-hand sides (a partial group pads with zeros).
#include "kernels.h"

namespace wcmg {

namespace {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// fragment f = ((((site * 8 + d) * T + mt) * T + ks) * 2 + part), 64 lanes x 4 halves each
__global__ void __launch_bounds__(256) k_mfma_fragments(h4* frag, const double2* Yt, int nsites, int n, int* flag) {
  const int T = n / 16;
  const size_t total = (size_t)nsites * 8 * T * T * 2 * 64;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int lane = (int)(t % 64);
  size_t f = t / 64;
  const int part = (int)(f % 2);
  f /= 2;
  const int ks = (int)(f % T);
  f /= T;
  const int mt = (int)(f % T);
  f /= T;  // f = site * 8 + d
  const double2* M = Yt + f * (size_t)n * n;
  const int row = 16 * mt + lane % 16;
  h4 v;
  for (int j = 0; j < 4; ++j) {
    const int col = 16 * ks + 4 * (lane / 16) + j;
    const double2 e = M[(size_t)col * n + row];  // column-major block
    const double x = part == 0 ? e.x : e.y;
    if (!(fabs(x) < 65000.0)) flag[0] = 1;  // outside the FP16 range: every writer stores 1
    v[j] = (_Float16)x;
  }
  frag[t] = v;
}

template <int T>
__global__ void __launch_bounds__(64 * T) k_coarse_hop_mfma(float2* out, const float2* in, const float2* x,
                                                            const h4* frag, double coeff, int site0, const int* nbr,
                                                            size_t vs, int nrhs) {
  constexpr int n = 16 * T;
  const int c = site0 + blockIdx.x;
  const int mt = threadIdx.x / 64, lane = threadIdx.x & 63;
  const int col = lane & 15, q = lane >> 4;
  const int r = blockIdx.y * 16 + col;  // right-hand side of this lane's column
  const bool live = r < nrhs;
  f4 acc_r = {0.f, 0.f, 0.f, 0.f}, acc_i = {0.f, 0.f, 0.f, 0.f};
  for (int d = 0; d < 8; ++d) {
    const int nb = nbr[(size_t)c * 8 + d];
    float2 v[T][4];
    float m = 0.f;
#pragma unroll
    for (int ks = 0; ks < T; ++ks)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[ks][j] = live ? in[(size_t)r * vs + (size_t)nb * n + 16 * ks + 4 * q + j] : make_float2(0.f, 0.f);
        m = fmaxf(m, fmaxf(fabsf(v[ks][j].x), fabsf(v[ks][j].y)));
      }
    // the four lanes q = 0..3 of a column hold its n entries
    m = fmaxf(m, __shfl_xor(m, 16));
    m = fmaxf(m, __shfl_xor(m, 32));
    const float s = m > 0.f ? m : 1.f, inv = 1.f / s;
    f4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
    const h4* fb = frag + ((size_t)(c * 8 + d) * T + mt) * T * 2 * 64 + lane;
#pragma unroll
    for (int ks = 0; ks < T; ++ks) {
      h4 br, bi, bn;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        br[j] = (_Float16)(v[ks][j].x * inv);
        bi[j] = (_Float16)(v[ks][j].y * inv);
        bn[j] = -bi[j];
      }
      const h4 ar = fb[(size_t)(ks * 2 + 0) * 64];
      const h4 ai = fb[(size_t)(ks * 2 + 1) * 64];
      cr = __builtin_amdgcn_mfma_f32_16x16x16f16(ar, br, cr, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f32_16x16x16f16(ai, bn, cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_16x16x16f16(ar, bi, ci, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_16x16x16f16(ai, br, ci, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc_r[j] += s * cr[j];
      acc_i[j] += s * ci[j];
    }
  }
  if (!live) return;
  const float cf = (float)coeff;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const size_t o = (size_t)r * vs + (size_t)c * n + 16 * mt + 4 * q + j;
    float2 y = make_float2(cf * acc_r[j], cf * acc_i[j]);
    if (x) {
      const float2 xv = x[o];
      y.x += xv.x;
      y.y += xv.y;
    }
    out[o] = y;
  }
}

}  // namespace

bool mfma_coarse_supported(int n) { return n == 16 || n == 32 || n == 48 || n == 64; }

size_t mfma_fragment_bytes(int nsites, int n) { return (size_t)nsites * 8 * n * n * 4; }

void build_mfma_fragments(void* frag, const void* Yt64, int nsites, int n, int* flag, hipStream_t st) {
  if (!mfma_coarse_supported(n)) fail(WCMG_EDIM, "coarse block size not supported by the matrix-core stencil");
  const int T = n / 16;
  const size_t total = (size_t)nsites * 8 * T * T * 2 * 64;
  hipLaunchKernelGGL(k_mfma_fragments, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     reinterpret_cast<h4*>(frag), reinterpret_cast<const double2*>(Yt64), nsites, n, flag);
  HIPCHK(hipGetLastError());
}

void launch_coarse_hop_mfma(void* out, const void* in, const void* x, const void* frag, double coeff, int parity,
                            const CoarseGeom& cg, const int* nbr, int nrhs, size_t vs, hipStream_t st) {
  const int n = cg.n;
  if (!mfma_coarse_supported(n)) fail(WCMG_EDIM, "coarse block size not supported by the matrix-core stencil");
  int site0 = 0, nsites = cg.V;
  if (parity >= 0) {
    site0 = parity * cg.Vh;
    nsites = cg.Vh;
  }
  if (nsites == 0 || nrhs < 1) return;
  dim3 grid(nsites, (nrhs + 15) / 16);
  auto o = reinterpret_cast<float2*>(out);
  auto i = reinterpret_cast<const float2*>(in);
  auto xx = reinterpret_cast<const float2*>(x);
  auto f = reinterpret_cast<const h4*>(frag);
  switch (n / 16) {
    case 1: hipLaunchKernelGGL(k_coarse_hop_mfma<1>, grid, dim3(64), 0, st, o, i, xx, f, coeff, site0, nbr, vs, nrhs); break;
    case 2: hipLaunchKernelGGL(k_coarse_hop_mfma<2>, grid, dim3(128), 0, st, o, i, xx, f, coeff, site0, nbr, vs, nrhs); break;
    case 3: hipLaunchKernelGGL(k_coarse_hop_mfma<3>, grid, dim3(192), 0, st, o, i, xx, f, coeff, site0, nbr, vs, nrhs); break;
    default: hipLaunchKernelGGL(k_coarse_hop_mfma<4>, grid, dim3(256), 0, st, o, i, xx, f, coeff, site0, nbr, vs, nrhs); break;
  }
  HIPCHK(hipGetLastError());
}

}  // namespace wcmg
