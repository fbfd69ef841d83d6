// Transfer between the fine lattice and the first coarse level
// (red-black paragraph): P from the null vectors split into space-time
// blocks x 2 chiralities, R = P^dag gamma5, and the pieces of the coarse
// operator construction Yhat = R D_p P.
//
//   R:  c(b, s, k) = (+1 | -1)_s  sum_{x in b, chirality(a) = s} conj(V_k(x,a)) r(x,a)
//   P:  e(x, a)    = sum_k V_k(x, a) c(block(x), chirality(a), k)
//
// V_k are the block-orthonormalised vectors (full-lattice spinors in the
// internal layout).  R launches one workgroup per (coarse site, vector),
// P one thread per fine site.
#include "kernels.h"
#include "hop_core.h"

namespace wcmg {

namespace {

__device__ __forceinline__ int coarse_internal(const BlockGeom& bg, int clex) {
  if (!bg.coarse_cb) return clex;
  int c0 = clex % bg.nb[0];
  int r = clex / bg.nb[0];
  int c1 = r % bg.nb[1];
  r /= bg.nb[1];
  int c2 = r % bg.nb[2];
  int c3 = r / bg.nb[2];
  int cp = (c0 + c1 + c2 + c3) & 1;
  return cp * (bg.Vc / 2) + (clex >> 1);
}

template <int NR>
__device__ __forceinline__ void block_sum(double (&v)[NR]) {
  // every thread gets the block-wide totals; blockDim.x a multiple of 64, <= 1024
  __shared__ double sh[NR][16];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NR; ++k) sh[k][wave] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[k][w];
    v[k] = s;
  }
}

// KB vectors per workgroup: the input spinor of each site is loaded once and
// dotted with the KB vectors (the sum over the block's sites in a fixed tree)
constexpr int kRestrictKB = 4;

// site of parity p visited at step l of block clex (the order of the
// restriction's loop over a block's half)
__device__ __forceinline__ int block_site(const DGeom& g, const BlockGeom& bg, int clex, int p, int l) {
  int r = clex, cc[4];
  cc[0] = r % bg.nb[0];
  r /= bg.nb[0];
  cc[1] = r % bg.nb[1];
  r /= bg.nb[1];
  cc[2] = r % bg.nb[2];
  cc[3] = r / bg.nb[2];
  const int bxh = bg.b[0] / 2;
  int lxh = l % bxh;
  r = l / bxh;
  int c[4];
  c[1] = cc[1] * bg.b[1] + r % bg.b[1];
  r /= bg.b[1];
  c[2] = cc[2] * bg.b[2] + r % bg.b[2];
  c[3] = cc[3] * bg.b[3] + r / bg.b[2];
  c[0] = cc[0] * bg.b[0] + 2 * lxh + ((p + c[1] + c[2] + c[3]) & 1);
  return cb_index(g, c);
}

// FP32 null vectors reordered block by block: float4 chunk c of the l-th
// site of parity p of block b of vector k at (((k 2 + p) Vc + b) 6 + c) half + l,
// so that a restriction workgroup reads each vector's block contiguously
__global__ void k_vec_blockmajor(const float4* __restrict__ v32, float4* __restrict__ out, int nvec, DGeom g,
                                 BlockGeom bg) {
  const int half = bg.bvol / 2;
  const size_t total = (size_t)nvec * 2 * bg.Vc * half;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int l = (int)(t % half);
    size_t r = t / half;
    const int b = (int)(r % bg.Vc);
    r /= bg.Vc;
    const int p = (int)(r % 2);
    const int k = (int)(r / 2);
    const int i = block_site(g, bg, b, p, l);
    const float4* src = v32 + (size_t)(2 * k + p) * 6 * g.Vh;
    float4* dst = out + ((size_t)(2 * k + p) * bg.Vc + b) * 6 * half;
#pragma unroll
    for (int c = 0; c < 6; ++c) dst[(size_t)c * half + l] = src[(size_t)c * g.Vh + i];
  }
}

// FP16 copy of FP32 vector chunks: float4 (two complex) -> uint2 (four halves)
__global__ void k_chunks_to_half(uint2* __restrict__ out, const float4* __restrict__ in, size_t n) {
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    const float4 v = in[t];
    const __half2 a = __floats2half2_rn(v.x, v.y), b = __floats2half2_rn(v.z, v.w);
    out[t] = make_uint2(*reinterpret_cast<const unsigned*>(&a), *reinterpret_cast<const unsigned*>(&b));
  }
}
__device__ __forceinline__ void unpack_half_chunk(uint2 t, cpx<float>& e0, cpx<float>& e1) {
  const float2 a = __half22float2(*reinterpret_cast<const __half2*>(&t.x));
  const float2 b = __half22float2(*reinterpret_cast<const __half2*>(&t.y));
  e0 = mk(a.x, a.y);
  e1 = mk(b.x, b.y);
}

// vbm (FP32 only): the block-major copy of the vectors, read in place of vecs;
// vbm16 (FP32 only): its FP16 copy, read in place of both
template <typename S>
__global__ void __launch_bounds__(128) k_restrict(void* out, size_t site_stride, size_t row_stride, const void* in,
                                                  const void* vecs, size_t vec_bytes, size_t half_bytes, int nvec,
                                                  int p, DGeom g, BlockGeom bg, int accumulate,
                                                  const float4* __restrict__ vbm = nullptr,
                                                  const uint2* __restrict__ vbm16 = nullptr) {
  using C = typename Compute<S>::T;
  using V2 = typename Vec2<C>::T;
  const int clex = blockIdx.x, k0 = blockIdx.y * kRestrictKB;
  const int kb = min(kRestrictKB, nvec - k0);
  int cc[4];
  {
    int r = clex;
    cc[0] = r % bg.nb[0];
    r /= bg.nb[0];
    cc[1] = r % bg.nb[1];
    r /= bg.nb[1];
    cc[2] = r % bg.nb[2];
    cc[3] = r / bg.nb[2];
  }
  double acc[4 * kRestrictKB];
#pragma unroll
  for (int j = 0; j < 4 * kRestrictKB; ++j) acc[j] = 0.0;
  const int half = bg.bvol / 2, bxh = bg.b[0] / 2;
  for (int l = threadIdx.x; l < half; l += blockDim.x) {
    int lxh = l % bxh, r = l / bxh;
    int ly = r % bg.b[1];
    r /= bg.b[1];
    int lz = r % bg.b[2];
    int lt = r / bg.b[2];
    int c[4];
    c[1] = cc[1] * bg.b[1] + ly;
    c[2] = cc[2] * bg.b[2] + lz;
    c[3] = cc[3] * bg.b[3] + lt;
    c[0] = cc[0] * bg.b[0] + 2 * lxh + ((p + c[1] + c[2] + c[3]) & 1);
    int i = cb_index(g, c);
    cpx<C> w[12];
    SpinorIO<S>::load(in, g.Vh, i, w);
#pragma unroll
    for (int kk = 0; kk < kRestrictKB; ++kk) {
      if (kk < kb) {
        cpx<C> v[12];
        if constexpr (sizeof(S) == 4) {
          if (vbm16) {
            const uint2* vb = vbm16 + ((size_t)(2 * (k0 + kk) + p) * bg.Vc + clex) * 6 * half;
#pragma unroll
            for (int cch = 0; cch < 6; ++cch) {
              cpx<float> e0, e1;
              unpack_half_chunk(vb[(size_t)cch * half + l], e0, e1);
              v[2 * cch] = mk((C)e0.r, (C)e0.i);
              v[2 * cch + 1] = mk((C)e1.r, (C)e1.i);
            }
          } else if (vbm) {
            const float4* vb = vbm + ((size_t)(2 * (k0 + kk) + p) * bg.Vc + clex) * 6 * half;
#pragma unroll
            for (int cch = 0; cch < 6; ++cch) {
              const float4 t = vb[(size_t)cch * half + l];
              v[2 * cch] = mk((C)t.x, (C)t.y);
              v[2 * cch + 1] = mk((C)t.z, (C)t.w);
            }
          } else {
            SpinorIO<S>::load(reinterpret_cast<const char*>(vecs) + (size_t)(k0 + kk) * vec_bytes +
                                  (size_t)p * half_bytes,
                              g.Vh, i, v);
          }
        } else {
          SpinorIO<S>::load(reinterpret_cast<const char*>(vecs) + (size_t)(k0 + kk) * vec_bytes + (size_t)p * half_bytes,
                            g.Vh, i, v);
        }
#pragma unroll
        for (int a = 0; a < 12; ++a) {
          const int s = a >= 6;
          acc[4 * kk + 2 * s] += (double)v[a].r * (double)w[a].r + (double)v[a].i * (double)w[a].i;
          acc[4 * kk + 2 * s + 1] += (double)v[a].r * (double)w[a].i - (double)v[a].i * (double)w[a].r;
        }
      }
    }
  }
  block_sum<4 * kRestrictKB>(acc);
  if ((int)threadIdx.x < kb) {
    const int kk = threadIdx.x, k = k0 + kk;
    V2* o = reinterpret_cast<V2*>(out) + (size_t)coarse_internal(bg, clex) * site_stride;
    V2* o0 = o + (size_t)k * row_stride;
    V2* o1 = o + (size_t)(nvec + k) * row_stride;
    double r0 = acc[4 * kk], i0 = acc[4 * kk + 1], r1 = -acc[4 * kk + 2], i1 = -acc[4 * kk + 3];
    if (accumulate) {
      r0 += (double)o0->x;
      i0 += (double)o0->y;
      r1 += (double)o1->x;
      i1 += (double)o1->y;
    }
    o0->x = (C)r0;
    o0->y = (C)i0;
    o1->x = (C)r1;
    o1->y = (C)i1;
  }
}

// v16 (FP32 only): FP16 copy of the vectors' chunks, read in place of vecs
template <typename S>
__global__ void __launch_bounds__(256) k_prolong(void* out, const void* coarse, const void* vecs, size_t vec_bytes,
                                                 size_t half_bytes, int nvec, int p, DGeom g, BlockGeom bg,
                                                 const uint2* __restrict__ v16 = nullptr) {
  using C = typename Compute<S>::T;
  using V2 = typename Vec2<C>::T;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.Vh) return;
  int c[4];
  cb_coords(g, i, p, c);
  int clex = (((c[3] / bg.b[3]) * bg.nb[2] + c[2] / bg.b[2]) * bg.nb[1] + c[1] / bg.b[1]) * bg.nb[0] + c[0] / bg.b[0];
  const V2* cv = reinterpret_cast<const V2*>(coarse) + (size_t)coarse_internal(bg, clex) * (2 * nvec);
  cpx<C> o[12];
#pragma unroll
  for (int a = 0; a < 12; ++a) o[a] = mk((C)0, (C)0);
  for (int k = 0; k < nvec; ++k) {
    cpx<C> v[12];
    if constexpr (sizeof(S) == 4) {
      if (v16) {
        const uint2* vk = v16 + (size_t)(2 * k + p) * 6 * g.Vh;
#pragma unroll
        for (int cch = 0; cch < 6; ++cch) {
          cpx<float> e0, e1;
          unpack_half_chunk(vk[(size_t)cch * g.Vh + i], e0, e1);
          v[2 * cch] = mk((C)e0.r, (C)e0.i);
          v[2 * cch + 1] = mk((C)e1.r, (C)e1.i);
        }
      } else {
        SpinorIO<S>::load(reinterpret_cast<const char*>(vecs) + (size_t)k * vec_bytes + (size_t)p * half_bytes, g.Vh,
                          i, v);
      }
    } else {
      SpinorIO<S>::load(reinterpret_cast<const char*>(vecs) + (size_t)k * vec_bytes + (size_t)p * half_bytes, g.Vh, i,
                        v);
    }
    V2 a0 = cv[k], a1 = cv[nvec + k];
    cpx<C> c0 = mk((C)a0.x, (C)a0.y), c1 = mk((C)a1.x, (C)a1.y);
#pragma unroll
    for (int a = 0; a < 6; ++a) cfma(o[a], v[a], c0);
#pragma unroll
    for (int a = 6; a < 12; ++a) cfma(o[a], v[a], c1);
  }
  SpinorIO<S>::store(out, g.Vh, i, o);
}

// Gram-Schmidt (classical, twice) per (block, chirality) on FP64 vectors.
constexpr int kOrthoSites = 4;  // max block sites per thread (block volume <= 1024)

__global__ void __launch_bounds__(256) k_block_ortho(double2* vecs, size_t vec_elems, int nvec, DGeom g,
                                                     BlockGeom bg, int* flag) {
  const int clex = blockIdx.x, s = blockIdx.y;
  int cc[4];
  {
    int r = clex;
    cc[0] = r % bg.nb[0];
    r /= bg.nb[0];
    cc[1] = r % bg.nb[1];
    r /= bg.nb[1];
    cc[2] = r % bg.nb[2];
    cc[3] = r / bg.nb[2];
  }
  // element offsets (component 6s) of the sites this thread owns
  size_t off[kOrthoSites];
  int nown = 0;
  for (int l = threadIdx.x; l < bg.bvol && nown < kOrthoSites; l += blockDim.x) {
    int lx = l % bg.b[0], r = l / bg.b[0];
    int ly = r % bg.b[1];
    r /= bg.b[1];
    int lz = r % bg.b[2];
    int lt = r / bg.b[2];
    int c[4] = {cc[0] * bg.b[0] + lx, cc[1] * bg.b[1] + ly, cc[2] * bg.b[2] + lz, cc[3] * bg.b[3] + lt};
    int p = (c[0] + c[1] + c[2] + c[3]) & 1;
    off[nown++] = (size_t)p * 12 * g.Vh + (size_t)(6 * s) * g.Vh + cb_index(g, c);
  }
  for (int k = 0; k < nvec; ++k) {
    double2* vk = vecs + (size_t)k * vec_elems;
    cpx<double> v[kOrthoSites][6];
    double n0[1] = {0.0};
    for (int o = 0; o < kOrthoSites; ++o)
      for (int a = 0; a < 6; ++a) {
        if (o < nown) {
          double2 t = vk[off[o] + (size_t)a * g.Vh];
          v[o][a] = mk(t.x, t.y);
          n0[0] += t.x * t.x + t.y * t.y;
        } else {
          v[o][a] = mk(0.0, 0.0);
        }
      }
    block_sum<1>(n0);
    for (int pass = 0; pass < 2; ++pass) {
      for (int j0 = 0; j0 < k; j0 += 8) {
        const int jn = min(8, k - j0);
        double cf[16];
        for (int j = 0; j < 16; ++j) cf[j] = 0.0;
        for (int j = 0; j < jn; ++j) {
          const double2* qj = vecs + (size_t)(j0 + j) * vec_elems;
          for (int o = 0; o < nown; ++o)
            for (int a = 0; a < 6; ++a) {
              double2 t = qj[off[o] + (size_t)a * g.Vh];
              cf[2 * j] += t.x * v[o][a].r + t.y * v[o][a].i;
              cf[2 * j + 1] += t.x * v[o][a].i - t.y * v[o][a].r;
            }
        }
        block_sum<16>(cf);
        for (int j = 0; j < jn; ++j) {
          const double2* qj = vecs + (size_t)(j0 + j) * vec_elems;
          cpx<double> c = mk(cf[2 * j], cf[2 * j + 1]);
          for (int o = 0; o < nown; ++o)
            for (int a = 0; a < 6; ++a) {
              double2 t = qj[off[o] + (size_t)a * g.Vh];
              v[o][a] = v[o][a] - c * mk(t.x, t.y);
            }
        }
      }
    }
    double nk[1] = {0.0};
    for (int o = 0; o < nown; ++o)
      for (int a = 0; a < 6; ++a) nk[0] += v[o][a].r * v[o][a].r + v[o][a].i * v[o][a].i;
    block_sum<1>(nk);
    double nrm = sqrt(nk[0]);
    if (!(nrm > 1e-12 * sqrt(n0[0])) && threadIdx.x == 0) *flag = 1;
    double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int o = 0; o < nown; ++o)
      for (int a = 0; a < 6; ++a) vk[off[o] + (size_t)a * g.Vh] = make_double2(inv * v[o][a].r, inv * v[o][a].i);
    __syncthreads();
  }
}

// Nine buckets of D_p = A A^-1 + H A^-1 acting on (v, u = A^-1 v), split by the
// block the hop comes from: bucket 0 collects v and every hop that stays in
// the block, bucket 1+d the hop from direction d when it crosses the block face.
struct SplitArgs {
  double2* bucket[9];
  const void* v;
  const void* u;
  const void* gauge;
  DGeom g;
  BlockGeom bg;
};

template <int MU>
__device__ __forceinline__ void split_mu(const SplitArgs& a, int p, int i, const int c[4], cpx<double> acc0[12]) {
  const DGeom& g = a.g;
  const size_t hb = (size_t)12 * g.Vh * 16;  // bytes of one FP64 parity half
  const void* u_op = reinterpret_cast<const char*>(a.u) + (size_t)(1 - p) * hb;
  const bool coarse_extent = a.bg.nb[MU] > 1;
#pragma unroll
  for (int back = 0; back < 2; ++back) {
    int n[4] = {c[0], c[1], c[2], c[3]};
    int nb;
    cpx<double> psi[12], h[6], hu[6], U[9], hd[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) hd[k] = mk(0.0, 0.0);
    bool cross;
    if (!back) {
      n[MU] = (n[MU] + 1 == g.L[MU]) ? 0 : n[MU] + 1;
      nb = cb_index(g, n);
      SpinorIO<double>::load(u_op, g.Vh, nb, psi);
      load_link<double, double>(a.gauge, g.Vh, p, MU, i, U);
      project<double, MU, false>(psi, h);
      link_mul<double, false>(U, h, hu);
      if (MU == 3 && c[3] == g.L[3] - 1)
        for (int k = 0; k < 6; ++k) hu[k] = g.t_bc * hu[k];
      if (MU < 3)
        for (int k = 0; k < 6; ++k) hu[k] = g.hs * hu[k];
      accumulate<double, MU, false>(hd, hu);
      cross = coarse_extent && (c[MU] % a.bg.b[MU] == a.bg.b[MU] - 1);
    } else {
      n[MU] = (n[MU] == 0) ? g.L[MU] - 1 : n[MU] - 1;
      nb = cb_index(g, n);
      SpinorIO<double>::load(u_op, g.Vh, nb, psi);
      load_link<double, double>(a.gauge, g.Vh, 1 - p, MU, nb, U);
      project<double, MU, true>(psi, h);
      link_mul<double, true>(U, h, hu);
      if (MU == 3 && c[3] == 0)
        for (int k = 0; k < 6; ++k) hu[k] = g.t_bc * hu[k];
      if (MU < 3)
        for (int k = 0; k < 6; ++k) hu[k] = g.hs * hu[k];
      accumulate<double, MU, true>(hd, hu);
      cross = coarse_extent && (c[MU] % a.bg.b[MU] == 0);
    }
    void* bout = reinterpret_cast<char*>(a.bucket[1 + 2 * MU + back]) + (size_t)p * hb;
    cpx<double> w[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      hd[k] = -0.5 * hd[k];
      w[k] = cross ? hd[k] : mk(0.0, 0.0);
      if (!cross) acc0[k] = acc0[k] + hd[k];
    }
    SpinorIO<double>::store(bout, g.Vh, i, w);
  }
}

__global__ void __launch_bounds__(128) k_hop_split(SplitArgs a) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= 2 * a.g.Vh) return;
  const int p = gid / a.g.Vh, i = gid % a.g.Vh;
  int c[4];
  cb_coords(a.g, i, p, c);
  const size_t hb = (size_t)12 * a.g.Vh * 16;
  cpx<double> acc0[12];
  SpinorIO<double>::load(reinterpret_cast<const char*>(a.v) + (size_t)p * hb, a.g.Vh, i, acc0);
  split_mu<0>(a, p, i, c, acc0);
  split_mu<1>(a, p, i, c, acc0);
  split_mu<2>(a, p, i, c, acc0);
  split_mu<3>(a, p, i, c, acc0);
  SpinorIO<double>::store(reinterpret_cast<char*>(a.bucket[0]) + (size_t)p * hb, a.g.Vh, i, acc0);
}

}  // namespace

int coarse_internal_index_host(const BlockGeom& bg, int clex) {
  if (!bg.coarse_cb) return clex;
  int c0 = clex % bg.nb[0];
  int r = clex / bg.nb[0];
  int c1 = r % bg.nb[1];
  r /= bg.nb[1];
  int c2 = r % bg.nb[2];
  int c3 = r / bg.nb[2];
  int cp = (c0 + c1 + c2 + c3) & 1;
  return cp * (bg.Vc / 2) + (clex >> 1);
}

void launch_vec_blockmajor(void* out, const void* v32, int nvec, const Geom& g, const BlockGeom& bg, hipStream_t st) {
  const size_t total = (size_t)nvec * 2 * bg.Vc * (bg.bvol / 2);
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_vec_blockmajor, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const float4*>(v32),
                     reinterpret_cast<float4*>(out), nvec, dgeom(g), bg);
  HIPCHK(hipGetLastError());
}

void launch_restrict(int prec, void* out, size_t site_stride, size_t row_stride, const void* in, const void* vecs,
                     int nvec, int p, const Geom& g, const BlockGeom& bg, bool accumulate, hipStream_t st,
                     const void* vbm, const void* vbm16) {
  dim3 grid(bg.Vc, (nvec + kRestrictKB - 1) / kRestrictKB), block(128);
  size_t hb = spinor_bytes(prec, g.Vh);
  if (prec == WCMG_F64)
    hipLaunchKernelGGL(k_restrict<double>, grid, block, 0, st, out, site_stride, row_stride, in, vecs, 2 * hb, hb,
                       nvec, p, dgeom(g), bg, (int)accumulate);
  else if (prec == WCMG_F32)
    hipLaunchKernelGGL(k_restrict<float>, grid, block, 0, st, out, site_stride, row_stride, in, vecs, 2 * hb, hb,
                       nvec, p, dgeom(g), bg, (int)accumulate, reinterpret_cast<const float4*>(vbm),
                       reinterpret_cast<const uint2*>(vbm16));
  else
    hipLaunchKernelGGL(k_restrict<__half>, grid, block, 0, st, out, site_stride, row_stride, in, vecs, 2 * hb, hb,
                       nvec, p, dgeom(g), bg, (int)accumulate);
  HIPCHK(hipGetLastError());
}

void launch_prolong(int prec, void* out, const void* coarse, const void* vecs, int nvec, int p, const Geom& g,
                    const BlockGeom& bg, hipStream_t st, const void* v16) {
  dim3 grid((g.Vh + 255) / 256), block(256);
  size_t hb = spinor_bytes(prec, g.Vh);
  if (prec == WCMG_F64)
    hipLaunchKernelGGL(k_prolong<double>, grid, block, 0, st, out, coarse, vecs, 2 * hb, hb, nvec, p, dgeom(g), bg);
  else if (prec == WCMG_F32)
    hipLaunchKernelGGL(k_prolong<float>, grid, block, 0, st, out, coarse, vecs, 2 * hb, hb, nvec, p, dgeom(g), bg,
                       reinterpret_cast<const uint2*>(v16));
  else
    hipLaunchKernelGGL(k_prolong<__half>, grid, block, 0, st, out, coarse, vecs, 2 * hb, hb, nvec, p, dgeom(g), bg);
  HIPCHK(hipGetLastError());
}

void launch_chunks_to_half(void* out, const void* in32, size_t nchunks, hipStream_t st) {
  const size_t blocks = std::min<size_t>((nchunks + 255) / 256, 65535);
  hipLaunchKernelGGL(k_chunks_to_half, dim3((unsigned)blocks), dim3(256), 0, st, reinterpret_cast<uint2*>(out),
                     reinterpret_cast<const float4*>(in32), nchunks);
  HIPCHK(hipGetLastError());
}

void launch_block_orthonormalize(void* vecs, int nvec, const Geom& g, const BlockGeom& bg, int* flag,
                                 hipStream_t st) {
  if (bg.bvol > 256 * kOrthoSites) fail(WCMG_EDIM, "block volume too large for orthonormalisation");
  dim3 grid(bg.Vc, 2), block(256);
  hipLaunchKernelGGL(k_block_ortho, grid, block, 0, st, reinterpret_cast<double2*>(vecs), (size_t)24 * g.Vh, nvec,
                     dgeom(g), bg, flag);
  HIPCHK(hipGetLastError());
}

void launch_hop_split(void* const* buckets, const void* v, const void* u, const void* gauge64, const Geom& g,
                      const BlockGeom& bg, hipStream_t st) {
  SplitArgs a;
  for (int k = 0; k < 9; ++k) a.bucket[k] = reinterpret_cast<double2*>(buckets[k]);
  a.v = v;
  a.u = u;
  a.gauge = gauge64;
  a.g = dgeom(g);
  a.bg = bg;
  dim3 grid((2 * g.Vh + 127) / 128), block(128);
  hipLaunchKernelGGL(k_hop_split, grid, block, 0, st, a);
  HIPCHK(hipGetLastError());
}

}  // namespace wcmg
