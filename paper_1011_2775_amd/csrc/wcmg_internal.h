// Internal types, layouts and device helpers of the wcmg library (gfx950).
//
// Data layouts in HBM (all "SoA by site", so that the 64 lanes of a
// wavefront touch consecutive addresses):
//
//  * Sites are split by parity p = (x+y+z+t) mod 2 (the red-black split of
//    Eq.(2)); within a parity the checkerboard index is lex/2 with
//    lex = ((t*Lz + z)*Ly + y)*Lx + x.  Vh = V/2 sites per parity.
//  * Spinor (one parity): 12 complex components (spin*3 + colour), stored
//    as chunks of 16 bytes: F64 -> 12 x double2, F32 -> 6 x float4
//    (2 complex), F16 -> 3 x 8 halves (4 complex) plus one float scale per
//    site.  Chunk c of site i lives at chunk_base[c*Vh + i].
//  * Gauge: links[p][mu][k][Vh] with k = 0..8 the row-major 3x3 entries,
//    as complex of the storage type; p is the parity of the site that owns
//    the link U_mu(x).  The time boundary phase is not folded into the
//    links; kernels apply it from the site coordinate.
//  * Clover: clov[p][kind][72][Vh] reals, kind 0 = A (4+m0 + clover),
//    kind 1 = A^-1.  Per chirality block (6x6 Hermitian, index
//    spin_local*3 + colour): 6 real diagonal entries, then the 15 complex
//    strictly-lower entries in row order (1,0),(2,0),(2,1),(3,0),...
//  * Null vectors: full-lattice spinors (both parities), one after another.
//  * Coarse vectors: [Vc_parity-split][2Nv] complex, see coarse.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/wcmg.h"

namespace wcmg {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Error {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);
void hip_check(hipError_t e, const char* what, const char* file, int line);
#define HIPCHK(x) ::wcmg::hip_check((x), #x, __FILE__, __LINE__)

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
struct Geom {
  int L[4];     // Lx, Ly, Lz, Lt
  int V;        // sites
  int Vh;       // sites per parity
  int Lxh;      // Lx / 2
  double t_bc;  // fermion phase on hops that wrap around t (fine level)
  double hs = 1.0;  // coefficient of the spatial hops (anisotropic lattices; 1: isotropic)
};

Geom make_geom(const int dims[4], int t_bc);

// ---------------------------------------------------------------------------
// precision / storage
// ---------------------------------------------------------------------------
inline size_t real_size(int prec) { return prec == WCMG_F64 ? 8 : (prec == WCMG_F32 ? 4 : 2); }
// bytes of one parity of a spinor (12 complex per site), F16 includes scales
inline size_t spinor_bytes(int prec, int Vh) {
  size_t b = (size_t)Vh * 24 * real_size(prec);
  if (prec == WCMG_F16) b += (size_t)Vh * sizeof(float);
  return b;
}
inline size_t gauge_bytes(int prec, int V) { return (size_t)V * 4 * 18 * real_size(prec); }
inline size_t clover_bytes(int prec, int V) { return (size_t)V * 2 * 72 * real_size(prec); }

// ---------------------------------------------------------------------------
// device complex helpers
// ---------------------------------------------------------------------------
template <typename T>
struct cpx {
  T r, i;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T r, T i) {
  cpx<T> c;
  c.r = r;
  c.i = i;
  return c;
}
template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk(a.r + b.r, a.i + b.i); }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk(a.r - b.r, a.i - b.i); }
template <typename T>
__device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return mk(a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r);
}
template <typename T>
__device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return mk(s * a.r, s * a.i); }
// conj(a) * b
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
  return mk(a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r);
}
template <typename T>
__device__ __forceinline__ cpx<T> ci(cpx<T> a) { return mk(-a.i, a.r); }   // i*a
template <typename T>
__device__ __forceinline__ cpx<T> cmi(cpx<T> a) { return mk(a.i, -a.r); }  // -i*a
template <typename T>
__device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return mk(a.r, -a.i); }
// acc += a*b
template <typename T>
__device__ __forceinline__ void cfma(cpx<T>& acc, cpx<T> a, cpx<T> b) {
  acc.r = fma(a.r, b.r, acc.r);
  acc.r = fma(-a.i, b.i, acc.r);
  acc.i = fma(a.r, b.i, acc.i);
  acc.i = fma(a.i, b.r, acc.i);
}
// acc += conj(a)*b
template <typename T>
__device__ __forceinline__ void cfmac(cpx<T>& acc, cpx<T> a, cpx<T> b) {
  acc.r = fma(a.r, b.r, acc.r);
  acc.r = fma(a.i, b.i, acc.r);
  acc.i = fma(a.r, b.i, acc.i);
  acc.i = fma(-a.i, b.r, acc.i);
}

// compute type for a storage type
template <typename S>
struct Compute {
  using T = float;
};
template <>
struct Compute<double> {
  using T = double;
};

// ---------------------------------------------------------------------------
// spinor chunk I/O (one parity, 12 complex per site)
// ---------------------------------------------------------------------------
// Loads of data a launch reads exactly once (links, clover, the diagonal
// input): non-temporal when the fields exceed the Infinity Cache, so that
// they do not evict the spinors that neighbouring sites read again; plain
// when the fields fit there and every launch finds them again.
typedef unsigned int ws_u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int ws_u32x4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8 || sizeof(T) == 16, "16, 8 or 4 bytes");
  if constexpr (sizeof(T) == 16) {
    return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const ws_u32x4*>(p)));
  } else if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const ws_u32x2*>(p)));
  } else {
    return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const unsigned int*>(p)));
  }
}
template <typename T>
__device__ __forceinline__ void st_stream(T* p, T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8 || sizeof(T) == 16, "16, 8 or 4 bytes");
  if constexpr (sizeof(T) == 16) {
    __builtin_nontemporal_store(__builtin_bit_cast(ws_u32x4, v), reinterpret_cast<ws_u32x4*>(p));
  } else if constexpr (sizeof(T) == 8) {
    __builtin_nontemporal_store(__builtin_bit_cast(ws_u32x2, v), reinterpret_cast<ws_u32x2*>(p));
  } else {
    __builtin_nontemporal_store(__builtin_bit_cast(unsigned int, v), reinterpret_cast<unsigned int*>(p));
  }
}
// plain or streamed element access
template <bool NT, typename T>
__device__ __forceinline__ T ld_maybe(const T* p) {
  if constexpr (NT)
    return ld_stream(p);
  else
    return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_maybe(T* p, T v) {
  if constexpr (NT)
    st_stream(p, v);
  else
    *p = v;
}

template <typename S>
struct SpinorIO;

template <>
struct SpinorIO<double> {
  static constexpr int kPrec = WCMG_F64;
  template <bool NT = false>
  __device__ __forceinline__ static void load(const void* base, int Vh, int i, cpx<double> v[12]) {
    const double2* p = reinterpret_cast<const double2*>(base);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      double2 t = ld_maybe<NT>(p + (size_t)c * Vh + i);
      v[c] = mk(t.x, t.y);
    }
  }
  template <bool NT = false>
  __device__ __forceinline__ static void store(void* base, int Vh, int i, const cpx<double> v[12]) {
    double2* p = reinterpret_cast<double2*>(base);
#pragma unroll
    for (int c = 0; c < 12; ++c) st_maybe<NT>(p + (size_t)c * Vh + i, make_double2(v[c].r, v[c].i));
  }
};

template <>
struct SpinorIO<float> {
  static constexpr int kPrec = WCMG_F32;
  template <bool NT = false>
  __device__ __forceinline__ static void load(const void* base, int Vh, int i, cpx<float> v[12]) {
    const float4* p = reinterpret_cast<const float4*>(base);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      float4 t = ld_maybe<NT>(p + (size_t)c * Vh + i);
      v[2 * c] = mk(t.x, t.y);
      v[2 * c + 1] = mk(t.z, t.w);
    }
  }
  template <bool NT = false>
  __device__ __forceinline__ static void store(void* base, int Vh, int i, const cpx<float> v[12]) {
    float4* p = reinterpret_cast<float4*>(base);
#pragma unroll
    for (int c = 0; c < 6; ++c)
      st_maybe<NT>(p + (size_t)c * Vh + i, make_float4(v[2 * c].r, v[2 * c].i, v[2 * c + 1].r, v[2 * c + 1].i));
  }
};

// F16: 3 chunks of 8 halves (uint4) followed by Vh float scales
template <>
struct SpinorIO<__half> {
  static constexpr int kPrec = WCMG_F16;
  __device__ __forceinline__ static const float* scales(const void* base, int Vh) {
    return reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + (size_t)Vh * 48);
  }
  template <bool NT = false>
  __device__ __forceinline__ static void load(const void* base, int Vh, int i, cpx<float> v[12]) {
    const uint4* p = reinterpret_cast<const uint4*>(base);
    float s = ld_maybe<NT>(scales(base, Vh) + i);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      uint4 t = ld_maybe<NT>(p + (size_t)c * Vh + i);
      unsigned w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        __half2 h = *reinterpret_cast<__half2*>(&w[k]);
        float2 f = __half22float2(h);
        v[4 * c + k] = mk(f.x * s, f.y * s);
      }
    }
  }
  template <bool NT = false>
  __device__ __forceinline__ static void store(void* base, int Vh, int i, const cpx<float> v[12]) {
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].r), fabsf(v[c].i)));
    float s = m > 0.f ? m : 1.f;
    float inv = 1.f / s;
    uint4* p = reinterpret_cast<uint4*>(base);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      unsigned w[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        __half2 h = __floats2half2_rn(v[4 * c + k].r * inv, v[4 * c + k].i * inv);
        w[k] = *reinterpret_cast<unsigned*>(&h);
      }
      st_maybe<NT>(p + (size_t)c * Vh + i, make_uint4(w[0], w[1], w[2], w[3]));
    }
    st_maybe<NT>(const_cast<float*>(scales(base, Vh)) + i, s);
  }
};

// ---------------------------------------------------------------------------
// link and clover loads
// ---------------------------------------------------------------------------
template <typename S>
struct Vec2;
template <>
struct Vec2<double> {
  using T = double2;
};
template <>
struct Vec2<float> {
  using T = float2;
};
template <>
struct Vec2<__half> {
  using T = __half2;
};

template <typename C>
__device__ __forceinline__ cpx<C> to_cpx(double2 v) { return mk((C)v.x, (C)v.y); }
template <typename C>
__device__ __forceinline__ cpx<C> to_cpx(float2 v) { return mk((C)v.x, (C)v.y); }
template <typename C>
__device__ __forceinline__ cpx<C> to_cpx(__half2 v) {
  float2 f = __half22float2(v);
  return mk((C)f.x, (C)f.y);
}

// link U[a][b] of (parity p, direction mu) at checkerboard site i
template <typename S, typename C, bool STREAM = false>
__device__ __forceinline__ void load_link(const void* gauge, int Vh, int p, int mu, int i, cpx<C> U[9]) {
  using V2 = typename Vec2<S>::T;
  const V2* g = reinterpret_cast<const V2*>(gauge) + ((size_t)(p * 4 + mu) * 9) * Vh;
#pragma unroll
  for (int k = 0; k < 9; ++k) U[k] = to_cpx<C>(ld_maybe<STREAM>(g + (size_t)k * Vh + i));
}

template <typename S>
__device__ __forceinline__ float to_f(S v);
template <>
__device__ __forceinline__ float to_f<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f<__half>(__half v) { return __half2float(v); }

// one chirality block (36 reals) of the packed clover (kind 0 = A, 1 = A^-1),
// applied to 6 complex in-place into out[6]
template <typename S, typename C>
__device__ __forceinline__ void clover_block_apply(const void* clov, int Vh, int p, int kind, int chi,
                                                   int i, const cpx<C> in[6], cpx<C> out[6]) {
  const S* c = reinterpret_cast<const S*>(clov) + ((size_t)(p * 2 + kind) * 72 + chi * 36) * Vh;
  C d[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) d[k] = (C)c[(size_t)k * Vh + i];
#pragma unroll
  for (int k = 0; k < 6; ++k) out[k] = mk(d[k] * in[k].r, d[k] * in[k].i);
  int t = 0;
#pragma unroll
  for (int r = 1; r < 6; ++r) {
#pragma unroll
    for (int s = 0; s < r; ++s) {
      cpx<C> L = mk((C)c[(size_t)(6 + 2 * t) * Vh + i], (C)c[(size_t)(7 + 2 * t) * Vh + i]);
      cfma(out[r], L, in[s]);    // lower entry (r,s)
      cfmac(out[s], L, in[r]);   // upper entry (s,r) = conj(L)
      ++t;
    }
  }
}

template <>
__device__ __forceinline__ void clover_block_apply<__half, float>(const void* clov, int Vh, int p, int kind,
                                                                  int chi, int i, const cpx<float> in[6],
                                                                  cpx<float> out[6]) {
  const __half* c = reinterpret_cast<const __half*>(clov) + ((size_t)(p * 2 + kind) * 72 + chi * 36) * Vh;
  float d[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) d[k] = __half2float(c[(size_t)k * Vh + i]);
#pragma unroll
  for (int k = 0; k < 6; ++k) out[k] = mk(d[k] * in[k].r, d[k] * in[k].i);
  int t = 0;
#pragma unroll
  for (int r = 1; r < 6; ++r) {
#pragma unroll
    for (int s = 0; s < r; ++s) {
      cpx<float> L = mk(__half2float(c[(size_t)(6 + 2 * t) * Vh + i]), __half2float(c[(size_t)(7 + 2 * t) * Vh + i]));
      cfma(out[r], L, in[s]);
      cfmac(out[s], L, in[r]);
      ++t;
    }
  }
}

template <typename S, typename C>
__device__ __forceinline__ void clover_apply(const void* clov, int Vh, int p, int kind, int i,
                                             const cpx<C> in[12], cpx<C> out[12]) {
  clover_block_apply<S, C>(clov, Vh, p, kind, 0, i, in, out);
  clover_block_apply<S, C>(clov, Vh, p, kind, 1, i, in + 6, out + 6);
}

// ---------------------------------------------------------------------------
// checkerboard geometry on the device
// ---------------------------------------------------------------------------
struct DGeom {
  int L[4];
  int Lxh;
  int Vh;
  double t_bc;
  double hs;  // spatial hop coefficient
};

inline DGeom dgeom(const Geom& g) {
  DGeom d;
  for (int k = 0; k < 4; ++k) d.L[k] = g.L[k];
  d.Lxh = g.Lxh;
  d.Vh = g.Vh;
  d.t_bc = g.t_bc;
  d.hs = g.hs;
  return d;
}

__device__ __forceinline__ void cb_coords(const DGeom& g, int i, int p, int c[4]) {
  int xh = i % g.Lxh;
  int r = i / g.Lxh;
  c[1] = r % g.L[1];
  r /= g.L[1];
  c[2] = r % g.L[2];
  c[3] = r / g.L[2];
  c[0] = 2 * xh + ((c[1] + c[2] + c[3] + p) & 1);
}

__device__ __forceinline__ int cb_index(const DGeom& g, const int c[4]) {
  return (((c[3] * g.L[2] + c[2]) * g.L[1] + c[1]) * g.L[0] + c[0]) >> 1;
}

// Map a launch block index onto a logical block so that each of the 8 XCDs
// (which receive workgroups round-robin) works on one contiguous range of
// sites; neighbours in z and t then hit the same L2.
__device__ __forceinline__ int xcd_block(int nlogical) {
  int b = blockIdx.x;
  int per = (nlogical + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}
inline int xcd_grid(int nlogical) { return ((nlogical + 7) >> 3) << 3; }

// ---------------------------------------------------------------------------
// small device buffer RAII
// ---------------------------------------------------------------------------
struct DBuf {
  void* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) {
    o.p = nullptr;
    o.n = 0;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(size_t bytes);  // (re)allocate, contents undefined
  void release();
  template <typename T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

}  // namespace wcmg
