// Persistent coarse-level GCR: one cooperative launch runs the whole
// approximate solve of the red-black reduced coarse operator (the coarse
// even-odd paragraph and the GCR of the solver paragraph), instead of a few
// hundred small launches with a host round trip per step.
//
//   b_r = b_e - Ytilde_eo b_o
//   GCR(m) on D_r_hat = 1 - Ytilde_eo Ytilde_oe, y_0 = 0, stopping at
//   ||r|| <= tol ||b_r|| (true residual recomputed at the end of every cycle)
//   c_e = X_ee^-1 y,  c_o = X_oo^-1 (b_o - Ytilde_oe y)
//
// Every workgroup owns the even sites w, w + W, w + 2W, ... (W workgroups)
// and the odd sites at the same offsets; the hops of a site are computed by
// its whole workgroup (column groups as in the stand-alone stencil), and
// the BLAS-1 work of a step touches only the workgroup's own sites, so the
// hop output of a site is consumed by the workgroup that wrote it.  Global
// sums go through per-workgroup partials: after a grid barrier every
// workgroup adds all partials in the same fixed order, so every workgroup
// takes the same decisions (convergence, breakdown) from bitwise the same
// numbers, and results do not depend on timing.
//
// A step takes two grid barriers.  The even-site hop q = D_r z_k is followed
// by the sums <q_j, q>, ||q||^2 and <q, r> (one barrier); since the q_j are
// orthonormal up to their norms and r is orthogonal to all of them,
// ||q_k||^2 = ||q||^2 - sum_j |<q_j, q>|^2 / ||q_j||^2 and <q_k, r> = <q, r>
// give alpha at once.  The update then needs no second reduction: the
// workgroup orthogonalises its own part of q_k and z_k, updates y and r, and
// builds the next odd-site hop by linearity, t <- t - alpha T_k with
// T_k = Ytilde_oe q_k = Ytilde_oe q - sum_j c_j T_j (the hop of q reads the
// neighbours' q, complete after the first barrier); the second barrier
// publishes t and ||r||^2.  The true residual at the end of every cycle
// removes what rounding these recurrences add.
//
// The grid barrier is a flag barrier: every workgroup stores the barrier's
// epoch to a cache line of its own, workgroup 0 waits for all of them and
// then stores the epoch to the generation word that the others wait for, so
// no address takes more than one write per barrier.  Every wait is bounded;
// past the bound it raises an abort flag that every waiting workgroup also
// polls, so all workgroups leave the kernel and the host reports the failure.
#include "kernels.h"

namespace wcmg {

namespace {

constexpr int kPT = 1024;              // threads per workgroup
constexpr int kPWaves = kPT / 64;      // wavefronts per workgroup
constexpr unsigned kSpinLimit = 1u << 22;
constexpr int kPMaxRestart = 64;       // longest GCR cycle

// two consecutive complex entries (rows 2r, 2r+1 of one column) of a coarse
// matrix (plain loads: small coarse operators stay in the Infinity Cache)
__device__ __forceinline__ void ld2(const float2* p, cpx<float>& e0, cpx<float>& e1) {
  const float4 t = *reinterpret_cast<const float4*>(p);
  e0 = mk(t.x, t.y);
  e1 = mk(t.z, t.w);
}
__device__ __forceinline__ void ld2(const double2* p, cpx<double>& e0, cpx<double>& e1) {
  const double2 t0 = p[0], t1 = p[1];
  e0 = mk(t0.x, t0.y);
  e1 = mk(t1.x, t1.y);
}

// Device-coherent access (relaxed atomics at agent scope: write-through
// stores, loads that do not hit stale lines of another compute unit or XCD)
// for everything one workgroup writes and another reads: residuals, the
// solution, the hop intermediate, the Krylov q vectors, the partial sums.
// With all such traffic coherent, a barrier needs only every wave's own
// stores to be complete, and no cache write-back or invalidation.
__device__ __forceinline__ float2 ldc(const float2* p) {
  const unsigned long long u =
      __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_bit_cast(float2, u);
}
__device__ __forceinline__ double2 ldc(const double2* p) {
  const double* d = reinterpret_cast<const double*>(p);
  double2 v;
  v.x = __hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  v.y = __hip_atomic_load(d + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return v;
}
__device__ __forceinline__ double ldc(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stc(float2* p, float2 v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), __builtin_bit_cast(unsigned long long, v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stc(double2* p, double2 v) {
  double* d = reinterpret_cast<double*>(p);
  __hip_atomic_store(d, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(d + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stc(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// element i as complex double, and back (rounded to the storage type)
template <typename V2>
__device__ __forceinline__ cpx<double> ldd(const V2* p, size_t i) {
  const V2 v = ldc(p + i);
  return mk((double)v.x, (double)v.y);
}
template <typename V2>
__device__ __forceinline__ void std_(V2* p, size_t i, cpx<double> c) {
  V2 v;
  v.x = c.r;
  v.y = c.i;
  stc(p + i, v);
}

// Flag barrier over ctl: generation word ctl[0], arrival flag of workgroup w
// at ctl[32 (w + 1)] (one 128-byte line each).  Epochs increase by one per
// barrier from the generation found at kernel start.  Returns false when a
// wait timed out or another workgroup aborted.
__device__ bool grid_barrier(unsigned* ctl, int* abort_flag, unsigned epoch) {
  __shared__ int ok_s;
  // every wave: its coherent stores have completed (the memory clobber keeps
  // the compiler from moving memory accesses across the wait)
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    ok_s = 1;
    __hip_atomic_store(ctl + 32 * (blockIdx.x + 1), epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (blockIdx.x == 0) {
    __syncthreads();
    for (int q = threadIdx.x; q < (int)gridDim.x; q += blockDim.x) {
      unsigned spins = 0;
      while (__hip_atomic_load(ctl + 32 * (q + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > kSpinLimit) {
          __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok_s = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0 && ok_s) __hip_atomic_store(ctl, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (threadIdx.x == 0 && ok_s) {
    unsigned spins = 0;
    while (__hip_atomic_load(ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > kSpinLimit) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok_s = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  return ok_s != 0;
}

// r - a q rounded to the storage type, without contraction, so that the
// owner of a site and the neighbours that rebuild it get the same bits
template <typename S>
__device__ __forceinline__ cpx<double> axpy_round(cpx<double> r, cpx<double> a, cpx<double> q) {
#pragma clang fp contract(off)
  const double vr = r.r - (a.r * q.r - a.i * q.i);
  const double vi = r.i - (a.r * q.i + a.i * q.r);
  return mk((double)(S)vr, (double)(S)vi);
}

// wavefront sum, the result valid in lane 0 (fixed shuffle tree)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  return v;
}

// Block sum of NR values into part[0..NR), fixed order (lanes, then waves).
template <int NR>
__device__ __forceinline__ void block_partial(double (&v)[NR], double* part, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    double s = wave_sum(v[k]);
    if (lane == 0) sh[k * kPWaves + wave] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < NR) {
    double s = 0.0;
    for (int q = 0; q < kPWaves; ++q) s += sh[threadIdx.x * kPWaves + q];
    stc(part + threadIdx.x, s);
  }
  __syncthreads();
}

// out[v] (LDS) = sum over workgroups of part[w * stride + v], v < nv: TPV
// threads per value (a power of two) each add a fixed strided subset of the
// workgroups, then a fixed shuffle tree (and, past one wavefront, LDS) adds
// the TPV subtotals; the same order in every workgroup
__device__ void grid_sum(const double* part, int stride, int nv, double* out, double* scratch) {
  if (nv <= 0) return;
  int tpv = 1;
  while (tpv * 2 * nv <= (int)blockDim.x && tpv < (int)gridDim.x) tpv *= 2;
  const int t = threadIdx.x, v = t / tpv, j = t - v * tpv;
  double s = 0.0;
  if (v < nv)
    for (int b = j; b < (int)gridDim.x; b += tpv) s += ldc(part + (size_t)b * stride + v);
  const int width = tpv < 64 ? tpv : 64;
  for (int off = width >> 1; off > 0; off >>= 1) s += __shfl_down(s, off, width);
  if (tpv <= 64) {
    if (v < nv && j == 0) out[v] = s;
  } else {
    // tpv / 64 wavefronts per value: their lane-0 subtotals in wave order
    const int lane = t & 63, wave = t >> 6;
    if (lane == 0) scratch[wave] = s;
    __syncthreads();
    if (v < nv && j == 0) {
      double u = 0.0;
      for (int q = 0; q < tpv / 64; ++q) u += scratch[wave + q];
      out[v] = u;
    }
  }
  __syncthreads();
}

// plain (cacheable) load of data this workgroup wrote itself
template <typename V2>
__device__ __forceinline__ cpx<double> ldo(const V2* p, size_t i) {
  const V2 v = p[i];
  return mk((double)v.x, (double)v.y);
}

struct PArgs {
  const void* Yt;    // [V][8][n][n] column-major hop blocks Ytilde
  const void* Xinv;  // [V][n][n] column-major
  const int* nbr;    // [V][8]
  const void* b;     // [V][n] right-hand side
  void* c;           // [V][n] solution
  void* t;           // [V][n] scratch (odd half)
  void* y;           // [Vh][n]
  void* r;           // [Vh][n]
  void* qraw;        // [Vh][n] D_r z of the current step, before orthogonalisation
  void* br;          // [Vh][n]
  void* Q;           // [restart][Vh][n]
  void* Z;           // [restart][Vh][n]
  void* T;           // [restart][V][n]: Ytilde_oe q_j on the odd sites
  double* part;      // [2][W][stride]: written before a barrier, read by all after it (two buffers
                     // alternate, so a fast workgroup never overwrites what a slow one still reads)
  unsigned* bar;     // barrier lines: generation, then one arrival flag per workgroup
  int* info;         // [0] iterations (accumulated), [1] status, [2] abort
  double tol;
  int Vh, n, restart, maxiter, fixed, G, stride;
};

// Rows of M v for one site (M: n x ncols column-major, v in LDS): lanes with
// column group 0 return rows 2rp, 2rp + 1; every lane of the block must call.
template <typename C, typename V2>
__device__ __forceinline__ void site_matvec(const V2* M, const cpx<C>* v, int n, int ncols, int G, cpx<C>* part,
                                            cpx<C>& o0, cpx<C>& o1) {
  const int R2 = n >> 1;
  const int g = threadIdx.x / R2, rp = threadIdx.x - g * R2;
  if (g < G) {
    cpx<C> a0 = mk((C)0, (C)0), a1 = a0;
    const V2* m = M + 2 * rp;
#pragma unroll 8
    for (int col = g; col < ncols; col += G) {
      cpx<C> e0, e1;
      ld2(m + (size_t)col * n, e0, e1);
      const cpx<C> x = v[col];
      cfma(a0, e0, x);
      cfma(a1, e1, x);
    }
    part[g * n + 2 * rp] = a0;
    part[g * n + 2 * rp + 1] = a1;
  }
  for (int h = G >> 1; h > 0; h >>= 1) {
    __syncthreads();
    if (g < h) {
      part[g * n + 2 * rp] = part[g * n + 2 * rp] + part[(g + h) * n + 2 * rp];
      part[g * n + 2 * rp + 1] = part[g * n + 2 * rp + 1] + part[(g + h) * n + 2 * rp + 1];
    }
  }
  o0 = mk((C)0, (C)0);
  o1 = o0;
  if (g == 0) {
    o0 = part[2 * rp];
    o1 = part[2 * rp + 1];
  }
}

// out(c) = xd(c) + coeff * sum_d Yt_d(c) in(nb(c, d))     (xd may be null)
// and, with Xl, out(c) = Xl(c) [ ... ] instead; with q, the neighbour values
// are in - alpha q (rounded as the owner rounds them)
template <typename S>
__device__ void site_hop(const PArgs& a, int c, const void* in_, const void* xd_, double coeff, const void* Xl_,
                         void* out_, cpx<typename Compute<S>::T>* vin, cpx<typename Compute<S>::T>* part,
                         const void* q_ = nullptr, cpx<double> alpha = cpx<double>{0.0, 0.0}) {
  using C = typename Compute<S>::T;
  using V2 = typename Vec2<S>::T;
  const int n = a.n;
  const V2* in = reinterpret_cast<const V2*>(in_);
  const V2* xd = reinterpret_cast<const V2*>(xd_);
  const V2* q = reinterpret_cast<const V2*>(q_);
  V2* out = reinterpret_cast<V2*>(out_);
  __syncthreads();  // the previous task is done with vin and part
  for (int t = threadIdx.x; t < 8 * n; t += kPT) {
    const int d = t / n, j = t - d * n;
    const size_t e = (size_t)a.nbr[(size_t)c * 8 + d] * n + j;
    if (q) {
      const cpx<double> v = axpy_round<S>(ldd(in, e), alpha, ldd(q, e));
      vin[t] = mk((C)v.r, (C)v.i);
    } else {
      const V2 w = ldc(in + e);
      vin[t] = mk((C)w.x, (C)w.y);
    }
  }
  __syncthreads();
  cpx<C> o[2];
  site_matvec<C, V2>(reinterpret_cast<const V2*>(a.Yt) + (size_t)c * 8 * n * n, vin, n, 8 * n, a.G, part, o[0],
                     o[1]);
  const int R2 = n >> 1;
  const int g = threadIdx.x / R2, rp = threadIdx.x - g * R2;
  cpx<C> s[2];
  if (g == 0) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int i = 2 * rp + k;
      s[k] = (C)coeff * o[k];
      if (xd) {
        const V2 w = ldc(xd + (size_t)c * n + i);
        s[k] = s[k] + mk((C)w.x, (C)w.y);
      }
    }
  }
  if (!Xl_) {
    if (g == 0) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        V2 w;
        w.x = (S)s[k].r;
        w.y = (S)s[k].i;
        stc(out + (size_t)c * n + 2 * rp + k, w);
      }
    }
    return;
  }
  // local matrix on the hop result: stage it in vin (rounded to storage precision)
  __syncthreads();
  if (g == 0) {
#pragma unroll
    for (int k = 0; k < 2; ++k) vin[2 * rp + k] = mk((C)(S)s[k].r, (C)(S)s[k].i);
  }
  __syncthreads();
  site_matvec<C, V2>(reinterpret_cast<const V2*>(Xl_) + (size_t)c * n * n, vin, n, n, a.G, part, o[0], o[1]);
  if (g == 0) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      V2 w;
      w.x = (S)o[k].r;
      w.y = (S)o[k].i;
      stc(out + (size_t)c * n + 2 * rp + k, w);
    }
  }
}

// out(c) = Xl(c) in(c)
template <typename S>
__device__ void site_local(const PArgs& a, int c, const void* in_, const void* Xl_, void* out_,
                           cpx<typename Compute<S>::T>* vin, cpx<typename Compute<S>::T>* part) {
  using C = typename Compute<S>::T;
  using V2 = typename Vec2<S>::T;
  const int n = a.n;
  const V2* in = reinterpret_cast<const V2*>(in_);
  V2* out = reinterpret_cast<V2*>(out_);
  __syncthreads();
  for (int t = threadIdx.x; t < n; t += kPT) {
    const V2 w = ldc(in + (size_t)c * n + t);
    vin[t] = mk((C)w.x, (C)w.y);
  }
  __syncthreads();
  cpx<C> o[2];
  site_matvec<C, V2>(reinterpret_cast<const V2*>(Xl_) + (size_t)c * n * n, vin, n, n, a.G, part, o[0], o[1]);
  const int R2 = n >> 1;
  const int g = threadIdx.x / R2, rp = threadIdx.x - g * R2;
  if (g == 0) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      V2 w;
      w.x = (S)o[k].r;
      w.y = (S)o[k].i;
      stc(out + (size_t)c * n + 2 * rp + k, w);
    }
  }
}

template <typename S>
__global__ void __launch_bounds__(kPT) k_coarse_gcr(PArgs a) {
  using C = typename Compute<S>::T;
  using V2 = typename Vec2<S>::T;
  extern __shared__ char smem[];  // hop operands, or the slice sums of the Gram-Schmidt step
  cpx<C>* vin = reinterpret_cast<cpx<C>*>(smem);  // 8n
  cpx<C>* hp = vin + 8 * a.n;                     // G * n
  __shared__ double sv[2 * kPMaxRestart + 8];      // grid sums
  __shared__ double sqq[kPMaxRestart];             // ||q_j||^2
  __shared__ double sh[4 * kPWaves];
  const int w = blockIdx.x, W = gridDim.x;
  const int n = a.n, Vh = a.Vh;
  const int nel = (w < Vh ? (Vh - w + W - 1) / W : 0) * n;  // elements of the owned even sites
  const size_t hv = (size_t)Vh * n;
  int* abort_flag = a.info + 2;
  // epochs continue from the generation the previous launch left
  unsigned epoch = __hip_atomic_load(a.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int cur = 0;  // partial buffer written in the current phase
  auto mine = [&]() { return a.part + ((size_t)cur * W + w) * a.stride; };
  // barrier, then the grid sums of the nv values of the phase just ended
  auto sync_sum = [&](int nv) -> bool {
    if (!grid_barrier(a.bar, abort_flag, ++epoch)) return false;
    if (nv > 0) grid_sum(a.part + (size_t)cur * W * a.stride, a.stride, nv, sv, sh);
    cur ^= 1;
    return true;
  };
  auto el = [&](int idx) -> size_t { return (size_t)(w + (idx / n) * W) * n + (idx % n); };
  V2* y = reinterpret_cast<V2*>(a.y);
  V2* br = reinterpret_cast<V2*>(a.br);
  auto Qv = [&](int j) { return reinterpret_cast<V2*>(a.Q) + (size_t)j * hv; };
  auto Zv = [&](int j) { return reinterpret_cast<V2*>(a.Z) + (size_t)j * hv; };

  // reduced source, r = b_r, y = 0, ||b_r||^2
  for (int i = w; i < Vh; i += W) site_hop<S>(a, i, a.b, a.b, -1.0, nullptr, a.br, vin, hp);
  __syncthreads();
  V2* r = reinterpret_cast<V2*>(a.r);
  V2* qraw = reinterpret_cast<V2*>(a.qraw);
  V2* t = reinterpret_cast<V2*>(a.t);
  auto Tv = [&](int j) { return reinterpret_cast<V2*>(a.T) + (size_t)j * 2 * hv; };  // full-size, odd half used
  {
    double v[1] = {0.0};
    for (int idx = threadIdx.x; idx < nel; idx += kPT) {
      const size_t e = el(idx);
      cpx<double> x = ldd(br, e);
      stc(r + e, ldc(br + e));
      std_(y, e, mk(0.0, 0.0));
      v[0] += x.r * x.r + x.i * x.i;
    }
    block_partial<1>(v, mine(), sh);
  }
  if (!sync_sum(1)) return;
  const double bn2 = sv[0];
  const double target = a.tol * sqrt(bn2);
  double rn2 = bn2;
  int iters = 0, status = 0;
  bool conv = !(bn2 > 0.0) || (!a.fixed && sqrt(rn2) <= target);
  if (!isfinite(bn2)) {
    status = WCMG_ENAN;
    conv = true;
  }
  __shared__ double salpha[3];  // alpha (re, im) and ||q_k||^2 of the current step
  while (!conv && iters < a.maxiter) {
    // cycle start: z_0 = r, t = Ytilde_oe r
    for (int i = w; i < Vh; i += W) site_hop<S>(a, Vh + i, r, nullptr, 1.0, nullptr, a.t, vin, hp);
    for (int idx = threadIdx.x; idx < nel; idx += kPT) {
      const size_t e = el(idx);
      stc(Zv(0) + e, ldc(r + e));
    }
    if (!sync_sum(0)) return;
    int k = 0;
    for (;;) {
      V2* Qk = Qv(k);
      V2* Zk = Zv(k);
      V2* Tk = Tv(k);
      // q = D_r z_k = r - Ytilde_eo t; <q_j, q> for j < k, ||q||^2 and <q, r> over the owned sites
      for (int i = w; i < Vh; i += W) site_hop<S>(a, i, a.t, r, -1.0, nullptr, a.qraw, vin, hp);
      __syncthreads();
      {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        for (int j = wave; j < k; j += kPWaves) {
          const V2* Qj = Qv(j);
          double sr = 0.0, si = 0.0;
          for (int idx = lane; idx < nel; idx += 64) {
            const size_t e = el(idx);
            cpx<double> u = ldo(Qj, e), qv = ldd(qraw, e);
            sr += u.r * qv.r + u.i * qv.i;
            si += u.r * qv.i - u.i * qv.r;
          }
          sr = wave_sum(sr);
          si = wave_sum(si);
          if (lane == 0) {
            stc(mine() + 2 * j, sr);
            stc(mine() + 2 * j + 1, si);
          }
        }
        double v[3] = {0.0, 0.0, 0.0};
        for (int idx = threadIdx.x; idx < nel; idx += kPT) {
          const size_t e = el(idx);
          const cpx<double> qv = ldd(qraw, e), rr = ldd(r, e);
          v[0] += qv.r * qv.r + qv.i * qv.i;
          v[1] += qv.r * rr.r + qv.i * rr.i;
          v[2] += qv.r * rr.i - qv.i * rr.r;
        }
        block_partial<3>(v, mine() + 2 * k, sh);
      }
      if (!sync_sum(2 * k + 3)) return;
      // q_k = q - sum_j c_j q_j with c_j = <q_j, q> / ||q_j||^2, the q_j orthogonal:
      // ||q_k||^2 = ||q||^2 - sum_j |<q_j, q>|^2 / ||q_j||^2, and <q_k, r> = <q, r>
      // (r is orthogonal to every q_j)
      if (threadIdx.x == 0) {
        double qq = sv[2 * k];
        for (int j = 0; j < k; ++j)
          if (sqq[j] > 0.0) qq -= (sv[2 * j] * sv[2 * j] + sv[2 * j + 1] * sv[2 * j + 1]) / sqq[j];
        salpha[2] = qq;
        salpha[0] = qq > 0.0 ? sv[2 * k + 1] / qq : 0.0;
        salpha[1] = qq > 0.0 ? sv[2 * k + 2] / qq : 0.0;
      }
      __syncthreads();
      const double qq = salpha[2];
      if (!(qq > 0.0) || !isfinite(qq)) {
        status = isfinite(qq) ? WCMG_EBREAKDOWN : WCMG_ENAN;
        break;
      }
      const cpx<double> alpha = mk(salpha[0], salpha[1]);
      // the pair (q_k, z_k) by classical Gram-Schmidt (the sum over j split over NS slices
      // of threads, combined in LDS in slice order); y += alpha z_k, r -= alpha q_k,
      // z_{k+1} = r, ||r||^2
      double vr[1] = {0.0};
      {
        cpx<double>* acc = reinterpret_cast<cpx<double>*>(smem);  // [2][kPT]
        V2* Zn = k + 1 < a.restart ? Zv(k + 1) : nullptr;
        const int CH = nel < kPT ? nel : kPT;
        for (int base = 0; base < nel; base += CH) {
          const int NS = k > 0 ? max(1, min(kPT / CH, k)) : 1;
          const int tt = threadIdx.x;
          const int sl = tt / CH, idx = base + (tt - sl * CH);
          if (k > 0 && sl < NS && idx < nel) {
            const size_t e = el(idx);
            cpx<double> aq = mk(0.0, 0.0), az = aq;
            for (int j = sl; j < k; j += NS) {
              const double d = sqq[j];
              const cpx<double> cj = d > 0.0 ? mk(sv[2 * j] / d, sv[2 * j + 1] / d) : mk(0.0, 0.0);
              aq = aq + cj * ldo(Qv(j), e);
              az = az + cj * ldo(Zv(j), e);
            }
            acc[tt] = aq;
            acc[kPT + tt] = az;
          }
          __syncthreads();
          if (tt < CH && idx < nel) {
            const size_t e = el(idx);
            cpx<double> q = ldd(qraw, e), z = ldo(Zk, e);
            if (k > 0) {
              cpx<double> sq = acc[tt], sz = acc[kPT + tt];
              for (int u = 1; u < NS; ++u) {
                sq = sq + acc[u * CH + tt];
                sz = sz + acc[kPT + u * CH + tt];
              }
              q = q - sq;
              z = z - sz;
            }
            // the stored (rounded) values, without reading them back
            const cpx<double> qs = mk((double)(S)q.r, (double)(S)q.i), zs = mk((double)(S)z.r, (double)(S)z.i);
            std_(Qk, e, qs);
            std_(Zk, e, zs);
            std_(y, e, ldd(y, e) + alpha * zs);
            const cpx<double> rs = axpy_round<S>(ldd(r, e), alpha, qs);
            std_(r, e, rs);
            if (Zn) std_(Zn, e, rs);
            vr[0] += rs.r * rs.r + rs.i * rs.i;
          }
          __syncthreads();
        }
      }
      // odd sites: T_k = Ytilde_oe q_k = Ytilde_oe q - sum_j c_j T_j, and t -= alpha T_k
      for (int i = w; i < Vh; i += W) site_hop<S>(a, Vh + i, a.qraw, nullptr, 1.0, nullptr, Tk, vin, hp);
      __syncthreads();
      {
        cpx<double>* acc = reinterpret_cast<cpx<double>*>(smem);  // [kPT]
        const int CH = nel < kPT ? nel : kPT;
        for (int base = 0; base < nel; base += CH) {
          const int NS = k > 0 ? max(1, min(kPT / CH, k)) : 1;
          const int tt = threadIdx.x;
          const int sl = tt / CH, idx = base + (tt - sl * CH);
          if (k > 0 && sl < NS && idx < nel) {
            const size_t e = el(idx) + hv;  // odd element of the owned odd site
            cpx<double> at = mk(0.0, 0.0);
            for (int j = sl; j < k; j += NS) {
              const double d = sqq[j];
              const cpx<double> cj = d > 0.0 ? mk(sv[2 * j] / d, sv[2 * j + 1] / d) : mk(0.0, 0.0);
              at = at + cj * ldo(Tv(j), e);
            }
            acc[tt] = at;
          }
          __syncthreads();
          if (tt < CH && idx < nel) {
            const size_t e = el(idx) + hv;
            cpx<double> tk = ldd(Tk, e);
            if (k > 0) {
              cpx<double> st = acc[tt];
              for (int u = 1; u < NS; ++u) st = st + acc[u * CH + tt];
              tk = tk - st;
            }
            const cpx<double> tks = mk((double)(S)tk.r, (double)(S)tk.i);
            std_(Tk, e, tks);
            std_(t, e, ldd(t, e) - alpha * tks);
          }
          __syncthreads();
        }
      }
      if (threadIdx.x == 0) sqq[k] = qq;
      block_partial<1>(vr, mine(), sh);
      if (!sync_sum(1)) return;
      rn2 = sv[0];
      ++k;
      ++iters;
      if (!isfinite(rn2)) {
        status = WCMG_ENAN;
        break;
      }
      if (k >= a.restart || iters >= a.maxiter || (!a.fixed && sqrt(rn2) <= target)) break;
    }
    if (status || a.fixed) break;
    // true residual r = b_r - D_r y at the end of the cycle (q_raw as scratch)
    for (int i = w; i < Vh; i += W) site_hop<S>(a, Vh + i, a.y, nullptr, 1.0, nullptr, a.t, vin, hp);
    if (!sync_sum(0)) return;
    for (int i = w; i < Vh; i += W) site_hop<S>(a, i, a.t, a.y, -1.0, nullptr, a.qraw, vin, hp);
    __syncthreads();
    {
      double v[1] = {0.0};
      for (int idx = threadIdx.x; idx < nel; idx += kPT) {
        const size_t e = el(idx);
        std_(r, e, ldd(br, e) - ldd(qraw, e));
        const cpx<double> rs = ldd(r, e);
        v[0] += rs.r * rs.r + rs.i * rs.i;
      }
      block_partial<1>(v, mine(), sh);
    }
    if (!sync_sum(1)) return;
    rn2 = sv[0];
    if (!isfinite(rn2)) {
      status = WCMG_ENAN;
      break;
    }
    if (sqrt(rn2) <= target) conv = true;
  }
  // c_e = X_ee^-1 y,  c_o = X_oo^-1 (b_o - Ytilde_oe y)   (y is final and visible after the last barrier)
  for (int i = w; i < Vh; i += W) {
    site_local<S>(a, i, a.y, a.Xinv, a.c, vin, hp);
    site_hop<S>(a, Vh + i, a.y, a.b, -1.0, a.Xinv, a.c, vin, hp);
  }
  if (w == 0 && threadIdx.x == 0) {
    a.info[0] += iters;
    if (status) a.info[1] = status;
  }
}

}  // namespace

size_t coarse_gcr_persistent_part_doubles() { return 2 * kPMaxRestart + 8; }

int coarse_gcr_persistent_grid(int prec, int n, int Vh) {
  int dev = 0, ncu = 0, coop = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  if (!coop || n % 2 || n > 256 || Vh <= 0) return 0;
  const size_t cb = prec == WCMG_F64 ? 16 : 8;
  int R2 = n / 2, G = 1;
  while (G < 64 && 2 * G * R2 <= kPT) G *= 2;
  const size_t shm = std::max((size_t)(8 * n + G * n) * cb, (size_t)2 * kPT * 16);
  int per = 0;
  if (prec == WCMG_F64)
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_coarse_gcr<double>, kPT, shm));
  else
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_coarse_gcr<float>, kPT, shm));
  if (per < 1) return 0;
  return std::min(std::min(ncu, Vh), 256);
}

void launch_coarse_gcr_persistent(int prec, const CoarseGcrArgs& g, hipStream_t st) {
  const int n = g.n;
  if (n % 2 || n > 256) fail(WCMG_EDIM, "coarse block size must be even and <= 256");
  if (g.restart < 1 || g.restart > kPMaxRestart) fail(WCMG_EINVAL, "coarse restart length out of range");
  if (g.grid < 1 || g.grid > 256) fail(WCMG_EINVAL, "persistent coarse solve needs 1..256 workgroups");
  PArgs a{};
  a.Yt = g.Yt;
  a.Xinv = g.Xinv;
  a.nbr = g.nbr;
  a.b = g.b;
  a.c = g.c;
  a.t = g.t;
  a.y = g.y;
  a.r = g.r;
  a.br = g.br;
  a.Q = g.Q;
  a.Z = g.Z;
  a.T = g.T;
  a.qraw = g.qraw;
  a.part = g.part;
  a.bar = g.bar;
  a.info = g.info;
  a.tol = g.tol;
  a.Vh = g.Vh;
  a.n = n;
  a.restart = g.restart;
  a.maxiter = g.maxiter;
  a.fixed = g.fixed;
  a.stride = (int)coarse_gcr_persistent_part_doubles();
  int R2 = n / 2, G = 1;
  while (G < 64 && 2 * G * R2 <= kPT) G *= 2;
  a.G = G;
  const size_t cb = prec == WCMG_F64 ? 16 : 8;
  const size_t shm = std::max((size_t)(8 * n + G * n) * cb, (size_t)2 * kPT * 16);
  void* args[] = {&a};
  if (prec == WCMG_F64)
    HIPCHK(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_coarse_gcr<double>), dim3(g.grid), dim3(kPT),
                                      args, (unsigned)shm, st));
  else
    HIPCHK(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_coarse_gcr<float>), dim3(g.grid), dim3(kPT),
                                      args, (unsigned)shm, st));
}

}  // namespace wcmg
