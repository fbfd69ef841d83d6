// Persistent coarse-level GCR: one cooperative launch runs the whole
// approximate solve of the red-black reduced coarse operator (the coarse
// even-odd paragraph and the GCR of the solver paragraph), instead of a few
// hundred small launches with a host round trip per step.
//
//   b_r = b_e - Ytilde_eo b_o
//   GCR(m) on D_r_hat = 1 - Ytilde_eo Ytilde_oe, y_0 = 0, stopping at
//   ||r|| <= tol ||b_r|| (true residual recomputed at the end of every cycle,
//   except in a launch that trusts a recurrence residual which met the
//   tolerance: the multigrid cycle's coarse solves)
//   c_e = X_ee^-1 y,  c_o = X_oo^-1 (b_o - Ytilde_oe y)
//
// Every workgroup owns the even sites w, w + W, w + 2W, ... (W workgroups)
// and the odd sites at the same offsets; the hops of a site are computed by
// its whole workgroup (in the thread layout of site_matvec), and
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
// removes what rounding these recurrences add (a launch for a
// preconditioner's loose tolerance may end on the recurrence residual).
//
// The grid barrier is a flag barrier: every workgroup stores the barrier's
// epoch to a cache line of its own and waits until every line holds it, so
// no address takes more than one write per barrier.  Every wait is bounded;
// past the bound it raises an abort flag that every waiting workgroup also
// polls, so all workgroups leave the kernel and the host reports the failure.
#include "kernels.h"

// No implicit multiply-add contraction in this file: the two kernels below
// evaluate the same expressions in different surroundings, and with only the
// explicit fma of the matrix products their results agree bit for bit.
#pragma clang fp contract(off)

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
// FP16 hop blocks (the coarse_fp16 storage): two complex halves in 8 bytes,
// widened exactly to FP32
__device__ __forceinline__ void ld2(const __half2* p, cpx<float>& e0, cpx<float>& e1) {
  const uint2 t = *reinterpret_cast<const uint2*>(p);
  const float2 a = __half22float2(__builtin_bit_cast(__half2, t.x));
  const float2 b = __half22float2(__builtin_bit_cast(__half2, t.y));
  e0 = mk(a.x, a.y);
  e1 = mk(b.x, b.y);
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

// Flag barrier over ctl: arrival flag of workgroup w at ctl[32 (w + 1)] (one
// 128-byte line each), generation word ctl[0].  Epochs increase by one per
// barrier from the generation found at kernel start.  Split in two: arrival
// (the workgroup's coherent stores complete, then its flag) and completion
// (every workgroup waits for every flag itself: one round trip once all have
// arrived, where a leader that collects the flags and releases the others
// would add a second, and would start collecting only when it is itself done
// with the work placed between arrival and completion), so that work that
// needs only some workgroups' arrival can run in between.  Workgroup 0 keeps
// the generation word at the latest epoch for the next launch.  Completion
// returns false when a wait timed out or another workgroup aborted.
__device__ void barrier_arrive(unsigned* ctl, unsigned epoch) {
  // every wave: its coherent stores have completed (the memory clobber keeps
  // the compiler from moving memory accesses across the wait)
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(ctl + 32 * (blockIdx.x + 1), epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ bool barrier_complete(unsigned* ctl, int* abort_flag, unsigned epoch) {
  __shared__ int ok_s;
  if (threadIdx.x == 0) ok_s = 1;
  __syncthreads();
  for (int q = threadIdx.x; q < (int)gridDim.x; q += blockDim.x) {
    unsigned spins = 0;
    // flags only grow; a workgroup may already have arrived at a later barrier
    while ((int)(__hip_atomic_load(ctl + 32 * (q + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - epoch) < 0) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > kSpinLimit) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok_s = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0 && ok_s)
    __hip_atomic_store(ctl, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return ok_s != 0;
}

__device__ bool grid_barrier(unsigned* ctl, int* abort_flag, unsigned epoch) {
  barrier_arrive(ctl, epoch);
  return barrier_complete(ctl, abort_flag, epoch);
}

// Wait until workgroup own (a distinct one per thread, -1 for none) has
// arrived at barrier `epoch` of ctl (its stores before the arrival are then
// visible to coherent loads).  false on time-out or abort.
__device__ bool arrival_wait(const unsigned* ctl, int* abort_flag, int own, unsigned epoch) {
  __shared__ int oka;
  if (threadIdx.x == 0) oka = 1;
  __syncthreads();
  if (own >= 0) {
    unsigned spins = 0;
    while ((int)(__hip_atomic_load(ctl + 32 * (own + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - epoch) < 0) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > kSpinLimit) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        oka = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  return oka != 0;
}

// complex product evaluated under this file's no-contraction rule (the
// operator of the common header may be fused differently in each caller)
__device__ __forceinline__ cpx<double> cmul(cpx<double> a, cpx<double> b) {
  return mk(a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r);
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

// sum over the 8 lanes of a lane octet (lane % 8), the same bits in all 8: the
// DPP (data-parallel primitive) butterfly (pairs, quads, then the half-row mirror
// that meets the other quad); a + b = b + a keeps the partners equal
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <typename C>
__device__ __forceinline__ C sum8(C v) {
  v = v + dpp_f<0xB1>(v);   // quad_perm [1,0,3,2]
  v = v + dpp_f<0x4E>(v);   // quad_perm [2,3,0,1]
  v = v + dpp_f<0x141>(v);  // row_half_mirror
  return v;
}

// wavefront sum, the same bits in every lane (all 64 lanes must be active):
// the octet butterfly of sum8, the two octets of each row of 16 lanes (row
// rotation by 8), then the four row sums read from lanes 0, 16, 32 and 48
// and added as (r0 + r1) + (r2 + r3).  Cross-lane moves inside the ALU
// instead of LDS permutes.
__device__ __forceinline__ double rdlane(double v, int l) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)u, l), hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v = sum8(v);
  v = v + dpp_f<0x128>(v);  // row_ror:8
  return (rdlane(v, 0) + rdlane(v, 16)) + (rdlane(v, 32) + rdlane(v, 48));
}

// NR wavefront sums at once (independent chains the compiler interleaves;
// each result bitwise that of wave_sum)
template <int NR>
__device__ __forceinline__ void wave_sum_n(double (&v)[NR]) {
#pragma unroll
  for (int k = 0; k < NR; ++k) v[k] = wave_sum(v[k]);
}

// Block sum of NR values into part[0..NR), fixed order (lanes, then waves).
template <int NR>
__device__ __forceinline__ void block_partial(double (&v)[NR], double* part, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  wave_sum_n<NR>(v);
#pragma unroll
  for (int k = 0; k < NR; ++k)
    if (lane == 0) sh[k * kPWaves + wave] = v[k];
  __syncthreads();
  if ((int)threadIdx.x < NR) {
    double s = 0.0;
    for (int q = 0; q < kPWaves; ++q) s += sh[threadIdx.x * kPWaves + q];
    stc(part + threadIdx.x, s);
  }
  __syncthreads();
}

// block_partial when every nonzero value is in wavefront 0 (the other
// wavefronts would add exact zeros): lane 0 stores the wavefront sums, with no
// LDS round and no block barrier
template <int NR>
__device__ __forceinline__ void wave0_partial(double (&v)[NR], double* part) {
  if (threadIdx.x < 64) {
    wave_sum_n<NR>(v);
#pragma unroll
    for (int k = 0; k < NR; ++k)
      if (threadIdx.x == 0) stc(part + k, v[k]);
  }
}

// out[v] (LDS) = sum over workgroups of part[w * stride + v], v < nv, in the
// one order that every grid sum of this file uses: lane l of a wavefront adds
// the partials of workgroups l, l + 64, l + 128, ... in turn (eight loads in
// flight), then the fixed shuffle tree adds the 64 lane sums.  Wavefront q
// sums the values q, q + 16, ...
__device__ void grid_sum(const double* part, int stride, int nv, double* out, double* /*scratch*/) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, NWv = blockDim.x >> 6, W = gridDim.x;
  for (int v = wave; v < nv; v += NWv) {
    double s = 0.0;
    for (int b0 = lane; b0 < W; b0 += 8 * 64) {
      double p[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (b0 + 64 * u < W) p[u] = ldc(part + (size_t)(b0 + 64 * u) * stride + v);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (b0 + 64 * u < W) s += p[u];
    }
    s = wave_sum(s);
    if (lane == 0) out[v] = s;
  }
  __syncthreads();
}

// Tagged slots: 16 bytes {tag, payload lo, payload hi, tag}, written and read
// whole with one coherent (agent-scope, the same cache bit as the relaxed
// agent-scope atomics) 16-byte buffer access.  A reader accepts a slot only
// when both tags equal the version it expects, so data that carries its own
// version needs no separate flag, no wait for the writer's stores to
// complete before a flag, and no barrier round trip: the read itself waits.
// A copy torn anywhere between the first and the last word shows two
// different tags and is read again.
typedef unsigned int tag_u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCohAux = 16;  // cache-policy operand of the buffer builtins: the sc1 bit

__device__ __forceinline__ __amdgpu_buffer_rsrc_t tag_rsrc(void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ void tag_store(__amdgpu_buffer_rsrc_t r, unsigned slot, unsigned tag, unsigned lo,
                                          unsigned hi) {
  tag_u32x4 v = {tag, lo, hi, tag};
  __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)(slot * 16u), 0, kCohAux);
}
__device__ __forceinline__ tag_u32x4 tag_load(__amdgpu_buffer_rsrc_t r, unsigned slot) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, (int)(slot * 16u), 0, kCohAux);
}
// reload slot until it carries `tag` (bounded; on time-out or abort raises the
// abort flag and returns what it has)
__device__ __forceinline__ tag_u32x4 tag_wait(__amdgpu_buffer_rsrc_t r, unsigned slot, unsigned tag, tag_u32x4 v,
                                              int* abort_flag) {
  unsigned spins = 0;
  while (!(v.x == tag && v.w == tag)) {
    if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > kSpinLimit) {
      __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
    v = tag_load(r, slot);
  }
  return v;
}
__device__ __forceinline__ double tag_double(tag_u32x4 v) {
  return __longlong_as_double((long long)(((unsigned long long)v.z << 32) | v.y));
}
__device__ __forceinline__ void tag_store_double(__amdgpu_buffer_rsrc_t r, unsigned slot, unsigned tag, double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  tag_store(r, slot, tag, (unsigned)u, (unsigned)(u >> 32));
}

// grid_sum over tagged partials (slot pbase + w stride + v of workgroup w, tag
// `tag`), in two stages so that no workgroup reads every partial: value v is
// summed once, in the order of grid_sum, by one wavefront of workgroup v mod W,
// which publishes the total in slot tbase + v (grid_sum_publish); every
// workgroup then reads the nv totals (grid_sum_read).  Each load is repeated
// until its slot carries the tag.  The values of a step are summed before any
// workgroup can publish partials of a later step into the same slots (it
// needs every total of the step in between, whose summing workgroups finish
// this step's sums first).
__device__ void grid_sum_publish(__amdgpu_buffer_rsrc_t rp, unsigned pbase, unsigned tbase, int stride, int nv,
                                 unsigned tag, int* abort_flag) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, NWv = blockDim.x >> 6, W = gridDim.x;
  for (int v = (int)blockIdx.x + W * wave; v < nv; v += W * NWv) {
    double s = 0.0;
    for (int b0 = lane; b0 < W; b0 += 8 * 64) {
      tag_u32x4 p[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (b0 + 64 * u < W) p[u] = tag_load(rp, pbase + (unsigned)((b0 + 64 * u) * stride + v));
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (b0 + 64 * u < W)
          s += tag_double(tag_wait(rp, pbase + (unsigned)((b0 + 64 * u) * stride + v), tag, p[u], abort_flag));
    }
    s = wave_sum(s);
    if (lane == 0) tag_store_double(rp, tbase + (unsigned)v, tag, s);
  }
}
// false when a wait timed out or another workgroup aborted
__device__ bool grid_sum_read(__amdgpu_buffer_rsrc_t rp, unsigned tbase, int nv, unsigned tag, double* out,
                              int* abort_flag) {
  for (int v = threadIdx.x; v < nv; v += blockDim.x)
    out[v] = tag_double(tag_wait(rp, tbase + (unsigned)v, tag, tag_load(rp, tbase + (unsigned)v), abort_flag));
  __syncthreads();
  return __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
}

// block_partial / wave0_partial into tagged slots slot0 + k
template <int NR>
__device__ __forceinline__ void block_partial_tag(double (&v)[NR], __amdgpu_buffer_rsrc_t rp, unsigned slot0,
                                                  unsigned tag, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  wave_sum_n<NR>(v);
#pragma unroll
  for (int k = 0; k < NR; ++k)
    if (lane == 0) sh[k * kPWaves + wave] = v[k];
  __syncthreads();
  if ((int)threadIdx.x < NR) {
    double s = 0.0;
    for (int q = 0; q < kPWaves; ++q) s += sh[threadIdx.x * kPWaves + q];
    tag_store_double(rp, slot0 + threadIdx.x, tag, s);
  }
  __syncthreads();
}
template <int NR>
__device__ __forceinline__ void wave0_partial_tag(double (&v)[NR], __amdgpu_buffer_rsrc_t rp, unsigned slot0,
                                                  unsigned tag) {
  if (threadIdx.x < 64) {
    wave_sum_n<NR>(v);
#pragma unroll
    for (int k = 0; k < NR; ++k)
      if (threadIdx.x == 0) tag_store_double(rp, slot0 + k, tag, v[k]);
  }
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
  unsigned* lflags;  // neighbour-wait lines of the one-site kernel, one per workgroup
  double tol;
  int Vh, n, restart, maxiter, fixed, stride;
  int trust;  // a cycle that met the tolerance by its recurrence residual ends the solve (no true residual)
  int sbytes;   // one-site kernel: LDS bytes before the Krylov basis
  int pl;       // one-site kernel: hop matrix column rounds staged in LDS
  int res_off;  // one-site kernel: LDS byte offset of the even site's resident hop blocks (-1: none)
  int res_ms;   // column stride (elements) of the resident copy: padded so that the eight columns
                // a wavefront reads at once fall into different LDS banks
  void* tags;   // one-site kernel, FP32 vectors: tagged slots, t [V][n], then q [V][n], then the
                // partial sums [2][W][stride] (nullptr: flags and barriers instead)
  unsigned tag_bytes;
};

// Thread layout of the site matrix-vector products (n rows, R2 = n / 2 row
// pairs): a wavefront holds 8 row pairs (lane / 8) x 8 column lanes
// (lane % 8); wavefront w takes row block w % NRB and column wave w / NRB, so
// the column groups are G = 8 CW and a thread owns columns cg, cg + G, ... of
// rows 2 rp, 2 rp + 1.  The 8 column lanes of a row pair are added inside the
// wavefront, the CW column waves through LDS after one barrier.
__host__ __device__ constexpr int mv_row_blocks(int n) { return (n / 2 + 7) / 8; }
__host__ __device__ constexpr int mv_col_waves(int n) { return kPWaves / mv_row_blocks(n); }

struct MvLayout {
  int rp, cg, cw, G, CW;
  bool active;  // the wavefront takes part (wave-uniform)
  bool rows;    // the row pair exists
  bool out;     // the thread returns the result of its row pair
};
__device__ __forceinline__ MvLayout mv_layout(int n, int tid) {
  const int NRB = mv_row_blocks(n), wave = tid >> 6, lane = tid & 63;
  MvLayout L;
  L.CW = mv_col_waves(n);
  L.G = 8 * L.CW;
  L.cw = wave / NRB;
  L.rp = (wave - L.cw * NRB) * 8 + (lane >> 3);
  L.cg = L.cw * 8 + (lane & 7);
  L.active = L.cw < L.CW;
  L.rows = L.rp < (n >> 1);
  L.out = L.active && L.rows && L.cw == 0 && (lane & 7) == 0;
  return L;
}

// Rows of M v for one site (M: n x ncols, column col at M + col * ms; v in
// LDS): true in the threads that hold rows 2 L.rp, 2 L.rp + 1 (o0, o1); every
// thread of the block must call.  part: CW n complex of LDS.
template <typename C, typename V2>
__device__ __forceinline__ bool site_matvec(const V2* M, int ms, const cpx<C>* v, int n, int ncols, cpx<C>* part,
                                            cpx<C>& o0, cpx<C>& o1) {
  const MvLayout L = mv_layout(n, threadIdx.x);
  if (L.active) {
    cpx<C> a0 = mk((C)0, (C)0), a1 = a0;
    if (L.rows) {
      const V2* m = M + 2 * L.rp;
#pragma unroll 8
      for (int col = L.cg; col < ncols; col += L.G) {
        cpx<C> e0, e1;
        ld2(m + (size_t)col * ms, e0, e1);
        const cpx<C> x = v[col];
        cfma(a0, e0, x);
        cfma(a1, e1, x);
      }
    }
    a0 = mk(sum8(a0.r), sum8(a0.i));
    a1 = mk(sum8(a1.r), sum8(a1.i));
    if ((threadIdx.x & 7) == 0 && L.rows) {
      part[L.cw * n + 2 * L.rp] = a0;
      part[L.cw * n + 2 * L.rp + 1] = a1;
    }
  }
  __syncthreads();
  o0 = mk((C)0, (C)0);
  o1 = o0;
  if (L.out) {
    o0 = part[2 * L.rp];
    o1 = part[2 * L.rp + 1];
    for (int q = 1; q < L.CW; ++q) {
      o0 = o0 + part[q * n + 2 * L.rp];
      o1 = o1 + part[q * n + 2 * L.rp + 1];
    }
  }
  return L.out;
}

// out(c) = xd(c) + coeff * sum_d Yt_d(c) in(nb(c, d))     (xd may be null)
// and, with Xl, out(c) = Xl(c) [ ... ] instead; with q, the neighbour values
// are in - alpha q (rounded as the owner rounds them).  MT: storage of the hop
// blocks (the vector type, or __half2 for FP16 blocks with FP32 arithmetic).
template <typename S, typename MT>
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
  const bool own = site_matvec<C, MT>(reinterpret_cast<const MT*>(a.Yt) + (size_t)c * 8 * n * n, n, vin, n, 8 * n,
                                      part, o[0], o[1]);
  const int rp = mv_layout(n, threadIdx.x).rp;
  cpx<C> s[2];
  if (own) {
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
    if (own) {
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
  if (own) {
#pragma unroll
    for (int k = 0; k < 2; ++k) vin[2 * rp + k] = mk((C)(S)s[k].r, (C)(S)s[k].i);
  }
  __syncthreads();
  site_matvec<C, V2>(reinterpret_cast<const V2*>(Xl_) + (size_t)c * n * n, n, vin, n, n, part, o[0], o[1]);
  if (own) {
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
  const bool own = site_matvec<C, V2>(reinterpret_cast<const V2*>(Xl_) + (size_t)c * n * n, n, vin, n, n, part, o[0],
                                      o[1]);
  const int rp = mv_layout(n, threadIdx.x).rp;
  if (own) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      V2 w;
      w.x = (S)o[k].r;
      w.y = (S)o[k].i;
      stc(out + (size_t)c * n + 2 * rp + k, w);
    }
  }
}

template <typename S, typename MT>
__global__ void __launch_bounds__(kPT) k_coarse_gcr(PArgs a) {
  using C = typename Compute<S>::T;
  using V2 = typename Vec2<S>::T;
  extern __shared__ char smem[];  // hop operands, or the slice sums of the Gram-Schmidt step
  cpx<C>* vin = reinterpret_cast<cpx<C>*>(smem);  // 8n
  cpx<C>* hp = vin + 8 * a.n;                     // CW * n (column-wave partials)
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
  for (int i = w; i < Vh; i += W) site_hop<S, MT>(a, i, a.b, a.b, -1.0, nullptr, a.br, vin, hp);
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
    for (int i = w; i < Vh; i += W) site_hop<S, MT>(a, Vh + i, r, nullptr, 1.0, nullptr, a.t, vin, hp);
    for (int idx = threadIdx.x; idx < nel; idx += kPT) {
      const size_t e = el(idx);
      stc(Zv(0) + e, ldc(r + e));
    }
    if (!sync_sum(0)) return;
    int k = 0;
    bool rec_conv = false;  // the cycle met the tolerance by its recurrence residual
    for (;;) {
      V2* Qk = Qv(k);
      V2* Zk = Zv(k);
      V2* Tk = Tv(k);
      // q = D_r z_k = r - Ytilde_eo t; <q_j, q> for j < k, ||q||^2 and <q, r> over the owned sites
      for (int i = w; i < Vh; i += W) site_hop<S, MT>(a, i, a.t, r, -1.0, nullptr, a.qraw, vin, hp);
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
          double p2[2] = {sr, si};
          wave_sum_n<2>(p2);
          sr = p2[0];
          si = p2[1];
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
              aq = aq + cmul(cj, ldo(Qv(j), e));
              az = az + cmul(cj, ldo(Zv(j), e));
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
            std_(y, e, ldd(y, e) + cmul(alpha, zs));
            const cpx<double> rs = axpy_round<S>(ldd(r, e), alpha, qs);
            std_(r, e, rs);
            if (Zn) std_(Zn, e, rs);
            vr[0] += rs.r * rs.r + rs.i * rs.i;
          }
          __syncthreads();
        }
      }
      // odd sites: T_k = Ytilde_oe q_k = Ytilde_oe q - sum_j c_j T_j, and t -= alpha T_k
      for (int i = w; i < Vh; i += W) site_hop<S, MT>(a, Vh + i, a.qraw, nullptr, 1.0, nullptr, Tk, vin, hp);
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
              at = at + cmul(cj, ldo(Tv(j), e));
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
            std_(t, e, ldd(t, e) - cmul(alpha, tks));
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
      if (!a.fixed && sqrt(rn2) <= target) {
        rec_conv = true;
        break;
      }
      if (k >= a.restart || iters >= a.maxiter) break;
    }
    if (status || a.fixed) break;
    if (a.trust && rec_conv) {
      conv = true;
      break;
    }
    // true residual r = b_r - D_r y at the end of the cycle (q_raw as scratch)
    for (int i = w; i < Vh; i += W) site_hop<S, MT>(a, Vh + i, a.y, nullptr, 1.0, nullptr, a.t, vin, hp);
    if (!sync_sum(0)) return;
    for (int i = w; i < Vh; i += W) site_hop<S, MT>(a, i, a.t, a.y, -1.0, nullptr, a.qraw, vin, hp);
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
    site_hop<S, MT>(a, Vh + i, a.y, a.b, -1.0, a.Xinv, a.c, vin, hp);
  }
  if (w == 0 && threadIdx.x == 0) {
    a.info[0] += iters;
    if (status) a.info[1] = status;
  }
}

// ---------------------------------------------------------------------------
// One site per workgroup (grid == Vh): workgroup w owns the even site w and
// the odd site Vh + w.  What only the owner reads stays on chip: the Krylov
// basis (q_j and z_j of the even site, T_j of the odd site) lives in LDS, and
// so do copies of the owned parts of y, r, b_r, t and q, so a step reads from
// memory only the hop matrices and the neighbours' values.  The vectors that
// other workgroups gather are still stored: q and t at every step, y for the
// true residual and the solution, r at the start of a cycle.
//
// The second barrier of a step becomes a neighbour wait: t on an odd site is
// read only by the even sites next to it, so every workgroup publishes an
// epoch on a line of its own and waits for the owners of the eight odd
// neighbours of its even site.  ||r_k||^2 joins the sums of the next step's
// grid barrier, so a cycle ends one even-site hop after the step that
// converged (that hop's result is dropped).  The arithmetic of every vector
// element and of every grid sum is that of the strided kernel above: both
// produce the same bits, and only the grid sum behind the stopping test runs
// in another order.
// ---------------------------------------------------------------------------

// publish epoch on this workgroup's line, then wait until the line of
// workgroup nbw (a distinct neighbour per thread, -1 for none) has reached it
__device__ bool neighbour_wait(unsigned* lines, int* abort_flag, int nbw, unsigned epoch) {
  __shared__ int okl;
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    okl = 1;
    __hip_atomic_store(lines + 32 * blockIdx.x, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (nbw >= 0) {
    unsigned spins = 0;
    while ((int)(__hip_atomic_load(lines + 32 * nbw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - epoch) < 0) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > kSpinLimit) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        okl = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  return okl != 0;
}

template <typename V2>
__device__ __forceinline__ cpx<double> cvt(V2 v) {
  return mk((double)v.x, (double)v.y);
}
template <typename V2>
__device__ __forceinline__ V2 tov2(cpx<double> c) {
  V2 v;
  v.x = c.r;
  v.y = c.i;
  return v;
}

// Hop of the one-site kernel:
//   out(c) = xd(c) + coeff * sum_d Ytilde_d(c) in(nb(c, d))   (then Xl(c) [...])
// thread t < 8n gathers element t % n of its neighbour nb (the t / n-th of c);
// xd is an LDS copy of the site's elements (xdl) or a global field (xdg) or
// absent; the result goes to a global field (outg, coherent stores) and/or an
// LDS copy (outl).  The first a.pl columns of every thread's share of the
// hop matrix go straight to LDS (global_load_lds, no registers) and the next
// few into registers before the gather is issued, so the matrix stream and the
// gather latency overlap; the rest is loaded as in site_matvec, and the sums
// run in its order.  With Mres (the site's hop blocks resident in LDS) every
// column comes from there and nothing is prefetched; the order of the sums is
// the same.  MT: storage of the hop blocks (FP16 blocks are never staged by
// global_load_lds: a.pl is 0 for them).
template <typename S, typename MT>
__device__ void hop1(const PArgs& a, int c, int nb, const typename Vec2<S>::T* in, const typename Vec2<S>::T* xdl,
                     const typename Vec2<S>::T* xdg, double coeff, const void* Xl, typename Vec2<S>::T* outg,
                     typename Vec2<S>::T* outl, cpx<typename Compute<S>::T>* vin,
                     cpx<typename Compute<S>::T>* part, char* pre, const MT* Mres = nullptr, int tin = -1,
                     unsigned tin_tag = 0, int tout = -1, unsigned tout_tag = 0) {
  using C = typename Compute<S>::T;
  using V2 = typename Vec2<S>::T;
  constexpr int NCH = sizeof(S) == 8 ? 2 : 1;  // 16-byte pieces of a thread's two entries of a column
  constexpr bool kStage = sizeof(MT) == sizeof(V2);  // LDS staging exists for blocks in the vector type only
  const int n = a.n, ncols = 8 * n, PL = (kStage && !Mres) ? a.pl : 0;
  // the thread index passes through an empty asm, so that the addresses derived
  // from it are formed here and not kept live across the whole solve (register
  // pressure: the hop is inlined at seven call sites)
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const MvLayout L = mv_layout(n, tid);
  const int G = L.G, lane = tid & 63, wv = tid >> 6, NW = mv_row_blocks(n) * L.CW;
  const bool mine = L.active && L.rows;  // the thread has matrix entries
  const int ms = Mres ? a.res_ms : n;    // column stride of the blocks
  const MT* M = (Mres ? Mres : reinterpret_cast<const MT*>(a.Yt) + (size_t)c * 8 * n * n) + 2 * L.rp;
  __syncthreads();  // the previous task is done with vin, part and the prefetch area
  if (kStage && mine) {
    // piece ch of column round u of wavefront wv: 1 KiB at pre + ((u NCH + ch) NW + wv) KiB, lane order
    for (int u = 0; u < PL; ++u) {
      const int col = L.cg + u * G;
      if (col < ncols) {
        const char* src = reinterpret_cast<const char*>(M + (size_t)col * ms);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
          __builtin_amdgcn_global_load_lds(
              src + 16 * ch,
              (__attribute__((address_space(3))) void*)(pre + ((size_t)((u * NCH + ch) * NW + wv) << 10)), 16, 0,
              0);
      }
    }
  }
  // the next PR rounds into registers, also before the gather (none from LDS)
  constexpr int PR = sizeof(S) == 8 ? 1 : 4;
  const int PRr = Mres ? 0 : PR;
  cpx<C> r0[PR], r1[PR];
  if (mine) {
#pragma unroll
    for (int u = 0; u < PR; ++u) {
      const int col = L.cg + (PL + u) * G;
      if (u < PRr && col < ncols) ld2(M + (size_t)col * ms, r0[u], r1[u]);
    }
  }
  // the gather runs in the wavefronts just below the last one, which never
  // stores: a wavefront's wait for its loads also waits for its earlier
  // coherent stores to complete, and the publishing stores of the solve come
  // from the last wavefront and the first ones
  const int gt = tid - max(0, kPT - 64 - ncols);
  if (gt >= 0 && gt < ncols) {
    if constexpr (sizeof(S) == 4) {
      if (tin >= 0) {
        // tagged input (tin: 0 t, 1 q): each slot is read until it carries tin_tag
        const __amdgpu_buffer_rsrc_t rt = tag_rsrc(a.tags, a.tag_bytes);
        const unsigned slot = (unsigned)(tin * 2 * a.Vh * n + nb * n + (gt - (gt / n) * n));
        const tag_u32x4 q = tag_wait(rt, slot, tin_tag, tag_load(rt, slot), a.info + 2);
        vin[gt] = mk((C)__uint_as_float(q.y), (C)__uint_as_float(q.z));
      } else {
        const V2 v = ldc(in + (size_t)nb * n + (gt - (gt / n) * n));
        vin[gt] = mk((C)v.x, (C)v.y);
      }
    } else {
      const V2 v = ldc(in + (size_t)nb * n + (gt - (gt / n) * n));
      vin[gt] = mk((C)v.x, (C)v.y);
    }
  }
  __syncthreads();
  if (L.active) {
    cpx<C> a0 = mk((C)0, (C)0), a1 = a0;
    if (L.rows) {
      // this thread's own staged pieces: complete once its wavefront's loads have returned
      if (PL > 0) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      for (int u = 0; u < PL; ++u) {
        const int col = L.cg + u * G;
        if (col < ncols) {
          cpx<C> e0, e1;
          const V2* q = reinterpret_cast<const V2*>(pre + ((size_t)(u * NCH * NW + wv) << 10) + 16 * lane);
          if (NCH == 1) {
            ld2(q, e0, e1);
          } else {
            const V2* q1 = reinterpret_cast<const V2*>(pre + ((size_t)((u * NCH + 1) * NW + wv) << 10) + 16 * lane);
            e0 = mk((C)q[0].x, (C)q[0].y);
            e1 = mk((C)q1[0].x, (C)q1[0].y);
          }
          const cpx<C> x = vin[col];
          cfma(a0, e0, x);
          cfma(a1, e1, x);
        }
      }
#pragma unroll
      for (int u = 0; u < PR; ++u) {
        const int col = L.cg + (PL + u) * G;
        if (u < PRr && col < ncols) {
          const cpx<C> x = vin[col];
          cfma(a0, r0[u], x);
          cfma(a1, r1[u], x);
        }
      }
#pragma unroll 8
      for (int col = L.cg + (PL + PRr) * G; col < ncols; col += G) {
        cpx<C> e0, e1;
        ld2(M + (size_t)col * ms, e0, e1);
        const cpx<C> x = vin[col];
        cfma(a0, e0, x);
        cfma(a1, e1, x);
      }
    }
    a0 = mk(sum8(a0.r), sum8(a0.i));
    a1 = mk(sum8(a1.r), sum8(a1.i));
    if ((lane & 7) == 0 && L.rows) {
      part[L.cw * n + 2 * L.rp] = a0;
      part[L.cw * n + 2 * L.rp + 1] = a1;
    }
  }
  __syncthreads();
  const int rp = L.rp;
  cpx<C> s[2];
  if (L.out) {
    cpx<C> o0 = part[2 * rp], o1 = part[2 * rp + 1];
    for (int q = 1; q < L.CW; ++q) {
      o0 = o0 + part[q * n + 2 * rp];
      o1 = o1 + part[q * n + 2 * rp + 1];
    }
    s[0] = (C)coeff * o0;
    s[1] = (C)coeff * o1;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int i = 2 * rp + k;
      if (xdl) s[k] = s[k] + mk((C)xdl[i].x, (C)xdl[i].y);
      if (xdg) {
        const V2 w = ldc(xdg + (size_t)c * n + i);
        s[k] = s[k] + mk((C)w.x, (C)w.y);
      }
    }
  }
  if (Xl) {
    // local matrix on the hop result, staged in vin (rounded to storage precision)
    __syncthreads();
    if (L.out) {
#pragma unroll
      for (int k = 0; k < 2; ++k) vin[2 * rp + k] = mk((C)(S)s[k].r, (C)(S)s[k].i);
    }
    __syncthreads();
    site_matvec<C, V2>(reinterpret_cast<const V2*>(Xl) + (size_t)c * n * n, n, vin, n, n, part, s[0], s[1]);
  }
  if (L.out) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      V2 w;
      w.x = (S)s[k].r;
      w.y = (S)s[k].i;
      if constexpr (sizeof(S) == 4) {
        if (tout >= 0)
          tag_store(tag_rsrc(a.tags, a.tag_bytes), (unsigned)(tout * 2 * a.Vh * n + c * n + 2 * rp + k), tout_tag,
                    __float_as_uint(w.x), __float_as_uint(w.y));
        else if (outg)
          stc(outg + (size_t)c * n + 2 * rp + k, w);
      } else {
        if (outg) stc(outg + (size_t)c * n + 2 * rp + k, w);
      }
      if (outl) outl[2 * rp + k] = w;
    }
  }
}

template <typename S, typename MT>
__global__ void __launch_bounds__(kPT) k_coarse_gcr_site(PArgs a) {
  using C = typename Compute<S>::T;
  using V2 = typename Vec2<S>::T;
  extern __shared__ char smem[];  // hop operands or Gram-Schmidt slice sums, then basis and copies
  const int n = a.n, Vh = a.Vh, R = a.restart, w = blockIdx.x, W = gridDim.x, tid = threadIdx.x;
  cpx<C>* vin = reinterpret_cast<cpx<C>*>(smem);  // 8n
  cpx<C>* hp = vin + 8 * n;                       // CW * n (column-wave partials)
  char* pre = reinterpret_cast<char*>(hp + (size_t)mv_col_waves(n) * n);  // hop matrix columns (a.pl rounds)
  V2* Qs = reinterpret_cast<V2*>(smem + a.sbytes);  // [R][n] q_j (even site)
  V2* Zs = Qs + (size_t)R * n;                      // [R][n] z_j (even site)
  V2* Ts = Zs + (size_t)R * n;                      // [R][n] T_j (odd site)
  V2* ym = Ts + (size_t)R * n;                      // owned elements: y, r, b_r (even), t (odd), q (even)
  V2* rm = ym + n;
  V2* bm = rm + n;
  V2* tm = bm + n;
  V2* qm = tm + n;
  __shared__ double sv[2 * kPMaxRestart + 8];  // grid sums
  __shared__ double sqq[kPMaxRestart];         // ||q_j||^2
  __shared__ double sh[4 * kPWaves];
  __shared__ double salpha[3];
  __shared__ cpx<double> scj[kPMaxRestart];  // Gram-Schmidt coefficients of the step
  __shared__ double spart[2 * kPMaxRestart + 4];  // the step's partial sums, before they are published
  const V2* b = reinterpret_cast<const V2*>(a.b);
  V2* y = reinterpret_cast<V2*>(a.y);
  V2* r = reinterpret_cast<V2*>(a.r);
  V2* t = reinterpret_cast<V2*>(a.t);
  V2* qraw = reinterpret_cast<V2*>(a.qraw);
  const size_t eo = (size_t)w * n, oo = (size_t)(Vh + w) * n;  // owned even / odd elements
  int* abort_flag = a.info + 2;
  // neighbours of the owned sites (for the gathering threads of hop1);
  // owners of the odd neighbours of the even site
  int nbE = 0, nbO = 0, nbw = -1, nbq = -1;
  const int gt = tid - max(0, kPT - 64 - 8 * n);
  const int lane = tid & 63, wave = tid >> 6;
  if (gt >= 0 && gt < 8 * n) {
    nbE = a.nbr[(size_t)w * 8 + gt / n];
    nbO = a.nbr[(size_t)(Vh + w) * 8 + gt / n];
  }
  if (tid < 8) {
    nbw = a.nbr[(size_t)w * 8 + tid] - Vh;
    for (int d = 0; d < tid; ++d)  // wait once per distinct owner
      if (a.nbr[(size_t)w * 8 + d] - Vh == nbw) nbw = -1;
    // owners of the odd site's even neighbours (whose q the odd hop reads)
    nbq = a.nbr[(size_t)(Vh + w) * 8 + tid];
    for (int d = 0; d < tid; ++d)
      if (a.nbr[(size_t)(Vh + w) * 8 + d] == nbq) nbq = -1;
  }
  // the even site's hop blocks, resident in LDS for the whole solve when they fit
  const MT* Mres = nullptr;
  if (a.res_off >= 0) {
    MT* dst = reinterpret_cast<MT*>(smem + a.res_off);
    const MT* src = reinterpret_cast<const MT*>(a.Yt) + (size_t)w * 8 * n * n;
    const int ms = a.res_ms;
    if ((n * sizeof(MT)) % 16 == 0 && (ms * sizeof(MT)) % 16 == 0) {
      // 16-byte pieces: u16 per column
      const int u16 = (int)(n * sizeof(MT) / 16), d16 = (int)(ms * sizeof(MT) / 16);
      for (int i = tid; i < 8 * n * u16; i += kPT) {
        const int col = i / u16, j = i - col * u16;
        reinterpret_cast<uint4*>(dst)[(size_t)col * d16 + j] = reinterpret_cast<const uint4*>(src)[i];
      }
    } else {
      for (int i = tid; i < 8 * n * n; i += kPT) {
        const int col = i / n, j = i - col * n;
        dst[(size_t)col * ms + j] = src[i];
      }
    }
    Mres = dst;
    __syncthreads();
  }
  // epochs continue from what the previous launch left (the same in every line)
  unsigned epoch = __hip_atomic_load(a.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned lep = __hip_atomic_load(a.lflags + 32 * w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int cur = 0;
  auto mine = [&]() { return a.part + ((size_t)cur * W + w) * a.stride; };
  // FP32 vectors with a tag area: t, q and the step's partial sums travel in
  // tagged slots (versions tver, qver, epoch), so a step has no flag wait and
  // no barrier; versions start above anything an earlier launch left
  const bool tagged = sizeof(S) == 4 && a.tags != nullptr;
  unsigned tver = epoch, qver = epoch;
  const unsigned pslot = (unsigned)(4 * Vh * n);              // first partial-sum slot
  const unsigned tslot = pslot + (unsigned)(2 * W * a.stride);  // first total slot
  const __amdgpu_buffer_rsrc_t rtag = tag_rsrc(a.tags, a.tag_bytes);
  auto sync_sum = [&](int nv) -> bool {
    if (!grid_barrier(a.bar, abort_flag, ++epoch)) return false;
    if (nv > 0) grid_sum(a.part + (size_t)cur * W * a.stride, a.stride, nv, sv, sh);
    cur ^= 1;
    return true;
  };

  // b_r = b_e - Ytilde_eo b_o, r = b_r, y = 0, ||b_r||^2
  hop1<S, MT>(a, w, nbE, b, nullptr, b, -1.0, nullptr, nullptr, bm, vin, hp, pre, Mres);
  __syncthreads();
  {
    double v[1] = {0.0};
    if (tid < n) {
      const cpx<double> x = cvt(bm[tid]);
      rm[tid] = bm[tid];
      stc(r + eo + tid, bm[tid]);
      ym[tid] = tov2<V2>(mk(0.0, 0.0));
      stc(y + eo + tid, ym[tid]);
      v[0] += x.r * x.r + x.i * x.i;
    }
    block_partial<1>(v, mine(), sh);
  }
  if (!sync_sum(1)) return;
  const double bn2 = sv[0];
  const double target = a.tol * sqrt(bn2);
  int iters = 0, status = 0;
  bool conv = !(bn2 > 0.0) || (!a.fixed && sqrt(bn2) <= target);
  if (!isfinite(bn2)) {
    status = WCMG_ENAN;
    conv = true;
  }
  while (!conv && iters < a.maxiter) {
    // cycle start: z_0 = r, t = Ytilde_oe r
    if (tagged) ++tver;
    hop1<S, MT>(a, Vh + w, nbO, r, nullptr, nullptr, 1.0, nullptr, t, tm, vin, hp, pre, nullptr, -1, 0,
                tagged ? 0 : -1, tver);
    if (tid < n) Zs[tid] = rm[tid];
    if (!sync_sum(0)) return;
    int k = 0;
    bool rec_conv = false;  // the cycle met the tolerance by its recurrence residual
    for (;;) {
      // q = D_r z_k = r - Ytilde_eo t on the even site (stored for the odd neighbours);
      // <q_j, q>, ||q||^2, <q, r> and ||r_k||^2
      if (tagged) ++qver;
      hop1<S, MT>(a, w, nbE, t, rm, nullptr, -1.0, nullptr, tagged ? nullptr : qraw, qm, vin, hp, pre, Mres,
                  tagged ? 0 : -1, tver);
      __syncthreads();
      const unsigned ep = epoch + 1;  // the step's sum
      const unsigned pbase = pslot + (unsigned)((cur * W + w) * a.stride);
      if (tagged && n <= 64) {
        // the last wavefront publishes q and, once the other wavefronts have
        // left their dot products in LDS, all the step's partial sums
        if (wave == kPWaves - 1) {
          if (lane < n)
            tag_store(rtag, (unsigned)(2 * Vh * n + w * n + lane), qver, __float_as_uint((float)qm[lane].x),
                      __float_as_uint((float)qm[lane].y));
          double v[4] = {0.0, 0.0, 0.0, 0.0};
          if (lane < n) {
            const cpx<double> qv = cvt(qm[lane]), rr = cvt(rm[lane]);
            v[0] += qv.r * qv.r + qv.i * qv.i;
            v[1] += qv.r * rr.r + qv.i * rr.i;
            v[2] += qv.r * rr.i - qv.i * rr.r;
            v[3] += rr.r * rr.r + rr.i * rr.i;
          }
          wave_sum_n<4>(v);
          if (lane == 0) {
#pragma unroll
            for (int m = 0; m < 4; ++m) spart[2 * k + m] = v[m];
          }
        } else {
          for (int j = wave; j < k; j += kPWaves - 1) {
            const V2* Qj = Qs + (size_t)j * n;
            double sr = 0.0, si = 0.0;
            if (lane < n) {
              const cpx<double> u = cvt(Qj[lane]), qv = cvt(qm[lane]);
              sr += u.r * qv.r + u.i * qv.i;
              si += u.r * qv.i - u.i * qv.r;
            }
            double p2[2] = {sr, si};
            wave_sum_n<2>(p2);
            if (lane == 0) {
              spart[2 * j] = p2[0];
              spart[2 * j + 1] = p2[1];
            }
          }
        }
        __syncthreads();
        if (wave == kPWaves - 1)
          for (int l = lane; l < 2 * k + 4; l += 64) tag_store_double(rtag, pbase + l, ep, spart[l]);
      } else {
        if (tagged) {
          // q published by the threads that hold it
          for (int i = tid; i < n; i += kPT)
            tag_store(rtag, (unsigned)(2 * Vh * n + w * n + i), qver, __float_as_uint((float)qm[i].x),
                      __float_as_uint((float)qm[i].y));
        }
        for (int j = wave; j < k; j += kPWaves) {
          const V2* Qj = Qs + (size_t)j * n;
          double sr = 0.0, si = 0.0;
          for (int idx = lane; idx < n; idx += 64) {
            const cpx<double> u = cvt(Qj[idx]), qv = cvt(qm[idx]);
            sr += u.r * qv.r + u.i * qv.i;
            si += u.r * qv.i - u.i * qv.r;
          }
          double p2[2] = {sr, si};
          wave_sum_n<2>(p2);
          sr = p2[0];
          si = p2[1];
          if (lane == 0) {
            if (tagged) {
              tag_store_double(rtag, pbase + 2 * j, ep, sr);
              tag_store_double(rtag, pbase + 2 * j + 1, ep, si);
            } else {
              stc(mine() + 2 * j, sr);
              stc(mine() + 2 * j + 1, si);
            }
          }
        }
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        if (tid < n) {
          const cpx<double> qv = cvt(qm[tid]), rr = cvt(rm[tid]);
          v[0] += qv.r * qv.r + qv.i * qv.i;
          v[1] += qv.r * rr.r + qv.i * rr.i;
          v[2] += qv.r * rr.i - qv.i * rr.r;
          v[3] += rr.r * rr.r + rr.i * rr.i;
        }
        if (tagged) {
          if (n <= 64)
            wave0_partial_tag<4>(v, rtag, pbase + 2 * k, ep);
          else
            block_partial_tag<4>(v, rtag, pbase + 2 * k, ep, sh);
        } else if (n <= 64) {
          wave0_partial<4>(v, mine() + 2 * k);
        } else {
          block_partial<4>(v, mine() + 2 * k, sh);
        }
      }
      // arrive at the step's barrier, then build the odd site's raw hop
      // T_k = Ytilde_oe q while the rest of the grid arrives: it needs only the
      // owners of the odd site's even neighbours (q is overwritten no earlier
      // than their next step, which waits for this workgroup's t), and is
      // unused when the step ends the cycle
      // (tagged: the hop's reads of q and the sum's reads of the partials wait
      // for their versions themselves)
      if (tagged) {
        // the summing workgroups sum right away (their wait for the last
        // partials overlaps the odd hop's wait for q), so that the totals are
        // out when the others finish the odd hop
        epoch = ep;
        grid_sum_publish(rtag, pslot + (unsigned)(cur * W * a.stride), tslot + (unsigned)(cur * a.stride), a.stride,
                         2 * k + 4, ep, abort_flag);
        hop1<S, MT>(a, Vh + w, nbO, qraw, nullptr, nullptr, 1.0, nullptr, nullptr, Ts + (size_t)k * n, vin, hp, pre,
                    nullptr, 1, qver);
        __syncthreads();
        if (!grid_sum_read(rtag, tslot + (unsigned)(cur * a.stride), 2 * k + 4, ep, sv, abort_flag)) return;
      } else {
        barrier_arrive(a.bar, ++epoch);
        if (!arrival_wait(a.bar, abort_flag, nbq, epoch)) return;
        hop1<S, MT>(a, Vh + w, nbO, qraw, nullptr, nullptr, 1.0, nullptr, nullptr, Ts + (size_t)k * n, vin, hp,
                    pre);
        if (!barrier_complete(a.bar, abort_flag, epoch)) return;
        grid_sum(a.part + (size_t)cur * W * a.stride, a.stride, 2 * k + 4, sv, sh);
      }
      cur ^= 1;
      if (k > 0) {  // r_k, the residual after the previous step
        const double rn2 = sv[2 * k + 3];
        if (!isfinite(rn2)) {
          status = WCMG_ENAN;
          break;
        }
        if (!a.fixed && sqrt(rn2) <= target) {
          rec_conv = true;
          break;
        }
      }
      // wavefront 0, lane j < k: c_j = <q_j, q> / ||q_j||^2 and |<q_j, q>|^2 / ||q_j||^2
      // (the same divisions as the strided kernel, done once instead of per
      // thread); then ||q_k||^2 = ||q||^2 - those terms, subtracted in order of j
      // from the lanes' registers (a zero term for ||q_j||^2 <= 0 leaves it as is)
      if (tid < 64) {
        double st = 0.0;
        if (tid < k) {
          const double d = sqq[tid];
          scj[tid] = d > 0.0 ? mk(sv[2 * tid] / d, sv[2 * tid + 1] / d) : mk(0.0, 0.0);
          st = d > 0.0 ? (sv[2 * tid] * sv[2 * tid] + sv[2 * tid + 1] * sv[2 * tid + 1]) / d : 0.0;
        }
        double qq = sv[2 * k];
        for (int j = 0; j < k; ++j) qq -= rdlane(st, j);
        if (tid == 0) {
          salpha[2] = qq;
          salpha[0] = qq > 0.0 ? sv[2 * k + 1] / qq : 0.0;
          salpha[1] = qq > 0.0 ? sv[2 * k + 2] / qq : 0.0;
        }
      }
      __syncthreads();
      const double qq = salpha[2];
      if (!(qq > 0.0) || !isfinite(qq)) {
        status = isfinite(qq) ? WCMG_EBREAKDOWN : WCMG_ENAN;
        break;
      }
      const cpx<double> alpha = mk(salpha[0], salpha[1]);
      const int NS = k > 0 ? max(1, min(kPT / n, k)) : 1;
      const int sl = tid / n, idx = tid - sl * n;
      cpx<double>* acc = reinterpret_cast<cpx<double>*>(smem);  // [2][kPT]
      // q_k, z_k by classical Gram-Schmidt (slices of j, added in slice order);
      // y += alpha z_k, r -= alpha q_k, z_{k+1} = r
      if (k > 0 && sl < NS) {
        cpx<double> aq = mk(0.0, 0.0), az = aq;
        for (int j = sl; j < k; j += NS) {
          const cpx<double> cj = scj[j];
          aq = aq + cmul(cj, cvt(Qs[(size_t)j * n + idx]));
          az = az + cmul(cj, cvt(Zs[(size_t)j * n + idx]));
        }
        acc[tid] = aq;
        acc[kPT + tid] = az;
      }
      __syncthreads();
      if (tid < n) {
        cpx<double> q = cvt(qm[tid]), z = cvt(Zs[(size_t)k * n + tid]);
        if (k > 0) {
          cpx<double> sq = acc[tid], sz = acc[kPT + tid];
          for (int u = 1; u < NS; ++u) {
            sq = sq + acc[u * n + tid];
            sz = sz + acc[kPT + u * n + tid];
          }
          q = q - sq;
          z = z - sz;
        }
        const cpx<double> qs = mk((double)(S)q.r, (double)(S)q.i), zs = mk((double)(S)z.r, (double)(S)z.i);
        Qs[(size_t)k * n + tid] = tov2<V2>(qs);
        Zs[(size_t)k * n + tid] = tov2<V2>(zs);
        ym[tid] = tov2<V2>(cvt(ym[tid]) + cmul(alpha, zs));  // to global memory at the end of the cycle
        const V2 rv = tov2<V2>(axpy_round<S>(cvt(rm[tid]), alpha, qs));
        rm[tid] = rv;
        if (k + 1 < R) Zs[(size_t)(k + 1) * n + tid] = rv;
      }
      // odd site: T_k = Ytilde_oe q - sum_j c_j T_j, t -= alpha T_k (the raw hop
      // is in Ts[k]; the barrier keeps the slice sums of q and z read above apart
      // from the slice sums of T written into the same LDS below)
      __syncthreads();
      if (k > 0 && sl < NS) {
        cpx<double> at = mk(0.0, 0.0);
        for (int j = sl; j < k; j += NS) {
          const cpx<double> cj = scj[j];
          at = at + cmul(cj, cvt(Ts[(size_t)j * n + idx]));
        }
        acc[tid] = at;
      }
      __syncthreads();
      if (tagged) ++tver;
      // (in the last wavefront, which publishes t)
      for (int i = tid - (kPT - 64); i >= 0 && i < n; i += 64) {
        cpx<double> tk = cvt(Ts[(size_t)k * n + i]);
        if (k > 0) {
          cpx<double> st = acc[i];
          for (int u = 1; u < NS; ++u) st = st + acc[u * n + i];
          tk = tk - st;
        }
        const cpx<double> tks = mk((double)(S)tk.r, (double)(S)tk.i);
        Ts[(size_t)k * n + i] = tov2<V2>(tks);
        const V2 tv = tov2<V2>(cvt(tm[i]) - cmul(alpha, tks));
        tm[i] = tv;
        if (tagged)
          tag_store(rtag, (unsigned)(oo + i), tver, __float_as_uint((float)tv.x), __float_as_uint((float)tv.y));
        else
          stc(t + oo + i, tv);
      }
      if (tid == 0) sqq[k] = qq;
      ++k;
      ++iters;
      if (k >= R || iters >= a.maxiter) break;
      // t of the owned odd site is published; the next even hop reads the neighbours' t
      // (tagged: that read waits for the version itself)
      if (!tagged && !neighbour_wait(a.lflags, abort_flag, nbw, ++lep)) return;
    }
    // y and t complete everywhere
    if (tid < n) stc(y + eo + tid, ym[tid]);
    if (!sync_sum(0)) return;
    if (status || a.fixed) break;
    if (a.trust && rec_conv) {
      conv = true;
      break;
    }
    // true residual r = b_r - D_r y at the end of the cycle
    if (tagged) ++tver;
    hop1<S, MT>(a, Vh + w, nbO, y, nullptr, nullptr, 1.0, nullptr, t, tm, vin, hp, pre, nullptr, -1, 0,
                tagged ? 0 : -1, tver);
    if (!sync_sum(0)) return;
    hop1<S, MT>(a, w, nbE, t, ym, nullptr, -1.0, nullptr, nullptr, qm, vin, hp, pre, Mres, tagged ? 0 : -1, tver);
    __syncthreads();
    {
      double v[1] = {0.0};
      if (tid < n) {
        const V2 rv = tov2<V2>(cvt(bm[tid]) - cvt(qm[tid]));
        rm[tid] = rv;
        stc(r + eo + tid, rv);
        const cpx<double> rs = cvt(rv);
        v[0] += rs.r * rs.r + rs.i * rs.i;
      }
      block_partial<1>(v, mine(), sh);
    }
    if (!sync_sum(1)) return;
    const double rn2 = sv[0];
    if (!isfinite(rn2)) {
      status = WCMG_ENAN;
      break;
    }
    if (sqrt(rn2) <= target) conv = true;
  }
  // c_e = X_ee^-1 y,  c_o = X_oo^-1 (b_o - Ytilde_oe y)   (y is complete after the last grid barrier)
  site_local<S>(a, w, a.y, a.Xinv, a.c, vin, hp);
  hop1<S, MT>(a, Vh + w, nbO, y, nullptr, b, -1.0, a.Xinv, reinterpret_cast<V2*>(a.c), nullptr, vin, hp, pre);
  if (w == 0 && tid == 0) {
    a.info[0] += iters;
    if (status) a.info[1] = status;
  }
}

}  // namespace

size_t coarse_gcr_persistent_part_doubles() { return 2 * kPMaxRestart + 8; }

size_t coarse_gcr_persistent_tag_bytes(int n, int Vh, int grid) {
  // t and q over all sites, then two buffers of partial sums per workgroup and
  // two of totals
  return ((size_t)4 * Vh * n + (size_t)2 * (grid + 1) * coarse_gcr_persistent_part_doubles()) * 16;
}

// column groups of the site matrix-vector products (eight per column wave)
static int persist_groups(int n) { return 8 * mv_col_waves(n); }

// column stride of the resident hop blocks: the first at least n whose byte
// length is 16 modulo 32, so that the eight columns a wavefront reads at once
// (at consecutive column indices) start in different LDS banks
static int resident_stride(int n, size_t elem) {
  int ms = n;
  while ((ms * elem) % 32 != 16) ++ms;
  return ms;
}

int coarse_gcr_persistent_grid(int prec, int n, int Vh) {
  int dev = 0, ncu = 0, coop = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  if (!coop || n % 2 || n > 256 || Vh <= 0) return 0;
  const size_t cb = prec == WCMG_F64 ? 16 : 8;
  const size_t shm = std::max((size_t)(8 * n + mv_col_waves(n) * n) * cb, (size_t)2 * kPT * 16);
  int per = 0;
  if (prec == WCMG_F64)
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_coarse_gcr<double, double2>, kPT, shm));
  else
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_coarse_gcr<float, float2>, kPT, shm));
  if (per < 1) return 0;
  return std::min(std::min(ncu, Vh), 256);
}

// whether one workgroup of kernel k with `bytes` of dynamic LDS fits a compute unit
static bool kernel_fits(const void* k, size_t bytes) {
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, kPT, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return per >= 1;
}

void launch_coarse_gcr_persistent(int prec, const CoarseGcrArgs& g, hipStream_t st) {
  const int n = g.n;
  if (n % 2 || n > 256) fail(WCMG_EDIM, "coarse block size must be even and <= 256");
  if (g.restart < 1 || g.restart > kPMaxRestart) fail(WCMG_EINVAL, "coarse restart length out of range");
  if (g.grid < 1 || g.grid > 256) fail(WCMG_EINVAL, "persistent coarse solve needs 1..256 workgroups");
  if (g.mat16 && prec != WCMG_F32) fail(WCMG_EINVAL, "FP16 hop blocks go with FP32 vectors");
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
  a.trust = g.trust;
  a.stride = (int)coarse_gcr_persistent_part_doubles();
  a.res_off = -1;
  a.tags = nullptr;
  a.tag_bytes = 0;
  const int G = persist_groups(n);
  const size_t cb = prec == WCMG_F64 ? 16 : 8;
  const size_t shm = std::max((size_t)(8 * n + mv_col_waves(n) * n) * cb, (size_t)2 * kPT * 16);
  a.lflags = reinterpret_cast<unsigned*>(reinterpret_cast<char*>(g.bar) + kPersistLocalOffset);
  a.sbytes = (int)shm;
  void* args[] = {&a};
  // one site per workgroup: vin, the column-group partials and as many rounds of
  // hop matrix columns as fit, overlapped by the Gram-Schmidt slice sums; then
  // the basis [3][restart][n] and five site copies.  FP16 hop blocks: no staged
  // rounds; instead the even site's 8 n^2 blocks stay in LDS for the whole solve
  // when they fit.
  const size_t basis = (size_t)(3 * g.restart + 5) * n * cb;
  const size_t hopb = (size_t)(8 * n + mv_col_waves(n) * n) * cb;
  const size_t round = (prec == WCMG_F64 ? 2 : 1) * (size_t)(mv_row_blocks(n) * mv_col_waves(n)) * 1024;
  const size_t lds_cap = 160 * 1024 - 4096;  // minus the kernel's static LDS, with margin
  const int rounds = (8 * n + G - 1) / G;
  int pl = 0;
  if (!g.mat16 && lds_cap > basis + hopb) pl = (int)std::min<size_t>(rounds, (lds_cap - basis - hopb) / round);
  const size_t sb = std::max(hopb + (size_t)pl * round, (size_t)2 * kPT * 16);
  const int ms = resident_stride(n, 4);
  const size_t res = g.mat16 ? (size_t)8 * n * ms * 4 : 0;
  const bool resident = g.mat16 && sb + basis + res <= lds_cap;
  const size_t site_shm = sb + basis + (resident ? res : 0);
  const void* ks = prec == WCMG_F64 ? reinterpret_cast<const void*>(k_coarse_gcr_site<double, double2>)
                   : g.mat16      ? reinterpret_cast<const void*>(k_coarse_gcr_site<float, __half2>)
                                  : reinterpret_cast<const void*>(k_coarse_gcr_site<float, float2>);
  if (!g.general && g.grid == g.Vh && 8 * n <= kPT && site_shm <= lds_cap && kernel_fits(ks, site_shm)) {
    a.sbytes = (int)sb;
    a.pl = pl;
    if (resident) {
      a.res_off = (int)(sb + basis);
      a.res_ms = ms;
    }
    // FP32 vectors: t, q and the step sums in tagged slots (no flag waits or barriers per step)
    if (prec == WCMG_F32 && g.tags && g.tag_bytes >= coarse_gcr_persistent_tag_bytes(n, g.Vh, g.grid) &&
        g.tag_bytes < ((size_t)1 << 31)) {
      a.tags = g.tags;
      a.tag_bytes = (unsigned)g.tag_bytes;
    }
    HIPCHK(hipLaunchCooperativeKernel(ks, dim3(g.grid), dim3(kPT), args, (unsigned)site_shm, st));
    return;
  }
  const void* kg = prec == WCMG_F64 ? reinterpret_cast<const void*>(k_coarse_gcr<double, double2>)
                   : g.mat16      ? reinterpret_cast<const void*>(k_coarse_gcr<float, __half2>)
                                  : reinterpret_cast<const void*>(k_coarse_gcr<float, float2>);
  HIPCHK(hipLaunchCooperativeKernel(kg, dim3(g.grid), dim3(kPT), args, (unsigned)shm, st));
}

}  // namespace wcmg
