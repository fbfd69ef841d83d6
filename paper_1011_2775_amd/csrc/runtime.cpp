// Host runtime: errors, buffers, timers, reductions, and the operator
// wrappers that sequence the kernels of the fine and coarse levels.
#include "runtime.h"

#include <cmath>
#include <cstring>

namespace wcmg {

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e == hipSuccess) return;
  std::string m = std::string(what) + ": " + hipGetErrorString(e) + " (" + file + ":" + std::to_string(line) + ")";
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) fail(WCMG_ENOMEM, m);
  if (e == hipErrorNoDevice || e == hipErrorInvalidDevice) fail(WCMG_ENODEV, m);
  fail(WCMG_EHIP, m);
}

void DBuf::alloc(size_t bytes) {
  if (bytes == n && p) return;
  release();
  if (bytes) HIPCHK(hipMalloc(&p, bytes));
  n = bytes;
}
void DBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  n = 0;
}

Geom make_geom(const int dims[4], int t_bc) {
  Geom g;
  long v = 1;
  for (int k = 0; k < 4; ++k) {
    g.L[k] = dims[k];
    v *= dims[k];
  }
  g.V = (int)v;
  g.Vh = (int)(v / 2);
  g.Lxh = dims[0] / 2;
  g.t_bc = (double)t_bc;
  return g;
}

BlockGeom make_block_geom(const int L[4], const int b[4]) {
  BlockGeom bg{};
  bg.Vc = 1;
  bg.bvol = 1;
  bool even = true;
  for (int k = 0; k < 4; ++k) {
    bg.b[k] = b[k];
    bg.nb[k] = L[k] / b[k];
    bg.Vc *= bg.nb[k];
    bg.bvol *= b[k];
    even = even && (bg.nb[k] % 2 == 0);
  }
  bg.coarse_cb = even ? 1 : 0;
  return bg;
}

CoarseGeom make_coarse_geom(const BlockGeom& bg, int nvec) {
  CoarseGeom cg{};
  for (int k = 0; k < 4; ++k) cg.L[k] = bg.nb[k];
  cg.V = bg.Vc;
  cg.split = bg.coarse_cb;
  cg.Vh = cg.split ? cg.V / 2 : cg.V;
  cg.n = 2 * nvec;
  return cg;
}

// ------------------------------------------------------------------ timers
hipEvent_t KernelTimer::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  return e;
}
void KernelTimer::begin(int cls, hipEvent_t* a) {
  if (only_persistent && (cls < 28 || cls > 30)) {
    *a = nullptr;  // the caller then records no end either
    return;
  }
  *a = get();
  HIPCHK(hipEventRecord(*a, st));
}
void KernelTimer::end(int cls, hipEvent_t a) {
  hipEvent_t b = get();
  HIPCHK(hipEventRecord(b, st));
  pending.push_back({cls, {a, b}});
}
void KernelTimer::drain() {
  if (pending.empty()) return;
  HIPCHK(hipStreamSynchronize(st));
  for (auto& pe : pending) {
    float ms_ = 0.f;
    HIPCHK(hipEventElapsedTime(&ms_, pe.second.first, pe.second.second));
    count[pe.first] += 1;
    ms[pe.first] += ms_;
    pool.push_back(pe.second.first);
    pool.push_back(pe.second.second);
  }
  pending.clear();
}
void KernelTimer::reset() {
  drain();
  for (int k = 0; k < kIds; ++k) count[k] = 0;
  for (int k = 0; k < kIds; ++k) ms[k] = 0.0;
}
KernelTimer::~KernelTimer() {
  for (auto& pe : pending) {
    (void)hipEventDestroy(pe.second.first);
    (void)hipEventDestroy(pe.second.second);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

// ------------------------------------------------------------------ reducer
void Reducer::init(hipStream_t s) {
  st = s;
  partial.alloc((size_t)kRedBlocks * 64 * sizeof(double));
  res.alloc(256 * sizeof(double));
  counter.alloc(256);
  HIPCHK(hipMemset(counter.p, 0, 256));
  HIPCHK(hipHostMalloc((void**)&host, 256 * sizeof(double), hipHostMallocDefault));
  HIPCHK(hipHostMalloc((void**)&host2, 16 * sizeof(double), hipHostMallocDefault));
  for (auto& e : ev2) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  part_b.alloc((size_t)kMaxBatch * kRedBlocks * 32 * sizeof(double));
}
const double* Reducer::fetch_rows(const double* dev, size_t pitch, int width, int rows) {
  if (width * rows > 256) fail(WCMG_EINVAL, "too many scalars for the host staging buffer");
  HIPCHK(hipMemcpy2DAsync(host, (size_t)width * sizeof(double), dev, pitch * sizeof(double),
                          (size_t)width * sizeof(double), rows, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return host;
}
// The copy is ordered after the reduction on the stream; values written by a
// kernel straight into host-mapped memory were not reliably visible to the
// host at stream synchronisation, so results always come back this way.
const double* Reducer::fetch_from(const double* dev, int n) {
  HIPCHK(hipMemcpyAsync(host, dev, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return host;
}
void Reducer::fetch_async(const double* dev, int n, int slot) {
  if (n > 8 || slot < 0 || slot > 1) fail(WCMG_EINVAL, "asynchronous fetch: at most 8 scalars in slot 0 or 1");
  HIPCHK(hipMemcpyAsync(host2 + 8 * slot, dev, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipEventRecord(ev2[slot], st));
}
const double* Reducer::fetch_wait(int slot) {
  HIPCHK(hipEventSynchronize(ev2[slot]));
  return host2 + 8 * slot;
}
Reducer::~Reducer() {
  for (auto& e : ev2)
    if (e) (void)hipEventDestroy(e);
  if (host2) (void)hipHostFree(host2);
  if (host) (void)hipHostFree(host);
}

double norm2(Ctx& c, int prec, const void* x, size_t n) {
  blas_norm2(prec, x, n, c.red.out(), c.st);
  return c.red.fetch(1)[0];
}

void* Ctx::scratch_buf(int slot, size_t bytes) {
  if ((int)scratch.size() <= slot) scratch.resize(slot + 1);
  if (scratch[slot].n < bytes) scratch[slot].alloc(bytes);
  return scratch[slot].p;
}

// ------------------------------------------------------------------ fine level
void FineWork::ensure(int p, const Geom& g, int nrhs) {
  size_t b = spinor_bytes(p, g.Vh) * (size_t)nrhs;
  if (prec == p && hb >= b) return;
  prec = p;
  hb = b;
  t1.alloc(b);
  t2.alloc(b);
  t3.alloc(b);
}

void FineOp::hop(void* out, const void* in, const void* x, int parity, int diag, bool postinv, double coeff,
                 int nrhs) {
  DslashArgs a;
  a.out = out;
  a.in = in;
  a.x = x;
  a.gauge = F->gauge[fp()].p;
  a.clov = F->clov[fp()].p;
  a.fprec = fp();
  a.g = dgeom(F->g);
  a.parity = parity;
  a.nblocks = 0;
  a.coeff = coeff;
  a.nrhs = nrhs;
  a.rstride = hb();
  if (ctx->tuner.on) {
    const std::array<int, 5> key{prec * 3 + fp(), diag, postinv ? 1 : 0, F->g.Vh, nrhs};
    auto it = ctx->tuner.best.find(key);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHK(hipStreamIsCapturing(st, &cs));
    if (it == ctx->tuner.best.end() && cs == hipStreamCaptureStatusNone) {
      // time every candidate shape on this very launch (the kernel only writes `out`)
      Tuner::Choice bestc{256, 0, 1e30};
      hipEvent_t e0, e1;
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      const int max_g = prec == WCMG_F64 ? 2 : 4;
      for (int threads : {64, 128, 256})
        for (int group : {-1, 1, 2, 4}) {
          if (group > max_g || (group > 1 && group > nrhs) || (group < 0 && nrhs == 1)) continue;
          DslashArgs t = a;
          t.threads = threads;
          t.group = group;
          launch_dslash(prec, diag, postinv, t, st);
          HIPCHK(hipEventRecord(e0, st));
          for (int rep = 0; rep < 3; ++rep) launch_dslash(prec, diag, postinv, t, st);
          HIPCHK(hipEventRecord(e1, st));
          HIPCHK(hipEventSynchronize(e1));
          float ms = 0.f;
          HIPCHK(hipEventElapsedTime(&ms, e0, e1));
          const double us = ms * 1e3 / 3.0;
          if (us < bestc.us) bestc = Tuner::Choice{threads, group, us};
        }
      HIPCHK(hipEventDestroy(e0));
      HIPCHK(hipEventDestroy(e1));
      it = ctx->tuner.best.emplace(key, bestc).first;
    }
    if (it != ctx->tuner.best.end()) {
      a.threads = it->second.threads;
      a.group = it->second.group;
    }
  }
  // timer id: precision x DIAG mode x clover-inverse post-multiply; batched launches
  // from 32, FP32 spinors with FP16 fields from 56
  const int id = fp() != prec ? 56 + diag * 2 + (postinv ? 1 : 0)
                              : (nrhs > 1 ? 32 : 0) + prec * 6 + diag * 2 + (postinv ? 1 : 0);
  hipEvent_t e = nullptr;
  if (ctx->timer.on) ctx->timer.begin(id, &e);
  launch_dslash(prec, diag, postinv, a, st);
  if (e) ctx->timer.end(id, e);
}

void FineOp::clover(void* out, const void* in, int parity, int kind, int nrhs) {
  // timer ids: one right-hand side 64 + precision, batches 67 + precision, FP16 fields
  // with FP32 spinors 70
  const int id = fp() != prec ? 70 : (nrhs > 1 ? 67 : 64) + prec;
  hipEvent_t e = nullptr;
  if (ctx->timer.on) ctx->timer.begin(id, &e);
  launch_clover(prec, out, in, F->clov[fp()].p, F->g.Vh, parity, kind, st, nrhs, hb(), fp());
  if (e) ctx->timer.end(id, e);
}

void FineOp::Dr(void* out, const void* y, int nrhs) {
  w->ensure(prec, F->g, nrhs);
  clover(w->t1.p, y, 0, 1, nrhs);                          // z = A_ee^-1 y
  hop(w->t2.p, w->t1.p, nullptr, 1, 0, true, 1.0, nrhs);   // w = A_oo^-1 H_oe z
  hop(out, w->t2.p, y, 0, 1, false, -1.0, nrhs);           // out = y - H_eo w
}

bool FineOp::Dr_red(void* out, void* y, const RedOut& o, void* e, const double* coef) {
  DslashArgs a;
  a.out = out;
  a.x = y;
  a.gauge = F->gauge[fp()].p;
  a.clov = F->clov[fp()].p;
  a.fprec = fp();
  a.g = dgeom(F->g);
  a.parity = 0;
  a.coeff = -1.0;
  a.nrhs = 1;
  a.rstride = hb();
  const bool pair_ok = (prec == WCMG_F64 && fp() == WCMG_F64) ||
                       (prec == WCMG_F32 && (fp() == WCMG_F32 || fp() == WCMG_F16));
  if (!pair_ok) return false;
  if ((size_t)xcd_grid((F->g.Vh + 255) / 256) * 3 > (size_t)kRedBlocks * 64) return false;
  w->ensure(prec, F->g, 1);
  a.in = w->t2.p;
  if (e) {
    // e += a y, y -= a out, z = A_ee^-1 y (timer 72 + spinor precision)
    hipEvent_t ev0 = nullptr;
    if (ctx->timer.on) ctx->timer.begin(72 + prec, &ev0);
    if (!launch_clover_mr(prec, w->t1.p, y, e, out, coef, F->clov[fp()].p, F->g.Vh, 0, fp(), st))
      fail(WCMG_EINVAL, "fused smoother update rejected after its checks passed");
    if (ev0) ctx->timer.end(72 + prec, ev0);
  } else {
    clover(w->t1.p, y, 0, 1, 1);  // z = A_ee^-1 y
  }
  hop(w->t2.p, w->t1.p, nullptr, 1, 0, true, 1.0, 1);  // w = A_oo^-1 H_oe z
  const int id = fp() != prec ? 56 + 2 : prec * 6 + 2;  // the DIAG = 1 hop's timer
  hipEvent_t ev = nullptr;
  if (ctx->timer.on) ctx->timer.begin(id, &ev);
  const bool ok = launch_dslash_red(prec, a, o, st);  // out = y - H_eo w, and the sums
  if (ev) ctx->timer.end(id, ev);
  if (!ok) fail(WCMG_EINVAL, "fused smoother hop rejected after its checks passed");
  return true;
}

void FineOp::Mx(void* out, const void* x, int nrhs) {
  w->ensure(prec, F->g, nrhs);
  hop(w->t2.p, x, nullptr, 1, 0, true, 1.0, nrhs);  // w = A_oo^-1 H_oe x
  hop(out, w->t2.p, x, 0, 2, false, -1.0, nrhs);    // out = A_ee x - H_eo w
}

void FineOp::Dr_dag(void* out, const void* y, int nrhs) {
  // D_r^dag = gamma5 (1 - A_ee^-1 H_eo A_oo^-1 H_oe) gamma5
  w->ensure(prec, F->g, nrhs);
  const size_t h = hb();
  for (int r = 0; r < nrhs; ++r) {
    spinor_convert(prec, (char*)w->t1.p + r * h, prec, (const char*)y + r * h, F->g.Vh, st);
    spinor_gamma5(prec, (char*)w->t1.p + r * h, F->g.Vh, st);
  }
  hop(w->t2.p, w->t1.p, nullptr, 1, 0, true, 1.0, nrhs);
  hop(out, w->t2.p, w->t1.p, 0, 1, true, -1.0, nrhs);
  for (int r = 0; r < nrhs; ++r) spinor_gamma5(prec, (char*)out + r * h, F->g.Vh, st);
}

void FineOp::D(void* oe, void* oo, const void* ie, const void* io, int nrhs) {
  hop(oe, io, ie, 0, 2, false, 1.0, nrhs);
  hop(oo, ie, io, 1, 2, false, 1.0, nrhs);
}

void FineOp::Dp(void* oe, void* oo, const void* ie, const void* io, int nrhs) {
  w->ensure(prec, F->g, nrhs);
  clover(w->t1.p, ie, 0, 1, nrhs);
  clover(w->t2.p, io, 1, 1, nrhs);
  hop(oe, w->t2.p, ie, 0, 1, false, 1.0, nrhs);
  hop(oo, w->t1.p, io, 1, 1, false, 1.0, nrhs);
}

void FineOp::reduced_source(void* br, const void* be, const void* bo, int nrhs) {
  w->ensure(prec, F->g, nrhs);
  clover(w->t1.p, bo, 1, 1, nrhs);
  hop(br, w->t1.p, be, 0, 1, false, -1.0, nrhs);
}

void FineOp::reconstruct(void* xe, void* xo, const void* ye, const void* bo, int nrhs) {
  w->ensure(prec, F->g, nrhs);
  clover(xe, ye, 0, 1, nrhs);
  hop(w->t1.p, xe, bo, 1, 1, false, -1.0, nrhs);
  clover(xo, w->t1.p, 1, 1, nrhs);
}

// ------------------------------------------------------------------ coarse level
void CoarseWork::ensure(size_t bytes) {
  if (t1.n < bytes) {
    t1.alloc(bytes);
    t2.alloc(bytes);
  }
}

void CoarseOp::Dfull(void* out, const void* in, int nrhs) {
  launch_coarse_hop(prec, out, in, in, C->Yhop[pi()].p, C->X[pi()].p, 2, 1.0, -1, C->cg, C->nbr.as<int>(), st, nrhs,
                    nall());
}

void CoarseOp::Dp(void* out, const void* in, int nrhs) {
  launch_coarse_hop(prec, out, in, in, C->Yt[pi()].p, nullptr, 1, 1.0, -1, C->cg, C->nbr.as<int>(), st, nrhs, nall());
}

void CoarseOp::Dr(void* out, const void* y, int nrhs) {
  w->ensure(nall() * csize() * nrhs);
  if (prec == WCMG_F32 && nrhs >= 2 && C->has_frag) {
    // batches run on the matrix cores (FP16 operands, FP32 accumulation)
    const int id = timer_base + 30;  // 50 (level 1), 52 (level 2), 126 (level 3)
    hipEvent_t e = nullptr;
    if (timer && timer->on) timer->begin(id, &e);
    launch_coarse_hop_mfma(w->t1.p, y, nullptr, C->frag.p, 1.0, 1, C->cg, C->nbr.as<int>(), nrhs, nall(), st);
    launch_coarse_hop_mfma(out, w->t1.p, y, C->frag.p, -1.0, 0, C->cg, C->nbr.as<int>(), nrhs, nall(), st);
    if (e) timer->end(id, e);
    return;
  }
  // single right-hand side: timer_base + precision; batches: timer_base + 4 + precision
  const int id = timer_base + pi() + (nrhs > 1 ? 4 : 0);
  hipEvent_t e = nullptr;
  if (timer && timer->on) timer->begin(id, &e);
  launch_coarse_hop(prec, w->t1.p, y, nullptr, C->Yt[pi()].p, nullptr, 0, 1.0, 1, C->cg, C->nbr.as<int>(), st, nrhs,
                    nall(), true);
  if (e) timer->end(id, e);
  e = nullptr;
  if (timer && timer->on) timer->begin(id, &e);
  launch_coarse_hop(prec, out, w->t1.p, y, C->Yt[pi()].p, nullptr, 1, -1.0, 0, C->cg, C->nbr.as<int>(), st, nrhs,
                    nall(), true);
  if (e) timer->end(id, e);
}

void CoarseOp::reduced_source(void* br, const void* b, int nrhs) {
  launch_coarse_hop(prec, br, b, b, C->Yt[pi()].p, nullptr, 1, -1.0, 0, C->cg, C->nbr.as<int>(), st, nrhs, nall());
}

void CoarseOp::reconstruct(void* c, const void* y, const void* b, int nrhs) {
  w->ensure(nall() * csize() * nrhs);
  launch_coarse_local(prec, c, y, C->Xinv[pi()].p, 0, C->cg, st, nrhs, nall());
  launch_coarse_hop(prec, w->t1.p, y, b, C->Yt[pi()].p, nullptr, 1, -1.0, 1, C->cg, C->nbr.as<int>(), st, nrhs,
                    nall());
  launch_coarse_local(prec, c, w->t1.p, C->Xinv[pi()].p, 1, C->cg, st, nrhs, nall());
}

}  // namespace wcmg
