// Solvers: flexible GCR, BiCGStab, the multigrid setup (Setup procedure
// section), the coarse-operator construction Yhat = R D_p P and the
// recursive GCR cycle (Implementation paragraph).
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>

#include "random.h"
#include "herm_eig.h"
#include "runtime.h"

namespace wcmg {

void GcrSpace::ensure(int restart) {
  if ((int)Z.size() < restart) {
    Z.resize(restart);
    Q.resize(restart);
  }
  for (int k = 0; k < restart; ++k) {
    if (Z[k].n < bytes) Z[k].alloc(bytes);
    if (Q[k].n < bytes) Q[k].alloc(bytes);
  }
  if (r.n < bytes) r.alloc(bytes);
  // beta, qa, the orthogonalisation coefficients [slot][slot] (complex) and the
  // solution-update coefficients of a cycle
  if (!scal.p)
    scal.alloc((2 * (kMaxRestart + 16) + 4 * kMaxRestart + 2 * kMaxRestart * kMaxRestart + 2 * kMaxRestart) *
               sizeof(double));
}

static bool finite(double v) { return std::isfinite(v); }

// WCMG_LOG=0..3 selects progress messages on stderr (0: none)
static int log_level() {
  static int lvl = [] {
    const char* e = std::getenv("WCMG_LOG");
    return e ? std::atoi(e) : 0;
  }();
  return lvl;
}

// Flexible GCR with classical Gram-Schmidt against the unnormalised basis
// q_j = A z_j, residual update r -= alpha q, and the solution update
// x += sum alpha_j z_j deferred to the end of each restart cycle.
KrylovResult gcr(Ctx& c, GcrSpace& S, const OpFn& A, const OpFn* K, void* x, const void* b, bool x_zero, double tol,
                 double target_norm, int restart, int maxiter, bool fixed, const GcrDeflation* defl) {
  const int nf = defl ? defl->K() : 0;  // fixed pairs at the head of the basis
  if (nf + restart > kMaxRestart) fail(WCMG_EINVAL, "deflation vectors plus restart length exceed 64");
  S.ensure(restart);
  const int prec = S.prec;
  const size_t n = S.n;
  hipStream_t st = c.st;
  Reducer& R = c.red;
  void* r = S.r.p;
  KrylovResult res;
  if (x_zero) {
    blas_zero(prec, x, n, st);
    blas_copy(prec, r, b, n, st);
  } else {
    A(r, x);
    blas_axpby(prec, 1.0, 0.0, b, -1.0, 0.0, r, n, st);
  }
  // fixed-length runs never read a scalar back (they can be captured into a graph)
  double rn2 = fixed ? 0.0 : norm2(c, prec, r, n);
  const double target = tol * target_norm;
  if (!finite(rn2)) {
    res.status = WCMG_ENAN;
    return res;
  }
  if (!fixed && std::sqrt(rn2) <= target) {
    res.rel_res = target_norm > 0 ? std::sqrt(rn2) / target_norm : 0.0;
    return res;
  }
  // device scalars: beta (multi-dot results) and per-step {||q||^2, <q,r>, ||r||^2};
  // slots 0..nf-1 belong to the fixed pairs (alpha 0: r is orthogonal to them)
  // the directions are kept as the raw preconditioned vectors z_j (only q_j =
  // A z~_j is orthogonalised); cmat holds the orthogonalisation coefficients,
  // from which the solution update of a cycle is recovered
  double* beta = S.scal.as<double>();
  double* qa = beta + 2 * (kMaxRestart + 16);
  double* cmat = qa + 4 * kMaxRestart;
  double* ycoef = cmat + 2 * kMaxRestart * kMaxRestart;
  std::vector<const void*> Qp(nf + restart), Zp(nf + restart), Dp(nf + restart + 2);
  for (int j = 0; j < nf; ++j) {
    Qp[j] = defl->Q[j];
    Zp[j] = defl->Z[j];
  }
  if (nf) blas_copy(WCMG_F64, qa, defl->qa, (size_t)2 * nf, st);
  // one step of the cycle: z_k = K r, q_k = A z_k, then <q_j, q> for the
  // basis, <q, q> and <r, q> in one pass and one pass that orthogonalises q
  // and updates r
  auto enqueue_step = [&](int k) {
    void* z = S.Z[k].p;
    void* q = S.Q[k].p;
    const int kk = nf + k;  // basis slot of this step
    Qp[kk] = q;
    Zp[kk] = z;
    if (K)
      (*K)(z, r);
    else
      blas_copy(prec, z, r, n, st);
    A(q, z);
    for (int j = 0; j < kk; ++j) Dp[j] = Qp[j];
    Dp[kk] = q;
    Dp[kk + 1] = r;
    blas_multi_cdot(prec, Dp.data(), kk + 2, q, n, R.out(beta), st);
    blas_gcr_step_dev(prec, Qp.data(), kk, q, r, n, beta, qa, cmat + (size_t)2 * kMaxRestart * kk,
                      R.out(qa + 4 * kk + 3), st);
  };
  // The top-level solve reads each step's scalars back asynchronously and,
  // while the residual is still far from the target, queues the next step
  // before that read completes, so that the device does not wait for the
  // host.  A queued step that turns out not to be needed only writes the next
  // basis slot and r, which the cycle end recomputes from x.
  const bool pipelined = !fixed && &S == &c.outer;
  double rn_prev = std::sqrt(rn2), ratio = 0.5;
  bool converged = false;
  while (res.iters < maxiter) {
    int k = 0;
    bool queued = false;  // step k already queued (with its scalars' copy into slot qslot)
    int qslot = 0;
    for (; k < restart;) {
      const int kk = nf + k;
      if (!queued) {
        enqueue_step(k);
        if (pipelined) R.fetch_async(qa + 4 * kk, 4, k & 1);
      }
      queued = false;
      if (fixed) {
        ++k;
        ++res.iters;
        if (res.iters >= maxiter) break;
        continue;
      }
      if (pipelined && k + 1 < restart && res.iters + 1 < maxiter && rn_prev * ratio * 0.25 > target) {
        enqueue_step(k + 1);
        qslot = (k + 1) & 1;
        R.fetch_async(qa + 4 * (kk + 1), 4, qslot);
        queued = true;
      }
      // {||q||^2, <q,r>, ||r||^2} of step k
      const double* o = pipelined ? R.fetch_wait(k & 1) : R.fetch_from(qa + 4 * kk, 4);
      const double qq = o[0];
      rn2 = o[3];
      if (log_level() >= 3 && n > 100000)
        std::fprintf(stderr, "[wcmg] gcr n=%zu iter %d rel.res %.3e\n", n, res.iters + 1,
                     target_norm > 0 ? std::sqrt(rn2) / target_norm : 0.0);
      if (!(qq > 0.0) || !finite(qq)) {
        res.status = finite(qq) ? WCMG_EBREAKDOWN : WCMG_ENAN;
        break;
      }
      ++k;
      ++res.iters;
      if (!finite(rn2)) {
        res.status = WCMG_ENAN;
        break;
      }
      if ((!fixed && std::sqrt(rn2) <= target) || res.iters >= maxiter) break;
      if (rn_prev > 0.0) ratio = std::min(1.0, std::sqrt(rn2) / rn_prev);
      rn_prev = std::sqrt(rn2);
    }
    if (queued) {
      // the step queued past the end of this run: its scalars' copy must be
      // complete before the slot is reused
      (void)R.fetch_wait(qslot);
    }
    if (k > 0) blas_gcr_update_x_raw(prec, Zp.data(), nf, nf + k, x, n, qa, cmat, kMaxRestart, ycoef, st);
    if (res.status != WCMG_OK) break;
    if (fixed) break;
    // true residual at the end of every cycle
    A(r, x);
    blas_axpby(prec, 1.0, 0.0, b, -1.0, 0.0, r, n, st);
    rn2 = norm2(c, prec, r, n);
    if (!finite(rn2)) {
      res.status = WCMG_ENAN;
      break;
    }
    if (std::sqrt(rn2) <= target) {
      converged = true;
      break;
    }
    rn_prev = std::sqrt(rn2);
  }
  res.rel_res = target_norm > 0 ? std::sqrt(rn2) / target_norm : 0.0;
  if (!fixed && !converged && res.status == WCMG_OK) res.status = WCMG_ENOCONV;
  if (log_level() >= 3 && n <= 100000)
    std::fprintf(stderr, "[wcmg] gcr n=%zu done: %d iterations, rel.res %.3e, status %d\n", n, res.iters,
                 res.rel_res, res.status);
  return res;
}

// BiCGStab (van der Vorst); s is formed in place of r.
// ---------------------------------------------------------------------------
// lockstep flexible GCR over a batch of right-hand sides: every step applies
// K and A to the whole batch in one pass; orthogonalisation and updates use
// per-right-hand-side coefficients held on the device (one host read of the
// nrhs x {||q||^2, <q,r>, ||r||^2} per step).  A right-hand side that has
// reached its tolerance keeps taking steps (its corrections are tiny) until
// the whole batch has converged.
// ---------------------------------------------------------------------------
void GcrSpaceB::ensure(int restart) {
  const size_t b = bytes();
  if ((int)Z.size() < restart) {
    Z.resize(restart);
    Q.resize(restart);
  }
  for (int k = 0; k < restart; ++k) {
    if (Z[k].n < b) Z[k].alloc(b);
    if (Q[k].n < b) Q[k].alloc(b);
  }
  if (r.n < b) r.alloc(b);
  const size_t sb = (size_t)kMaxBatch * kGcrCoefs * sizeof(double);
  if (scal.n < sb) scal.alloc(sb);
  const size_t cb = (size_t)kMaxBatch * (2 * kMaxRestart * kMaxRestart + 2 * kMaxRestart) * sizeof(double);
  if (cm.n < cb) cm.alloc(cb);
}

std::vector<KrylovResult> gcr_b(Ctx& c, GcrSpaceB& S, const OpFn& A, const OpFn* K, void* x, const void* b,
                                bool x_zero, double tol, const double* target_norm, int restart, int maxiter,
                                bool fixed) {
  const int nr = S.nrhs;
  if (nr < 1 || nr > kMaxBatch) fail(WCMG_EINVAL, "batch size out of range");
  S.ensure(restart);
  const int prec = S.prec;
  const size_t n = S.n, vs = S.vs;
  const size_t es = prec == WCMG_F64 ? 16 : 8;
  hipStream_t st = c.st;
  Reducer& R = c.red;
  void* r = S.r.p;
  std::vector<KrylovResult> res(nr);
  auto each = [&](auto&& f) {
    for (int i = 0; i < nr; ++i) f(i, (size_t)i * vs * es);
  };
  if (x_zero) {
    each([&](int, size_t o) {
      blas_zero(prec, (char*)x + o, n, st);
      blas_copy(prec, (char*)r + o, (const char*)b + o, n, st);
    });
  } else {
    A(r, x);
    each([&](int, size_t o) { blas_axpby(prec, 1.0, 0.0, (const char*)b + o, -1.0, 0.0, (char*)r + o, n, st); });
  }
  std::vector<double> rn2(nr), target(nr);
  std::vector<char> done(nr, 0), conv(nr, 0);
  if (!fixed) {
    blas_norm2_b(prec, r, vs, n, nr, R.outb(R.dres(), 1), st);
    const double* h = R.fetch(nr);
    for (int i = 0; i < nr; ++i) rn2[i] = h[i];
  }
  bool all = true;
  for (int i = 0; i < nr; ++i) {
    target[i] = tol * target_norm[i];
    if (!finite(rn2[i])) {
      res[i].status = WCMG_ENAN;
      done[i] = 1;
    } else if (std::sqrt(rn2[i]) <= target[i]) {
      done[i] = conv[i] = 1;
    }
    all = all && done[i];
  }
  double* cbase = S.scal.as<double>();
  double* beta = cbase;
  double* qa = cbase + 2 * (kMaxRestart + 16);
  const size_t cs = kGcrCoefs;
  // directions kept raw, as in gcr(): per right-hand side the orthogonalisation
  // coefficients [slot][slot] and then the cycle's update coefficients
  double* cmb = S.cm.as<double>();
  const size_t cms = 2 * kMaxRestart * kMaxRestart + 2 * kMaxRestart;
  std::vector<const void*> Qp(restart), Zp(restart), Dp(restart + 2);
  int iters = 0;
  if (!(all && !fixed)) {
    while (iters < maxiter) {
      int k = 0;
      bool stop = false;
      for (; k < restart;) {
        void* z = S.Z[k].p;
        void* q = S.Q[k].p;
        Qp[k] = q;
        Zp[k] = z;
        if (K)
          (*K)(z, r);
        else
          each([&](int, size_t o) { blas_copy(prec, (char*)z + o, (const char*)r + o, n, st); });
        A(q, z);
        for (int j = 0; j < k; ++j) Dp[j] = Qp[j];
        Dp[k] = q;
        Dp[k + 1] = r;
        blas_multi_cdot_b(prec, Dp.data(), k + 2, q, vs, n, nr, R.outb(beta, cs), st);
        blas_gcr_step_b(prec, Qp.data(), k, q, r, vs, n, nr, beta, cs, qa, cs, cmb + (size_t)2 * kMaxRestart * k, cms,
                        R.outb(qa + 4 * k + 3, cs), st);
        ++k;
        ++iters;
        if (fixed) {
          for (int i = 0; i < nr; ++i) res[i].iters = iters;
          if (iters >= maxiter) {
            stop = true;
            break;
          }
          continue;
        }
        const double* o = R.fetch_rows(qa + 4 * k - 4, cs, 4, nr);
        all = true;
        for (int i = 0; i < nr; ++i) {
          const double qq = o[4 * i];
          rn2[i] = o[4 * i + 3];
          if (!done[i]) {
            res[i].iters = iters;
            if (!finite(qq) || !finite(rn2[i])) {
              res[i].status = WCMG_ENAN;
              done[i] = 1;
            } else if (!(qq > 0.0)) {
              res[i].status = WCMG_EBREAKDOWN;
              done[i] = 1;
            } else if (!fixed && std::sqrt(rn2[i]) <= target[i]) {
              done[i] = 1;
            }
          }
          all = all && done[i];
        }
        if ((!fixed && all) || iters >= maxiter) {
          stop = true;
          break;
        }
      }
      if (k > 0)
        blas_gcr_update_x_raw_b(prec, Zp.data(), k, x, vs, n, nr, qa, cs, cmb, cms, kMaxRestart,
                                cmb + (size_t)2 * kMaxRestart * kMaxRestart, cms, st);
      if (fixed) break;
      // true residuals at the end of every cycle
      A(r, x);
      each([&](int, size_t o) { blas_axpby(prec, 1.0, 0.0, (const char*)b + o, -1.0, 0.0, (char*)r + o, n, st); });
      blas_norm2_b(prec, r, vs, n, nr, R.outb(R.dres(), 1), st);
      const double* h = R.fetch(nr);
      all = true;
      for (int i = 0; i < nr; ++i) {
        rn2[i] = h[i];
        if (res[i].status == WCMG_OK) {
          conv[i] = finite(rn2[i]) && std::sqrt(rn2[i]) <= target[i];
          done[i] = conv[i];
        }
        all = all && (done[i] || res[i].status != WCMG_OK);
      }
      if (all) break;
      (void)stop;
    }
  }
  for (int i = 0; i < nr; ++i) {
    res[i].rel_res = target_norm[i] > 0 ? std::sqrt(rn2[i]) / target_norm[i] : 0.0;
    if (!fixed && !conv[i] && res[i].status == WCMG_OK) res[i].status = WCMG_ENOCONV;
  }
  return res;
}

// relative size of <rhat, r> or <rhat, A p> below which BiCGStab restarts
// (exact breakdown only: restarting on near-breakdown made the iteration
// diverge on operators whose spectrum surrounds the origin)
constexpr double kBicgBreakdown = 1e-30;
constexpr int kBicgMaxRestarts = 1000;

KrylovResult bicgstab(Ctx& c, int prec, size_t n, const OpFn& A, void* x, const void* b, double tol,
                      double target_norm, int maxiter) {
  const size_t bytes = n * (prec == WCMG_F64 ? 16 : 8);
  void* r = c.scratch_buf(4, bytes);
  void* rhat = c.scratch_buf(5, bytes);
  void* p = c.scratch_buf(6, bytes);
  void* v = c.scratch_buf(7, bytes);
  void* t = c.scratch_buf(8, bytes);
  hipStream_t st = c.st;
  Reducer& R = c.red;
  KrylovResult res;
  const double target = tol * target_norm;
  int restarts = 0;
  double rhat_n = 0.0;
  auto start = [&]() -> double {
    A(r, x);
    blas_axpby(prec, 1.0, 0.0, b, -1.0, 0.0, r, n, st);
    blas_copy(prec, rhat, r, n, st);
    blas_zero(prec, p, n, st);
    blas_zero(prec, v, n, st);
    double r2 = norm2(c, prec, r, n);
    rhat_n = std::sqrt(r2);
    return r2;
  };
  double rn2 = start();
  double rho_r = 1.0, rho_i = 0.0, al_r = 1.0, al_i = 0.0, om_r = 1.0, om_i = 0.0;
  double rn_r = rn2, rn_i = 0.0;  // <rhat, r>
  auto cdiv = [](double ar, double ai, double br, double bi, double& cr, double& ci) {
    double d = br * br + bi * bi;
    cr = (ar * br + ai * bi) / d;
    ci = (ai * br - ar * bi) / d;
  };
  auto cmul = [](double ar, double ai, double br, double bi, double& cr, double& ci) {
    cr = ar * br - ai * bi;
    ci = ar * bi + ai * br;
  };
  int verifications = 0;
  for (;;) {
    if (!finite(rn2)) {
      res.status = WCMG_ENAN;
      break;
    }
    if (std::sqrt(rn2) <= target) {
      // the recursive residual drifts from b - A x over long runs: confirm with
      // the true residual and continue from the current iterate if needed
      const double tr2 = start();
      if (std::sqrt(tr2) <= target || ++verifications > 50) {
        rn2 = tr2;
        break;
      }
      rn2 = tr2;
      rho_r = al_r = om_r = 1.0;
      rho_i = al_i = om_i = 0.0;
      rn_r = rn2;
      rn_i = 0.0;
    }
    if (res.iters >= maxiter) break;
    if (log_level() >= 2 && res.iters % 1000 == 0)
      std::fprintf(stderr, "[wcmg] bicgstab iter %d rel.res %.3e restarts %d checks %d\n", res.iters,
                   std::sqrt(rn2) / target_norm, restarts, verifications);
    double t1r, t1i, t2r, t2i, br, bi;
    cdiv(rn_r, rn_i, rho_r, rho_i, t1r, t1i);
    cdiv(al_r, al_i, om_r, om_i, t2r, t2i);
    cmul(t1r, t1i, t2r, t2i, br, bi);
    blas_bicg_p(prec, br, bi, om_r, om_i, r, v, p, n, st);
    A(v, p);
    blas_cdot(prec, rhat, v, n, R.out(), st);
    const double* d = R.fetch(2);
    double rv_r = d[0], rv_i = d[1];
    const double scale = std::sqrt(rn2) * rhat_n;
    if (std::hypot(rv_r, rv_i) <= kBicgBreakdown * scale || std::hypot(rn_r, rn_i) <= kBicgBreakdown * scale) {
      // breakdown: restart from the current iterate with a fresh shadow residual
      if (++restarts > kBicgMaxRestarts) {
        res.status = WCMG_EBREAKDOWN;
        break;
      }
      rn2 = start();
      rho_r = al_r = om_r = 1.0;
      rho_i = al_i = om_i = 0.0;
      rn_r = rn2;
      rn_i = 0.0;
      continue;
    }
    cdiv(rn_r, rn_i, rv_r, rv_i, al_r, al_i);
    blas_axpby(prec, -al_r, -al_i, v, 1.0, 0.0, r, n, st);  // r <- s = r - alpha v
    A(t, r);
    blas_cdot_norm(prec, t, r, n, R.out(), st);
    d = R.fetch(3);
    if (!(d[2] > 0.0)) {
      // s = 0: x += alpha p solves the system
      blas_axpby(prec, al_r, al_i, p, 1.0, 0.0, x, n, st);
      rn2 = norm2(c, prec, r, n);
      ++res.iters;
      break;
    }
    om_r = d[0] / d[2];
    om_i = d[1] / d[2];
    rho_r = rn_r;
    rho_i = rn_i;
    blas_bicg_update(prec, al_r, al_i, om_r, om_i, p, r, t, x, r, rhat, n, R.out(), st);
    d = R.fetch(3);
    rn2 = d[0];
    rn_r = d[1];
    rn_i = d[2];
    ++res.iters;
  }
  res.rel_res = target_norm > 0 ? std::sqrt(rn2) / target_norm : 0.0;
  if (res.status == WCMG_OK && std::sqrt(rn2) > target) res.status = WCMG_ENOCONV;
  return res;
}

// ---------------------------------------------------------------------------
// the paper's comparison solvers on the reduced system D_r y = b_r
// ---------------------------------------------------------------------------
// Mixed-precision BiCGStab by iterative refinement (the Implementation
// paragraph compares the multigrid solver with a BiCGStab whose work runs in
// single precision inside double-precision restarts): the residual
// r = b_r - D_r y is formed in FP64, an FP32 BiCGStab solves D_r e = r from
// zero to a relative inner_tol, and y += e in FP64, until the FP64 residual
// meets tol * target_norm.  res.iters counts FP32 BiCGStab iterations (two
// D_r applies each); *cycles the refinement cycles.
KrylovResult mp_bicgstab(Ctx& c, LatticeState& L, void* y, const void* b, bool y_zero, double tol,
                         double target_norm, int maxiter, double inner_tol, int* cycles) {
  hipStream_t st = c.st;
  const Geom& g = L.F.g;
  const size_t n = (size_t)12 * g.Vh;
  FineOp op64{&c, &L.F, WCMG_F64, &c.fw[0], st};
  FineOp op32{&c, &L.F, WCMG_F32, &c.fw[1], st};
  void* r = c.scratch_buf(33, spinor_bytes(WCMG_F64, g.Vh));
  void* e = c.scratch_buf(34, spinor_bytes(WCMG_F64, g.Vh));
  void* r32 = c.scratch_buf(35, spinor_bytes(WCMG_F32, g.Vh));
  void* e32 = c.scratch_buf(36, spinor_bytes(WCMG_F32, g.Vh));
  void* y_prev = c.scratch_buf(37, spinor_bytes(WCMG_F64, g.Vh));
  OpFn A32 = [&](void* o, const void* i) { op32.Dr(o, i); };
  if (y_zero) blas_zero(WCMG_F64, y, n, st);
  KrylovResult res;
  const double target = tol * target_norm;
  int ncyc = 0, first_iters = 0;
  double prev = std::numeric_limits<double>::infinity();
  for (;;) {
    op64.Dr(r, y);
    blas_axpby(WCMG_F64, 1.0, 0.0, b, -1.0, 0.0, r, n, st);  // r = b - D_r y
    const double rn = std::sqrt(norm2(c, WCMG_F64, r, n));
    res.rel_res = target_norm > 0 ? rn / target_norm : 0.0;
    if (!finite(rn)) {
      res.status = WCMG_ENAN;
      break;
    }
    if (rn <= target) break;
    if (res.iters >= maxiter || !(rn < prev)) {  // out of iterations, or a cycle that did not help
      res.status = WCMG_ENOCONV;
      break;
    }
    prev = rn;
    spinor_convert(WCMG_F32, r32, WCMG_F64, r, g.Vh, st);  // spinor layouts differ per precision
    blas_zero(WCMG_F32, e32, n, st);
    // the inner solve stops at inner_tol, or at the outer target if that is looser
    const double itol = std::max(inner_tol, 0.5 * target / rn);
    // the first cycle gets an eighth of the budget, later ones at most three times
    // the first one's iterations (an FP32 solve that stagnates near the critical
    // mass would otherwise spend the whole budget in one cycle); a capped cycle's
    // correction is still taken when it lowers the FP64 residual
    const int left = maxiter - res.iters;
    const int cap = std::min(left, std::max(1000, ncyc == 0 ? maxiter / 8 : 3 * first_iters));
    KrylovResult k = bicgstab(c, WCMG_F32, n, A32, e32, r32, std::min(itol, 0.5), rn, cap);
    if (ncyc == 0) first_iters = k.iters;
    res.iters += k.iters;
    ++ncyc;
    if (k.status == WCMG_ENAN) {
      res.status = WCMG_ENAN;
      break;
    }
    spinor_convert(WCMG_F64, e, WCMG_F32, e32, g.Vh, st);
    blas_copy(WCMG_F64, y_prev, y, n, st);
    blas_axpby(WCMG_F64, 1.0, 0.0, e, 1.0, 0.0, y, n, st);  // y += e
    // a correction that does not lower the FP64 residual (an FP32 solve that
    // diverged) is taken back exactly (from the copy: subtracting a huge e again
    // would not restore y), and the refinement stops there
    op64.Dr(r, y);
    blas_axpby(WCMG_F64, 1.0, 0.0, b, -1.0, 0.0, r, n, st);
    const double rn_new = std::sqrt(norm2(c, WCMG_F64, r, n));
    if (!(rn_new < rn)) {
      blas_copy(WCMG_F64, y, y_prev, n, st);
      res.rel_res = target_norm > 0 ? rn / target_norm : 0.0;
      res.status = WCMG_ENOCONV;
      break;
    }
  }
  if (cycles) *cycles = ncyc;
  return res;
}

// CGNR: conjugate gradients on the normal equations D_r^dag D_r y = D_r^dag b,
// tracking the residual r = b - D_r y of the reduced system itself (the
// other classical Krylov baseline of the Introduction's comparison); FP64.
// Each iteration applies D_r and D_r^dag once.
KrylovResult cgnr(Ctx& c, LatticeState& L, void* y, const void* b, bool y_zero, double tol, double target_norm,
                  int maxiter) {
  hipStream_t st = c.st;
  const Geom& g = L.F.g;
  const size_t n = (size_t)12 * g.Vh;
  const size_t hb = spinor_bytes(WCMG_F64, g.Vh);
  FineOp op{&c, &L.F, WCMG_F64, &c.fw[0], st};
  void* r = c.scratch_buf(33, hb);
  void* z = c.scratch_buf(34, hb);
  void* p = c.scratch_buf(37, hb);
  void* w = c.scratch_buf(38, hb);
  Reducer& R = c.red;
  KrylovResult res;
  const double target = tol * target_norm;
  if (y_zero) blas_zero(WCMG_F64, y, n, st);
  auto restart = [&]() -> double {
    op.Dr(r, y);
    blas_axpby(WCMG_F64, 1.0, 0.0, b, -1.0, 0.0, r, n, st);  // r = b - D_r y
    op.Dr_dag(z, r);
    blas_copy(WCMG_F64, p, z, n, st);
    return norm2(c, WCMG_F64, z, n);
  };
  double zz = restart();
  double rn = std::sqrt(norm2(c, WCMG_F64, r, n));
  int verifications = 0;
  for (;;) {
    res.rel_res = target_norm > 0 ? rn / target_norm : 0.0;
    if (!finite(rn) || !finite(zz)) {
      res.status = WCMG_ENAN;
      break;
    }
    if (rn <= target) {
      // confirm with the true residual (the recursion drifts over long runs)
      zz = restart();
      rn = std::sqrt(norm2(c, WCMG_F64, r, n));
      if (rn <= target || ++verifications > 50) {
        res.rel_res = target_norm > 0 ? rn / target_norm : 0.0;
        if (rn > target) res.status = WCMG_ENOCONV;
        break;
      }
      continue;
    }
    if (res.iters >= maxiter) {
      res.status = WCMG_ENOCONV;
      break;
    }
    if (!(zz > 0.0)) {
      res.status = WCMG_EBREAKDOWN;
      break;
    }
    op.Dr(w, p);
    const double ww = norm2(c, WCMG_F64, w, n);
    if (!(ww > 0.0)) {
      res.status = WCMG_EBREAKDOWN;
      break;
    }
    const double alpha = zz / ww;
    blas_axpby(WCMG_F64, alpha, 0.0, p, 1.0, 0.0, y, n, st);  // y += alpha p
    blas_axpy_norm(WCMG_F64, -alpha, 0.0, w, r, n, R.out(), st);  // r -= alpha w
    rn = std::sqrt(R.fetch(1)[0]);
    op.Dr_dag(z, r);
    const double zz_new = norm2(c, WCMG_F64, z, n);
    blas_axpby(WCMG_F64, 1.0, 0.0, z, zz_new / zz, 0.0, p, n, st);  // p = z + beta p
    zz = zz_new;
    ++res.iters;
  }
  return res;
}

// ---------------------------------------------------------------------------
// coarse red-black GCR in one cooperative launch
// ---------------------------------------------------------------------------
bool persistent_available(PersistWork& w, int prec, const CoarseLevel& C, int restart) {
  if (!C.cg.split || restart < 1 || restart > kMaxRestart) return false;
  if (w.grid < 0) w.grid = coarse_gcr_persistent_grid(prec, C.cg.n, C.cg.Vh);
  return w.grid > 0;
}

void persistent_launch_bufs(Ctx& c, int grid, const PersistBufs& B, CoarseLevel& C, int prec, void* out,
                            const void* in, void* t, void* y, void* r, void* br, double tol, int restart,
                            int maxiter, bool fixed, bool general, bool mat16, bool trust) {
  CoarseGcrArgs a{};
  const int pi = prec == WCMG_F64 ? 0 : 1;
  if (mat16 && (prec != WCMG_F32 || !C.Yt16.p)) fail(WCMG_EINVAL, "FP16 hop blocks need FP32 vectors");
  a.Yt = mat16 ? C.Yt16.p : C.Yt[pi].p;
  a.mat16 = mat16 ? 1 : 0;
  a.Xinv = C.Xinv[pi].p;
  a.nbr = C.nbr.as<int>();
  a.b = in;
  a.c = out;
  a.t = t;
  a.y = y;
  a.r = r;
  a.br = br;
  a.Q = B.Q;
  a.Z = B.Z;
  a.T = B.T;
  a.qraw = B.qraw;
  a.part = B.part;
  a.bar = reinterpret_cast<unsigned*>(B.ctl);
  a.info = reinterpret_cast<int*>(reinterpret_cast<char*>(B.ctl) + kPersistInfoOffset);
  a.tol = tol;
  a.Vh = C.cg.Vh;
  a.n = C.cg.n;
  a.restart = restart;
  a.maxiter = maxiter;
  a.fixed = fixed ? 1 : 0;
  a.grid = grid;
  a.general = general ? 1 : 0;
  a.trust = trust ? 1 : 0;
  a.tags = B.tags;
  a.tag_bytes = B.tag_bytes;
  launch_coarse_gcr_persistent(prec, a, c.st);
}

void persistent_launch(Ctx& c, PersistWork& w, CoarseLevel& C, int prec, void* out, const void* in, void* t, void* y,
                       void* r, void* br, double tol, int restart, int maxiter, bool fixed, bool general,
                       bool mat16, bool trust) {
  const size_t cs = prec == WCMG_F64 ? 16 : 8;
  const size_t hv = (size_t)C.cg.Vh * C.cg.n;
  restart = std::min(restart, std::max(1, maxiter));
  w.q.alloc((size_t)restart * hv * cs);
  w.z.alloc((size_t)restart * hv * cs);
  w.t.alloc((size_t)restart * 2 * hv * cs);
  w.qraw.alloc(hv * cs);
  const size_t tb = coarse_gcr_persistent_tag_bytes(C.cg.n, C.cg.Vh, w.grid);
  if (!w.ctl.p || w.tags.n < tb) {
    // the barrier epochs restart from zero together with every tag
    w.part.alloc(2 * (size_t)w.grid * coarse_gcr_persistent_part_doubles() * sizeof(double));
    w.ctl.alloc(kPersistCtlBytes);
    w.tags.alloc(tb);
    HIPCHK(hipMemsetAsync(w.ctl.p, 0, kPersistCtlBytes, c.st));
    HIPCHK(hipMemsetAsync(w.tags.p, 0, w.tags.n, c.st));
  }
  PersistBufs B{w.q.p, w.z.p, w.t.p, w.qraw.p, w.part.as<double>(), w.ctl.p, w.tags.p, tb};
  persistent_launch_bufs(c, w.grid, B, C, prec, out, in, t, y, r, br, tol, restart, maxiter, fixed, general, mat16,
                         trust);
  w.pending = true;
}

// Carving plan of the allocation-free coarse solve: every buffer 256-byte
// aligned, in this order; with base == nullptr only the size is computed.
namespace {
struct Carve {
  char* base;
  size_t used = 0;
  void* take(size_t b) {
    used = (used + 255) & ~(size_t)255;
    void* p = base ? base + used : nullptr;
    used += b;
    return p;
  }
};
struct NoAllocPlan {
  void *vb, *vx, *t, *y, *r, *br;
  PersistBufs B;
};
NoAllocPlan plan_noalloc(Carve& k, const CoarseLevel& C, int prec, int restart, int grid) {
  const size_t cs = prec == WCMG_F64 ? 16 : 8;
  const size_t nall = (size_t)C.cg.V * C.cg.n, hv = (size_t)C.cg.Vh * C.cg.n;
  NoAllocPlan P{};
  P.B.ctl = k.take(kPersistCtlBytes);  // first: the control block is cleared at every call
  P.B.part = reinterpret_cast<double*>(k.take(2 * (size_t)grid * coarse_gcr_persistent_part_doubles() * 8));
  P.vb = k.take(nall * cs);
  P.vx = k.take(nall * cs);
  P.t = k.take(nall * cs);
  P.y = k.take(nall * cs);
  P.r = k.take(nall * cs);
  P.br = k.take(nall * cs);
  P.B.Q = k.take((size_t)restart * hv * cs);
  P.B.Z = k.take((size_t)restart * hv * cs);
  P.B.T = k.take((size_t)restart * 2 * hv * cs);
  P.B.qraw = k.take(hv * cs);
  P.B.tag_bytes = coarse_gcr_persistent_tag_bytes(C.cg.n, C.cg.Vh, grid);
  P.B.tags = k.take(P.B.tag_bytes);
  return P;
}
}  // namespace

size_t coarse_solve_noalloc_bytes(const CoarseLevel& C, int prec, int restart, int grid) {
  Carve k{nullptr};
  plan_noalloc(k, C, prec, restart, grid);
  return k.used;
}

void coarse_solve_noalloc(Ctx& c, CoarseLevel& C, int prec, void* base, int grid, void* x, const void* b,
                          double tol, int max_iter, int restart, wcmg_stats* s) {
  Carve k{reinterpret_cast<char*>(base)};
  restart = std::min(restart, std::max(1, max_iter));
  NoAllocPlan P = plan_noalloc(k, C, prec, restart, grid);
  const size_t nall = (size_t)C.cg.V * C.cg.n;
  // the previous call's barrier epochs, counters, status words and tags are not ours
  noalloc_zero(P.B.ctl, kPersistCtlBytes, c.st);
  noalloc_zero(P.B.tags, P.B.tag_bytes, c.st);
  launch_coarse_canon(prec, P.vb, const_cast<void*>(b), C.perm.as<int>(), C.cg.V, C.cg.n, true, c.st);
  auto t0 = std::chrono::steady_clock::now();
  persistent_launch_bufs(c, grid, P.B, C, prec, P.vx, P.vb, P.t, P.y, P.r, P.br, tol, restart, max_iter, false,
                         false);
  // iterations, status and the barrier-abort flag of the launch (pinned staging, no allocation)
  HIPCHK(hipMemcpyAsync(c.red.host, reinterpret_cast<char*>(P.B.ctl) + kPersistInfoOffset, 3 * sizeof(int),
                        hipMemcpyDeviceToHost, c.st));
  HIPCHK(hipStreamSynchronize(c.st));
  const int* info = reinterpret_cast<const int*>(c.red.host);
  if (info[2]) fail(WCMG_EHIP, "persistent coarse solve: a grid barrier timed out");
  wcmg_stats st{};
  st.iters = info[0];
  st.status = info[1];
  st.t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  launch_coarse_canon(prec, P.vx, x, C.perm.as<int>(), C.cg.V, C.cg.n, false, c.st);
  // ||b - Yhat x|| / ||b|| of the full coarse system
  CoarseOp op{&C, prec, nullptr, c.st};
  op.Dfull(P.t, P.vx);
  blas_axpby(prec, 1.0, 0.0, P.vb, -1.0, 0.0, P.t, nall, c.st);
  const double rr = norm2(c, prec, P.t, nall), bb = norm2(c, prec, P.vb, nall);
  st.true_rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
  if (s) *s = st;
}

long persistent_collect(Ctx& c, PersistWork& w, int* status) {
  if (status) *status = WCMG_OK;
  if (!w.pending) return 0;
  w.pending = false;
  int info[3] = {0, 0, 0};
  char* ctl = w.ctl.as<char>();
  HIPCHK(hipMemcpyAsync(info, ctl + kPersistInfoOffset, sizeof(info), hipMemcpyDeviceToHost, c.st));
  HIPCHK(hipStreamSynchronize(c.st));
  HIPCHK(hipMemsetAsync(ctl + kPersistInfoOffset, 0, sizeof(info), c.st));
  if (info[2]) {
    // barrier flags of an aborted launch are inconsistent: start again from zero
    HIPCHK(hipMemsetAsync(ctl, 0, kPersistCtlBytes, c.st));
    fail(WCMG_EHIP, "persistent coarse solve: a grid barrier timed out");
  }
  if (status) *status = info[1];
  return info[0];
}

// ---------------------------------------------------------------------------
// multigrid preconditioner: fine Wilson-clover level and one or two coarse
// stencil levels, recursive flexible GCR ("Implementation" paragraph)
// ---------------------------------------------------------------------------
struct MGSolver {
  Ctx& c;
  LatticeState& L;
  int sp;  // precision of the fine part of the preconditioner
  int cp;  // precision of the coarse levels
  int fprec = -1;  // storage of the fields in the fine smoother (F16 or as sp)
  DBuf r_s, e_s, res_s, Ar_s;
  struct Level {
    DBuf cb, cc, cbr, cy;       // right-hand side, solution, reduced forms
    DBuf rfull, e, res, Ar;     // preconditioner and smoother work of this level
    GcrSpace space{};
    GcrSpaceB bspace{};         // lockstep space for batches
    int batch = 1;              // right-hand sides the buffers hold
    long calls = 0, iters = 0;
    PersistWork pw;             // the coarsest GCR as one cooperative launch (coarse_launch 0, 2)
    DBuf d_in, d_out, d_br, d_y;  // FP64 vectors of the deflated coarsest solve (coarsest 2)
    GcrSpace space64{};
  };
  int batch = 1;  // right-hand sides the fine buffers hold
  std::vector<Level> lv;  // lv[li]: coarse level li + 1
  long calls = 0, iters = 0;
  // work buffers owned by the preconditioner: a captured graph keeps their
  // addresses, so nothing outside may reallocate them
  FineWork fwork;
  CoarseWork cwork;
  // graph mode (cycle_mode 2): the preconditioner captured once and replayed
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  DBuf g_r, g_z;

  ~MGSolver() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
  }
  bool fixed() const { return L.params.cycle_mode == 1 || L.params.cycle_mode == 2; }
  bool graph_failed = false;  // cycle_mode 3: the capture was refused; the body runs eagerly

  MGSolver(Ctx& ctx, LatticeState& lat) : c(ctx), L(lat) {
    sp = L.params.smoother_prec == WCMG_F64 ? WCMG_F64 : WCMG_F32;
    // F16: FP32 spinors and arithmetic with half-precision links and clover
    fprec = L.params.smoother_prec == WCMG_F16 ? WCMG_F16 : -1;
    cp = sp;
    const Geom& g = L.F.g;
    size_t hb = spinor_bytes(sp, g.Vh);
    r_s.alloc(hb);
    e_s.alloc(hb);
    res_s.alloc(hb);
    Ar_s.alloc(hb);
    const size_t cs = (cp == WCMG_F64 ? 16 : 8);
    lv.resize(L.params.nlevels);
    for (size_t li = 0; li < lv.size(); ++li) {
      CoarseLevel& C = *L.levels[li];
      Level& V = lv[li];
      const size_t nall = (size_t)C.cg.V * C.cg.n;
      for (DBuf* b : {&V.cb, &V.cc, &V.cbr, &V.cy, &V.rfull, &V.e, &V.res, &V.Ar}) b->alloc(nall * cs);
      V.space.prec = cp;
      V.space.n = C.cg.split ? (size_t)C.cg.Vh * C.cg.n : nall;
      V.space.bytes = V.space.n * cs;
    }
  }

  int nlev() const { return L.params.nlevels; }
  const void* vecs(int prec) const { return prec == WCMG_F64 ? L.T0.v64.p : L.T0.v32.p; }
  const void* vbm(int prec) const { return prec == WCMG_F32 ? L.T0.vbm32.p : nullptr; }
  bool half_transfer(int prec) const { return prec == WCMG_F32 && L.params.transfer_fp16 != 0 && L.T0.v16.p; }
  const void* v16(int prec) const { return half_transfer(prec) ? L.T0.v16.p : nullptr; }
  const void* vbm16(int prec) const { return half_transfer(prec) ? L.T0.vbm16.p : nullptr; }
  CoarseOp cop(int li) {
    CoarseOp o{L.levels[li].get(), cp, &cwork, c.st, &c.timer};
    o.timer_base = li < 2 ? 20 + 2 * li : 96 + 2 * (li - 2);
    return o;
  }

  // approximate solution of coarse level li + 1: out = Dhat^-1 in (full vectors)
  void coarse_solve(int li, void* out, void* in) {
    CoarseLevel& C = *L.levels[li];
    Level& V = lv[li];
    CoarseOp op = cop(li);
    const wcmg_mg_params& p = L.params;
    const bool last = li + 1 == nlev();
    ++V.calls;
    if (last && p.coarsest == 1) {
      dense_inverse_apply(cp, L.dense.p, L.dense_n, in, out, c.st);
      V.iters += 1;
      return;
    }
    if (last && p.coarsest == 2) {
      deflated_solve(li, out, in);
      return;
    }
    if (last && C.cg.split && persistent_ok(li)) {
      persistent_solve(li, out, in);
      return;
    }
    OpFn Kf = [this, li](void* o, const void* i) { precondition_coarse(li, o, i); };
    const OpFn* K = (!last && C.cg.split) ? &Kf : nullptr;
    KrylovResult kr;
    const bool fx = fixed();
    if (C.cg.split) {
      op.reduced_source(V.cbr.p, in);
      double bn = fx ? 1.0 : std::sqrt(norm2(c, cp, V.cbr.p, op.neven()));
      OpFn A = [&](void* o, const void* i) { op.Dr(o, i); };
      kr = gcr(c, V.space, A, K, V.cy.p, V.cbr.p, true, p.tol[li], bn, p.restart[li], p.max_iter[li], fx);
      op.reconstruct(out, V.cy.p, in);
    } else {
      double bn = fx ? 1.0 : std::sqrt(norm2(c, cp, in, op.nall()));
      OpFn A = [&](void* o, const void* i) { op.Dfull(o, i); };
      kr = gcr(c, V.space, A, nullptr, out, in, true, p.tol[li], bn, p.restart[li], p.max_iter[li], fx);
    }
    V.iters += kr.iters;
  }

  // unpreconditioned coarsest GCR in one cooperative launch: not under graph
  // capture (cycle_mode 2), and only where the device runs the whole grid at once
  bool persistent_ok(int li) {
    const wcmg_mg_params& p = L.params;
    if (p.coarse_launch == 1 || p.cycle_mode == 2) return false;  // cycle_mode 3 captures it
    return persistent_available(lv[li].pw, cp, *L.levels[li], p.restart[li]);
  }

  void persistent_solve(int li, void* out, void* in) {
    Level& V = lv[li];
    const wcmg_mg_params& p = L.params;
    const int id = 28 + li;
    hipEvent_t e = nullptr;
    if (c.timer.on) c.timer.begin(id, &e);
    persistent_launch(c, V.pw, *L.levels[li], cp, out, in, V.rfull.p, V.cy.p, V.res.p, V.cbr.p, p.tol[li],
                      p.restart[li], p.max_iter[li], fixed(), p.coarse_launch == 2,
                      p.coarse_fp16 != 0 && cp == WCMG_F32, true);
    if (e) c.timer.end(id, e);
  }

  // coarsest == 2: FP64 GCR on the coarsest operator with the deflation pairs
  // at the head of its basis, started from the deflated guess Z (Q^dag b)
  void deflated_solve(int li, void* out, void* in) {
    CoarseLevel& C = *L.levels[li];
    Level& V = lv[li];
    const wcmg_mg_params& p = L.params;
    hipStream_t st = c.st;
    CoarseOp op{&C, WCMG_F64, &cwork, st};
    const bool split = C.cg.split;
    const size_t nall = op.nall(), n = split ? op.neven() : nall, vb = nall * 16;
    for (DBuf* b : {&V.d_in, &V.d_out, &V.d_br, &V.d_y}) b->alloc(vb);
    V.space64.prec = WCMG_F64;
    V.space64.n = n;
    V.space64.bytes = vb;
    blas_convert(WCMG_F64, V.d_in.p, cp, in, nall, st);
    void* rhs = V.d_in.p;
    if (split) {
      op.reduced_source(V.d_br.p, V.d_in.p);
      rhs = V.d_br.p;
    }
    GcrDeflation D;
    for (int j = 0; j < L.defl_k; ++j) {
      D.Q.push_back((char*)L.defl_q.p + (size_t)j * vb);
      D.Z.push_back((char*)L.defl_z.p + (size_t)j * vb);
    }
    D.qa = L.defl_qa.as<double>();
    double* dots = L.defl_tmp.as<double>();
    double* coef = dots + 2 * (kMaxRestart + 16);
    blas_multi_cdot(WCMG_F64, D.Q.data(), L.defl_k, rhs, n, c.red.out(dots), st);
    blas_defl_coefs(dots, coef, L.defl_k, st);
    blas_zero(WCMG_F64, V.d_y.p, n, st);
    blas_gcr_update_x_dev(WCMG_F64, D.Z.data(), L.defl_k, V.d_y.p, n, coef, st);
    const bool fx = fixed();
    const double bn = fx ? 1.0 : std::sqrt(norm2(c, WCMG_F64, rhs, n));
    OpFn A = [&](void* o, const void* i) {
      if (split)
        op.Dr(o, i);
      else
        op.Dfull(o, i);
    };
    KrylovResult kr = gcr(c, V.space64, A, nullptr, V.d_y.p, rhs, false, p.tol[li], bn, p.restart[li],
                          p.max_iter[li], fx, &D);
    if (split)
      op.reconstruct(V.d_out.p, V.d_y.p, V.d_in.p);
    else
      blas_copy(WCMG_F64, V.d_out.p, V.d_y.p, nall, st);
    blas_convert(cp, out, WCMG_F64, V.d_out.p, nall, st);
    V.iters += kr.iters;
  }

  // iterations the persistent coarse solves counted on the device (raises
  // if one of them lost its grid barrier); returns the first failure code
  // they reported (breakdown, NaN), WCMG_OK when none did
  int collect_device_stats() {
    int first = WCMG_OK;
    for (Level& V : lv) {
      int code = WCMG_OK;
      V.iters += persistent_collect(c, V.pw, &code);
      if (code != WCMG_OK && first == WCMG_OK) first = code;
    }
    return first;
  }

  // MR smoothing of e towards D_r e = r on the even half of n elements
  // DrRed(out, in, o, e, coef): D_r with <out, in>, ||out||^2 reduced into o in
  // its own last launch, the pending update of e and in (coefficients coef,
  // previous D_r result in out) fused into its first (e null: none); returns
  // false, launching nothing, where it does not apply
  template <typename DrFn, typename DrRedFn>
  void mr_smooth(const DrFn& Dr, const DrRedFn& DrRed, int prec, void* e, const void* r, void* res, void* Ar,
                 size_t n) {
    const int nu = L.params.nu_post;
    if (nu <= 0) return;
    hipStream_t st = c.st;
    Dr(Ar, e);
    blas_copy(prec, res, r, n, st);
    blas_axpby(prec, -1.0, 0.0, Ar, 1.0, 0.0, res, n, st);
    // alpha = <Ar, r> / ||Ar||^2 stays on the device: no host round trip; with the
    // fused D_r the update of step i runs inside the first launch of step i + 1
    bool pending = false;
    for (int i = 0; i < nu; ++i) {
      if (DrRed(Ar, res, c.red.out(), pending ? e : nullptr, c.red.dres())) {
        pending = true;
        continue;
      }
      Dr(Ar, res);
      blas_cdot_norm(prec, Ar, res, n, c.red.out(), st);
      blas_mr_update_dev(prec, c.red.dres(), e, res, Ar, n, st);
    }
    if (pending) blas_mr_update_dev(prec, c.red.dres(), e, res, Ar, n, st);
  }

  // K_li(r_e) on coarse level li + 1: even part of P (next-level solve) R (r_e, 0), then MR
  void precondition_coarse(int li, void* z, const void* r) {
    hipStream_t st = c.st;
    CoarseLevel& C = *L.levels[li];
    CoarseTransfer& T = *L.ctr[li];
    CoarseLevel& Cn = *L.levels[li + 1];
    Level& V = lv[li];
    Level& W = lv[li + 1];
    CoarseOp op = cop(li);
    const size_t ne = op.neven(), na = op.nall();
    const void* P = cp == WCMG_F64 ? T.v64.p : T.v32.p;
    blas_copy(cp, V.rfull.p, r, ne, st);
    blas_zero(cp, (char*)V.rfull.p + ne * op.csize(), na - ne, st);
    launch_ctr_restrict(cp, W.cb.p, Cn.cg.n, 0, V.rfull.p, 0, P, T.vstride(), T.members.as<int>(), Cn.cg.V,
                        T.bg.bvol, C.cg.n, T.nvec, 1, st);
    coarse_solve(li + 1, W.cc.p, W.cb.p);
    launch_ctr_prolong(cp, V.e.p, 0, W.cc.p, 0, P, T.vstride(), T.blk.as<int>(), C.cg.V, C.cg.n, T.nvec, 1, st);
    mr_smooth([&](void* o, const void* i) { op.Dr(o, i); },
              [](void*, void*, const RedOut&, void*, const double*) { return false; }, cp, V.e.p, r, V.res.p, V.Ar.p,
              ne);
    blas_copy(cp, z, V.e.p, ne, st);
  }

  // K(r_e): even part of P (coarse solve) R (r_e, 0), then MR smoothing on D_r
  void precondition(void* z64, const void* r64) {
    if (L.params.cycle_mode == 2) return precondition_graph(z64, r64);
    if (L.params.cycle_mode == 3 && graph_ready()) return precondition_graph(z64, r64);
    precondition_body(z64, r64);
  }

  // cycle_mode 3: the body is a pure sequence of kernels -- no host read --
  // when the only coarse level is solved by the persistent launch, whose
  // adaptive tolerance lives on the device; then it is captured and replayed
  // like cycle_mode 2 (anything else runs eagerly)
  bool graph_ready() {
    const wcmg_mg_params& p = L.params;
    if (graph_failed || p.nlevels != 1 || p.coarsest != 0 || !L.levels[0]->cg.split) return false;
    return persistent_ok(0);
  }

  // cycle_mode 2: the body (kernels only: fixed inner lengths, device
  // scalars) is captured once on a side stream into a graph that works on
  // buffers of its own, and replayed on the context stream
  void precondition_graph(void* z64, const void* r64) {
    const Geom& g = L.F.g;
    const size_t n = (size_t)12 * g.Vh;
    if (!gexec) {
      const size_t hb = spinor_bytes(WCMG_F64, g.Vh);
      g_r.alloc(hb);
      g_z.alloc(hb);
      blas_copy(WCMG_F64, g_r.p, r64, n, c.st);
      precondition_body(g_z.p, g_r.p);  // eager run: every buffer is allocated before the capture
      HIPCHK(hipStreamSynchronize(c.st));
      if (!cap) HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      hipStream_t keep = c.st;
      const bool timer_on = c.timer.on;
      c.timer.on = false;
      c.st = cap;
      HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
      bool body_ok = true;
      Error body_err{WCMG_OK, ""};
      try {
        precondition_body(g_z.p, g_r.p);
      } catch (const Error& err) {
        body_ok = false;
        body_err = err;
      }
      hipError_t e = hipStreamEndCapture(cap, &graph);
      c.st = keep;
      c.timer.on = timer_on;
      if (body_ok && e == hipSuccess) e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
      if (!body_ok || e != hipSuccess) {
        (void)hipGetLastError();
        if (graph) (void)hipGraphDestroy(graph);
        graph = nullptr;
        gexec = nullptr;
        // cycle_mode 2 needs the graph; cycle_mode 3 runs the same body eagerly instead
        if (L.params.cycle_mode == 2) {
          if (!body_ok) throw body_err;
          HIPCHK(e);
        }
        graph_failed = true;
        precondition_body(z64, r64);
        return;
      }
    }
    blas_copy(WCMG_F64, g_r.p, r64, n, c.st);
    HIPCHK(hipGraphLaunch(gexec, c.st));
    blas_copy(WCMG_F64, z64, g_z.p, n, c.st);
    ++calls;
    if (L.params.cycle_mode == 3) {
      // the replayed persistent launch counts its steps on the device as the eager one does
      ++lv[0].calls;
      lv[0].pw.pending = true;
    }
  }

  void precondition_body(void* z64, const void* r64) {
    const Geom& g = L.F.g;
    hipStream_t st = c.st;
    FineOp op{&c, &L.F, sp, &fwork, st, fprec};
    const size_t n = (size_t)12 * g.Vh;
    CoarseLevel& C = *L.levels[0];
    Level& V = lv[0];
    spinor_convert(sp, r_s.p, WCMG_F64, r64, g.Vh, st);
    launch_restrict(sp, V.cb.p, C.cg.n, 1, r_s.p, vecs(sp), L.T0.nvec, 0, g, L.T0.bg, false, st, vbm(sp),
                    vbm16(sp));
    coarse_solve(0, V.cc.p, V.cb.p);
    launch_prolong(sp, e_s.p, V.cc.p, vecs(sp), L.T0.nvec, 0, g, L.T0.bg, st, v16(sp));
    mr_smooth([&](void* o, const void* i) { op.Dr(o, i); },
              [&](void* o, void* i, const RedOut& ro, void* ee, const double* cf) {
                return op.Dr_red(o, i, ro, ee, cf);
              },
              sp, e_s.p, r_s.p, res_s.p, Ar_s.p, n);
    spinor_convert(WCMG_F64, z64, sp, e_s.p, g.Vh, st);
    ++calls;
  }

  // ---- batches of right-hand sides (lockstep) ----
  void ensure_batch(int nrhs) {
    const Geom& g = L.F.g;
    if (batch < nrhs) {
      const size_t hb = spinor_bytes(sp, g.Vh) * nrhs;
      for (DBuf* b : {&r_s, &e_s, &res_s, &Ar_s}) b->alloc(hb);
      batch = nrhs;
    }
    const size_t cs = (cp == WCMG_F64 ? 16 : 8);
    for (size_t li = 0; li < lv.size(); ++li) {
      Level& V = lv[li];
      if (V.batch >= nrhs) continue;
      CoarseLevel& C = *L.levels[li];
      const size_t nall = (size_t)C.cg.V * C.cg.n;
      for (DBuf* b : {&V.cb, &V.cc, &V.cbr, &V.cy, &V.rfull, &V.e, &V.res, &V.Ar}) b->alloc(nall * cs * nrhs);
      V.batch = nrhs;
    }
  }

  // MR smoothing of nrhs right-hand sides (n elements each, vs apart) in lockstep
  template <typename DrFn>
  void mr_smooth_b(const DrFn& Dr, int prec, void* e, const void* r, void* res, void* Ar, size_t n, size_t vs,
                   int nrhs) {
    const int nu = L.params.nu_post;
    if (nu <= 0) return;
    hipStream_t st = c.st;
    const size_t es = prec == WCMG_F64 ? 16 : 8;
    Dr(Ar, e);
    for (int i = 0; i < nrhs; ++i) {
      const size_t o = (size_t)i * vs * es;
      blas_copy(prec, (char*)res + o, (const char*)r + o, n, st);
      blas_axpby(prec, -1.0, 0.0, (char*)Ar + o, 1.0, 0.0, (char*)res + o, n, st);
    }
    for (int it = 0; it < nu; ++it) {
      Dr(Ar, res);
      blas_cdot_norm_b(prec, Ar, res, vs, n, nrhs, c.red.outb(c.red.dres(), 3), st);
      blas_mr_update_b(prec, c.red.dres(), 3, e, res, Ar, vs, n, nrhs, st);
    }
  }

  void coarse_solve_b(int li, void* out, void* in, int nrhs) {
    CoarseLevel& C = *L.levels[li];
    Level& V = lv[li];
    CoarseOp op = cop(li);
    const wcmg_mg_params& p = L.params;
    const bool last = li + 1 == nlev();
    const size_t cs = op.csize(), na = op.nall();
    ++V.calls;
    if (last && p.coarsest == 1) {
      for (int i = 0; i < nrhs; ++i)
        dense_inverse_apply(cp, L.dense.p, L.dense_n, (char*)in + i * na * cs, (char*)out + i * na * cs, c.st);
      V.iters += 1;
      return;
    }
    OpFn Kf = [this, li, nrhs](void* o, const void* i) { precondition_coarse_b(li, o, i, nrhs); };
    const OpFn* K = (!last && C.cg.split) ? &Kf : nullptr;
    V.bspace.prec = cp;
    V.bspace.nrhs = nrhs;
    V.bspace.vs = na;
    std::vector<double> bn(nrhs);
    std::vector<KrylovResult> kr;
    const bool fx = fixed();
    auto norms = [&](const void* v, size_t cnt) {
      if (fx) {
        std::fill(bn.begin(), bn.end(), 1.0);
        return;
      }
      blas_norm2_b(cp, v, na, cnt, nrhs, c.red.outb(c.red.dres(), 1), c.st);
      const double* h = c.red.fetch(nrhs);
      for (int i = 0; i < nrhs; ++i) bn[i] = std::sqrt(h[i]);
    };
    if (C.cg.split) {
      op.reduced_source(V.cbr.p, in, nrhs);
      V.bspace.n = op.neven();
      norms(V.cbr.p, op.neven());
      OpFn A = [&](void* o, const void* i) { op.Dr(o, i, nrhs); };
      kr = gcr_b(c, V.bspace, A, K, V.cy.p, V.cbr.p, true, p.tol[li], bn.data(), p.restart[li], p.max_iter[li], fx);
      op.reconstruct(out, V.cy.p, in, nrhs);
    } else {
      V.bspace.n = na;
      norms(in, na);
      OpFn A = [&](void* o, const void* i) { op.Dfull(o, i, nrhs); };
      kr = gcr_b(c, V.bspace, A, nullptr, out, in, true, p.tol[li], bn.data(), p.restart[li], p.max_iter[li], fx);
    }
    int mx = 0;
    for (auto& k : kr) mx = std::max(mx, k.iters);
    V.iters += mx;
  }

  void precondition_coarse_b(int li, void* z, const void* r, int nrhs) {
    hipStream_t st = c.st;
    CoarseLevel& C = *L.levels[li];
    CoarseTransfer& T = *L.ctr[li];
    CoarseLevel& Cn = *L.levels[li + 1];
    Level& V = lv[li];
    Level& W = lv[li + 1];
    CoarseOp op = cop(li);
    const size_t ne = op.neven(), na = op.nall(), cs = op.csize();
    const size_t nan = (size_t)Cn.cg.V * Cn.cg.n;
    const void* P = cp == WCMG_F64 ? T.v64.p : T.v32.p;
    for (int i = 0; i < nrhs; ++i) {
      const size_t o = (size_t)i * na * cs;
      blas_copy(cp, (char*)V.rfull.p + o, (const char*)r + o, ne, st);
      blas_zero(cp, (char*)V.rfull.p + o + ne * cs, na - ne, st);
    }
    launch_ctr_restrict(cp, W.cb.p, Cn.cg.n, nan, V.rfull.p, na, P, T.vstride(), T.members.as<int>(), Cn.cg.V,
                        T.bg.bvol, C.cg.n, T.nvec, nrhs, st);
    coarse_solve_b(li + 1, W.cc.p, W.cb.p, nrhs);
    launch_ctr_prolong(cp, V.e.p, na, W.cc.p, nan, P, T.vstride(), T.blk.as<int>(), C.cg.V, C.cg.n, T.nvec, nrhs, st);
    mr_smooth_b([&](void* o, const void* i) { op.Dr(o, i, nrhs); }, cp, V.e.p, r, V.res.p, V.Ar.p, ne, na, nrhs);
    for (int i = 0; i < nrhs; ++i) {
      const size_t o = (size_t)i * na * cs;
      blas_copy(cp, (char*)z + o, (const char*)V.e.p + o, ne, st);
    }
  }

  // batched K(r_e) on nrhs FP64 even halves stored back to back
  void precondition_b(void* z64, const void* r64, int nrhs) {
    ensure_batch(nrhs);
    const Geom& g = L.F.g;
    hipStream_t st = c.st;
    FineOp op{&c, &L.F, sp, &fwork, st, fprec};
    const size_t n = (size_t)12 * g.Vh;
    const size_t h64 = spinor_bytes(WCMG_F64, g.Vh), hs = spinor_bytes(sp, g.Vh);
    CoarseLevel& C = *L.levels[0];
    Level& V = lv[0];
    const size_t na = (size_t)C.cg.V * C.cg.n, cs = cp == WCMG_F64 ? 16 : 8;
    for (int i = 0; i < nrhs; ++i) {
      spinor_convert(sp, (char*)r_s.p + i * hs, WCMG_F64, (const char*)r64 + i * h64, g.Vh, st);
      launch_restrict(sp, (char*)V.cb.p + i * na * cs, C.cg.n, 1, (char*)r_s.p + i * hs, vecs(sp), L.T0.nvec, 0, g,
                      L.T0.bg, false, st, vbm(sp), vbm16(sp));
    }
    coarse_solve_b(0, V.cc.p, V.cb.p, nrhs);
    for (int i = 0; i < nrhs; ++i)
      launch_prolong(sp, (char*)e_s.p + i * hs, (char*)V.cc.p + i * na * cs, vecs(sp), L.T0.nvec, 0, g, L.T0.bg,
                     st, v16(sp));
    mr_smooth_b([&](void* o, const void* i) { op.Dr(o, i, nrhs); }, sp, e_s.p, r_s.p, res_s.p, Ar_s.p, n, n, nrhs);
    for (int i = 0; i < nrhs; ++i)
      spinor_convert(WCMG_F64, (char*)z64 + i * h64, sp, (char*)e_s.p + i * hs, g.Vh, st);
    ++calls;
  }
};

static void require_hierarchy(LatticeState& L) {
  if (!L.have_params) fail(WCMG_ESTATE, "multigrid parameters not set");
  const int nl = L.params.nlevels;
  if ((int)L.levels.size() < nl) fail(WCMG_ESTATE, "coarse operator not built");
  for (int l = 0; l < nl; ++l)
    if (!L.levels[l]->built) fail(WCMG_ESTATE, "coarse operator not built");
  if (L.params.coarsest == 1 && L.dense_n == 0) fail(WCMG_ESTATE, "coarsest dense inverse not built");
  if (L.params.coarsest == 2 && L.defl_k == 0) fail(WCMG_ESTATE, "coarsest deflation space not built");
}

// ---------------------------------------------------------------------------
// setup: inverse iteration on D_p with Rayleigh-quotient monitoring
// ---------------------------------------------------------------------------
// inverse iteration on the coarse operator Dhat_p = Dhat X^-1 of coarse level
// `level` (>= 1) for the vectors that build coarse level level + 1
static void mg_setup_null_vectors_coarse(Ctx& c, LatticeState& L, int level) {
  const wcmg_mg_params& p = L.params;
  if (level >= p.nlevels) fail(WCMG_EINVAL, "the parameters have no coarse level below this one");
  if ((int)L.levels.size() < level || !L.levels[level - 1]->built) fail(WCMG_ESTATE, "coarse level not built");
  hipStream_t st = c.st;
  CoarseLevel& C1 = *L.levels[level - 1];
  const int nvec = p.nvec[level];
  const size_t n = (size_t)C1.cg.V * C1.cg.n;
  // coarse levels have no half-precision operator: F16 runs as F32 here
  const int sp = p.setup_prec == WCMG_F64 ? WCMG_F64 : WCMG_F32;
  const size_t cs = sp == WCMG_F64 ? 16 : 8;
  CoarseOp cop{&C1, sp, &c.cw[sp == WCMG_F64 ? 0 : 1], st};
  OpFn Dp = [&](void* o, const void* i) { cop.Dp(o, i); };
  while ((int)L.ctr.size() < level) L.ctr.emplace_back(new CoarseTransfer());
  CoarseTransfer& T = *L.ctr[level - 1];
  T.nf = C1.cg.n;
  T.nsites = C1.cg.V;
  T.raw.alloc((size_t)nvec * n * 16);
  void* v = c.scratch_buf(9, n * cs);
  void* x = c.scratch_buf(10, n * cs);
  void* w = c.scratch_buf(11, n * cs);
  void* v64 = c.scratch_buf(16, n * 16);
  void* prev = c.scratch_buf(17, (size_t)nvec * n * cs);
  GcrSpace S{sp, n, n * cs, {}, {}, DBuf()};
  std::vector<const void*> found;
  std::vector<double> cf(2 * nvec);
  for (int k = 0; k < nvec; ++k) {
    random_coarse_vector(v64, p.seed, k, level, C1.perm.as<int>(), C1.cg.V, C1.cg.n, st);
    reals_convert(sp, v, reinterpret_cast<const double*>(v64), 2 * n, st);
    double rho_old = -1.0;
    for (int step = 0; step < p.setup_max_steps; ++step) {
      gcr(c, S, Dp, nullptr, x, v, true, 0.0, 1.0, p.setup_relax, p.setup_relax, true);
      blas_copy(sp, v, x, n, st);
      for (int pass = 0; pass < 2 && k > 0; ++pass) {
        blas_multi_cdot(sp, found.data(), k, v, n, c.red.out(), st);
        const double* d = c.red.fetch(2 * k);
        for (int j = 0; j < 2 * k; ++j) cf[j] = -d[j];
        blas_multi_axpy(sp, cf.data(), found.data(), k, v, n, st);
      }
      double nv = std::sqrt(norm2(c, sp, v, n));
      if (!(nv > 0.0) || !finite(nv)) fail(WCMG_ENAN, "setup vector vanished");
      blas_axpby(sp, 1.0 / nv, 0.0, v, 0.0, 0.0, v, n, st);
      Dp(w, v);
      double rho = norm2(c, sp, w, n);
      if (rho_old > 0.0 && std::fabs(rho - rho_old) / rho < p.setup_rq_tol) break;
      rho_old = rho;
    }
    void* keep = (char*)prev + (size_t)k * n * cs;
    blas_copy(sp, keep, v, n, st);
    found.push_back(keep);
    void* dst = (char*)T.raw.p + (size_t)k * n * 16;
    blas_convert(WCMG_F64, dst, sp, v, n, st);
  }
  HIPCHK(hipStreamSynchronize(st));
  T.nvec = nvec;
  T.have_vecs = true;
  T.orth = false;
  for (size_t l = level; l < L.levels.size(); ++l) L.levels[l]->built = false;
  L.dense_n = 0;
  L.mg.reset();
}

void mg_setup_null_vectors(Ctx& c, LatticeState& L, int level) {
  if (level >= 1) return mg_setup_null_vectors_coarse(c, L, level);
  if (level != 0) fail(WCMG_EINVAL, "level out of range");
  if (!L.F.have_clover) fail(WCMG_ESTATE, "clover not set");
  if (!L.have_params) fail(WCMG_ESTATE, "multigrid parameters not set");
  const wcmg_mg_params& p = L.params;
  const Geom& g = L.F.g;
  hipStream_t st = c.st;
  const int nvec = p.nvec[0];
  // arithmetic of the inverse iteration: F64, F32, or F32 vectors with F16 fields
  const int sp = p.setup_prec == WCMG_F64 ? WCMG_F64 : WCMG_F32;
  const int fp = p.setup_prec == WCMG_F16 ? WCMG_F16 : -1;
  const size_t hb = spinor_bytes(sp, g.Vh), hb64 = spinor_bytes(WCMG_F64, g.Vh);
  const size_t n = (size_t)24 * g.Vh;
  FineOp op{&c, &L.F, sp, &c.fw[sp], st, fp};
  OpFn Dp = [&](void* o, const void* i) {
    op.Dp(o, (char*)o + hb, i, (const char*)i + hb);
  };
  L.T0.raw.alloc((size_t)nvec * 2 * hb64);
  void* v = c.scratch_buf(9, 2 * hb);
  void* x = c.scratch_buf(10, 2 * hb);
  void* w = c.scratch_buf(11, 2 * hb);
  void* v64 = c.scratch_buf(16, 2 * hb64);
  // the vectors found so far, in the setup's precision
  void* prev = c.scratch_buf(17, (size_t)nvec * 2 * hb);
  GcrSpace S{sp, n, 2 * hb, {}, {}, DBuf()};
  std::vector<const void*> found;
  std::vector<double> cf(2 * nvec);
  for (int k = 0; k < nvec; ++k) {
    random_fine_vector(v64, p.seed, k, 0, g, st);
    spinor_convert(sp, v, WCMG_F64, v64, g.Vh, st);
    spinor_convert(sp, (char*)v + hb, WCMG_F64, (char*)v64 + hb64, g.Vh, st);
    double rho_old = -1.0;
    for (int step = 0; step < p.setup_max_steps; ++step) {
      gcr(c, S, Dp, nullptr, x, v, true, 0.0, 1.0, p.setup_relax, p.setup_relax, true);
      blas_copy(sp, v, x, n, st);
      for (int pass = 0; pass < 2 && k > 0; ++pass) {
        blas_multi_cdot(sp, found.data(), k, v, n, c.red.out(), st);
        const double* d = c.red.fetch(2 * k);
        for (int j = 0; j < 2 * k; ++j) cf[j] = -d[j];
        blas_multi_axpy(sp, cf.data(), found.data(), k, v, n, st);
      }
      double nv = std::sqrt(norm2(c, sp, v, n));
      if (!(nv > 0.0) || !finite(nv)) fail(WCMG_ENAN, "setup vector vanished");
      blas_axpby(sp, 0.0, 0.0, v, 1.0 / nv, 0.0, v, n, st);
      Dp(w, v);
      double rho = norm2(c, sp, w, n);
      if (rho_old > 0.0 && std::fabs(rho - rho_old) / rho < p.setup_rq_tol) break;
      rho_old = rho;
    }
    void* keep = (char*)prev + (size_t)k * 2 * hb;
    blas_copy(sp, keep, v, n, st);
    found.push_back(keep);
    void* dst = (char*)L.T0.raw.p + (size_t)k * 2 * hb64;
    spinor_convert(WCMG_F64, dst, sp, v, g.Vh, st);
    spinor_convert(WCMG_F64, (char*)dst + hb64, sp, (char*)v + hb, g.Vh, st);
  }
  HIPCHK(hipStreamSynchronize(st));
  L.T0.nvec = nvec;
  L.T0.have_vecs = true;
  L.T0.orth = false;
  for (auto& lv : L.levels) lv->built = false;
  L.mg.reset();
}

// ---------------------------------------------------------------------------
// coarse operator  Yhat = R D_p P, direction resolved
// ---------------------------------------------------------------------------
static void build_coarse_tables(CoarseLevel& C) {
  const BlockGeom& bg = C.bg;
  const int V = bg.Vc;
  C.perm_host.resize(V);
  for (int l = 0; l < V; ++l) C.perm_host[l] = coarse_internal_index_host(bg, l);
  std::vector<int> nbr((size_t)V * 8);
  for (int l = 0; l < V; ++l) {
    int c[4] = {l % bg.nb[0], (l / bg.nb[0]) % bg.nb[1], (l / (bg.nb[0] * bg.nb[1])) % bg.nb[2],
                l / (bg.nb[0] * bg.nb[1] * bg.nb[2])};
    for (int mu = 0; mu < 4; ++mu)
      for (int back = 0; back < 2; ++back) {
        int o[4] = {c[0], c[1], c[2], c[3]};
        o[mu] = (o[mu] + (back ? -1 : 1) + bg.nb[mu]) % bg.nb[mu];
        int ol = ((o[3] * bg.nb[2] + o[2]) * bg.nb[1] + o[1]) * bg.nb[0] + o[0];
        nbr[(size_t)C.perm_host[l] * 8 + 2 * mu + back] = C.perm_host[ol];
      }
  }
  C.nbr.alloc(nbr.size() * sizeof(int));
  HIPCHK(hipMemcpy(C.nbr.p, nbr.data(), nbr.size() * sizeof(int), hipMemcpyHostToDevice));
  C.perm.alloc((size_t)V * sizeof(int));
  HIPCHK(hipMemcpy(C.perm.p, C.perm_host.data(), (size_t)V * sizeof(int), hipMemcpyHostToDevice));
}

// X, the eight hops, X^-1, Ytilde = Y X^-1 and the FP32 copies from Y9
static void finalize_coarse(Ctx& c, CoarseLevel& C, int* flag) {
  hipStream_t st = c.st;
  const int n = C.cg.n, V = C.cg.V;
  const size_t nn = (size_t)n * n;
  int hflag[2] = {0, 0};
  // split into X and the eight hops, invert X, form Ytilde = Y X^-1
  C.X[0].alloc((size_t)V * nn * 16);
  C.Yhop[0].alloc((size_t)V * 8 * nn * 16);
  HIPCHK(hipMemcpy2DAsync(C.X[0].p, nn * 16, C.Y9.p, 9 * nn * 16, nn * 16, V, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpy2DAsync(C.Yhop[0].p, 8 * nn * 16, (char*)C.Y9.p + nn * 16, 9 * nn * 16, 8 * nn * 16, V,
                          hipMemcpyDeviceToDevice, st));
  C.Xinv[0].alloc((size_t)V * nn * 16);
  HIPCHK(hipMemcpyAsync(C.Xinv[0].p, C.X[0].p, (size_t)V * nn * 16, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemsetAsync(flag, 0, 64, st));
  launch_batched_inverse(C.Xinv[0].as<double>(), V, n, flag, st);
  C.Yt[0].alloc((size_t)V * 8 * nn * 16);
  launch_coarse_right_mul(C.Yt[0].as<double>(), C.Yhop[0].as<double>(), C.Xinv[0].as<double>(), C.nbr.as<int>(), V,
                          n, st);
  // FP32 copies for the mixed-precision cycle
  C.X[1].alloc((size_t)V * nn * 8);
  C.Xinv[1].alloc((size_t)V * nn * 8);
  C.Yhop[1].alloc((size_t)V * 8 * nn * 8);
  C.Yt[1].alloc((size_t)V * 8 * nn * 8);
  launch_reals_convert(WCMG_F32, C.X[1].p, C.X[0].as<double>(), (size_t)V * nn * 2, st);
  launch_reals_convert(WCMG_F32, C.Xinv[1].p, C.Xinv[0].as<double>(), (size_t)V * nn * 2, st);
  launch_reals_convert(WCMG_F32, C.Yhop[1].p, C.Yhop[0].as<double>(), (size_t)V * 8 * nn * 2, st);
  launch_reals_convert(WCMG_F32, C.Yt[1].p, C.Yt[0].as<double>(), (size_t)V * 8 * nn * 2, st);
  C.Yt16.alloc((size_t)V * 8 * nn * 4);
  launch_reals_convert(WCMG_F16, C.Yt16.p, C.Yt[0].as<double>(), (size_t)V * 8 * nn * 2, st);
  HIPCHK(hipMemcpyAsync(hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hflag[0]) fail(WCMG_ERANK, "singular coarse site block");
  // FP16 fragments for the batched stencil on the matrix cores (red-black levels)
  C.has_frag = false;
  if (C.cg.split && mfma_coarse_supported(n)) {
    C.frag.alloc(mfma_fragment_bytes(V, n));
    HIPCHK(hipMemsetAsync(flag, 0, 64, st));
    build_mfma_fragments(C.frag.p, C.Yt[0].p, V, n, flag, st);
    HIPCHK(hipMemcpyAsync(hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    C.has_frag = hflag[0] == 0;
  }
}

// dense FP64 inverse of the full operator of coarse level index li (the coarsest)
static void build_dense(Ctx& c, LatticeState& L, int li) {
  CoarseLevel& C = *L.levels[li];
  const int N = C.cg.V * C.cg.n;
  if (N > kMaxDense) fail(WCMG_EDIM, "coarsest level too large for the dense solve");
  hipStream_t st = c.st;
  L.dense.alloc((size_t)N * 2 * N * 16);
  int* piv = (int*)c.scratch_buf(13, 64);
  void* pval = c.scratch_buf(14, 64);
  void* f = c.scratch_buf(15, (size_t)N * 16);
  int* flag = (int*)c.scratch_buf(12, 64);
  HIPCHK(hipMemsetAsync(flag, 0, 64, st));
  dense_inverse_build(L.dense.p, C.Y9.p, C.nbr.as<int>(), C.cg.V, C.cg.n, piv, pval, f, flag, st);
  int hflag = 0;
  HIPCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hflag) fail(WCMG_ERANK, "coarsest operator is singular");
  L.dense_n = N;
}

// Deflation pairs of the coarsest operator A (coarsest == 2): block inverse
// iteration on m = min(2K, 96) random vectors (three steps, each vector
// solved to 1e-4 by GCR and the block orthonormalised), then a Rayleigh-Ritz
// step for the smallest singular values inside that subspace: with H =
// (AW)^dag (AW) = Y diag(s^2) Y^dag, the K pairs Z_j = W y_j / s_j and
// Q_j = (AW) y_j / s_j satisfy Q_j = A Z_j with the Q orthonormal (once more
// Gram-Schmidt, twice, against rounding).  Inverse iteration alone (the
// Setup section's relaxation) gives subspaces too far from the low modes:
// deflating with them made the coarsest GCR slower, not faster.
static void build_deflation(Ctx& c, LatticeState& L, int li) {
  const wcmg_mg_params& p = L.params;
  CoarseLevel& C = *L.levels[li];
  const int K = p.nvec[p.nlevels];
  hipStream_t st = c.st;
  CoarseOp op{&C, WCMG_F64, &c.cw[0], st};
  const bool split = C.cg.split;
  const size_t nall = op.nall();
  const size_t n = split ? op.neven() : nall;
  const size_t vb = nall * 16;  // full-size buffers: the red-black operator works on them
  const int m = std::min(2 * K, 96);
  if ((size_t)m > n) fail(WCMG_EDIM, "too many deflation vectors for the coarsest dimension");
  OpFn A = [&](void* o, const void* i) {
    if (split)
      op.Dr(o, i);
    else
      op.Dfull(o, i);
  };
  L.defl_k = 0;
  DBuf wbuf, awbuf;
  wbuf.alloc((size_t)m * vb);
  awbuf.alloc((size_t)m * vb);
  std::vector<const void*> W(m), AW(m);
  for (int i = 0; i < m; ++i) {
    W[i] = (char*)wbuf.p + (size_t)i * vb;
    AW[i] = (char*)awbuf.p + (size_t)i * vb;
  }
  auto wv = [&](int i) { return const_cast<void*>(W[i]); };
  auto awv = [&](int i) { return const_cast<void*>(AW[i]); };
  std::vector<double> cf(2 * m);
  // orthonormalise a list of vectors in place (classical Gram-Schmidt, twice), applying the
  // same combinations to a second list when given
  auto orthonormalise = [&](std::vector<const void*>& X, std::vector<const void*>* Y, int cnt) {
    for (int k = 0; k < cnt; ++k) {
      void* xk = const_cast<void*>(X[k]);
      for (int pass = 0; pass < 2 && k > 0; ++pass) {
        blas_multi_cdot(WCMG_F64, X.data(), k, xk, n, c.red.out(), st);
        const double* d = c.red.fetch(2 * k);
        for (int j = 0; j < 2 * k; ++j) cf[j] = -d[j];
        blas_multi_axpy(WCMG_F64, cf.data(), X.data(), k, xk, n, st);
        if (Y) blas_multi_axpy(WCMG_F64, cf.data(), Y->data(), k, const_cast<void*>((*Y)[k]), n, st);
      }
      const double s = std::sqrt(norm2(c, WCMG_F64, xk, n));
      if (!(s > 0.0) || !finite(s)) fail(WCMG_ERANK, "deflation vectors are linearly dependent");
      blas_axpby(WCMG_F64, 1.0 / s, 0.0, xk, 0.0, 0.0, xk, n, st);
      if (Y) {
        void* yk = const_cast<void*>((*Y)[k]);
        blas_axpby(WCMG_F64, 1.0 / s, 0.0, yk, 0.0, 0.0, yk, n, st);
      }
    }
  };
  for (int i = 0; i < m; ++i)
    random_coarse_vector(wv(i), p.seed, i, 8 + li, C.perm.as<int>(), C.cg.V, C.cg.n, st);
  orthonormalise(W, nullptr, m);
  void* x = c.scratch_buf(19, vb);
  GcrSpace S{WCMG_F64, n, vb, {}, {}, DBuf()};
  for (int step = 0; step < 3; ++step) {
    for (int i = 0; i < m; ++i) {
      gcr(c, S, A, nullptr, x, wv(i), true, 1e-4, 1.0, 30, 1000, false);
      blas_copy(WCMG_F64, wv(i), x, n, st);
    }
    orthonormalise(W, nullptr, m);
  }
  // Rayleigh-Ritz for the smallest singular values of A on span(W)
  for (int i = 0; i < m; ++i) A(awv(i), wv(i));
  std::vector<std::complex<double>> H((size_t)m * m);
  for (int j = 0; j < m; ++j) {
    blas_multi_cdot(WCMG_F64, AW.data(), m, awv(j), n, c.red.out(), st);
    const double* d = c.red.fetch(2 * m);
    for (int i = 0; i < m; ++i) H[(size_t)i * m + j] = std::complex<double>(d[2 * i], d[2 * i + 1]);
  }
  std::vector<double> ev;
  std::vector<std::complex<double>> Yv;
  hermitian_eig(H, m, ev, Yv);
  L.defl_q.alloc((size_t)K * vb);
  L.defl_z.alloc((size_t)K * vb);
  std::vector<const void*> Zs(K), Qs(K);
  for (int j = 0; j < K; ++j) {
    Zs[j] = (char*)L.defl_z.p + (size_t)j * vb;
    Qs[j] = (char*)L.defl_q.p + (size_t)j * vb;
    if (!(ev[j] > 0.0)) fail(WCMG_ERANK, "coarsest operator is singular on the deflation subspace");
    const double inv = 1.0 / std::sqrt(ev[j]);
    for (int i = 0; i < m; ++i) {
      const std::complex<double> yv = Yv[(size_t)i * m + j] * inv;
      cf[2 * i] = yv.real();
      cf[2 * i + 1] = yv.imag();
    }
    blas_zero(WCMG_F64, const_cast<void*>(Zs[j]), n, st);
    blas_zero(WCMG_F64, const_cast<void*>(Qs[j]), n, st);
    blas_multi_axpy(WCMG_F64, cf.data(), W.data(), m, const_cast<void*>(Zs[j]), n, st);
    blas_multi_axpy(WCMG_F64, cf.data(), AW.data(), m, const_cast<void*>(Qs[j]), n, st);
  }
  orthonormalise(Qs, &Zs, K);
  std::vector<double> qa(4 * (size_t)K, 0.0);
  for (int j = 0; j < K; ++j) qa[4 * j] = 1.0;
  L.defl_qa.alloc(qa.size() * sizeof(double));
  L.defl_tmp.alloc((2 * (kMaxRestart + 16) + 4 * kMaxRestart) * sizeof(double));
  HIPCHK(hipMemcpyAsync(L.defl_qa.p, qa.data(), qa.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  L.defl_k = K;
}

// level-2 operator R2 Dhat_p P2 from the level-1 stencil (direction resolved)
// coarse level level + 1 (level >= 1) from coarse level `level` and its vectors
static void mg_build_coarse_next(Ctx& c, LatticeState& L, int level) {
  const wcmg_mg_params& p = L.params;
  if (level >= p.nlevels) fail(WCMG_EINVAL, "the parameters have no coarse level below this one");
  if ((int)L.levels.size() < level || !L.levels[level - 1]->built) fail(WCMG_ESTATE, "coarse level not built");
  if ((int)L.ctr.size() < level || !L.ctr[level - 1]->have_vecs) fail(WCMG_ESTATE, "coarse-level null vectors not set");
  hipStream_t st = c.st;
  CoarseLevel& C1 = *L.levels[level - 1];
  CoarseTransfer& T = *L.ctr[level - 1];
  T.bg = make_block_geom(C1.cg.L, p.block[level]);
  T.nvec = p.nvec[level];
  T.nf = C1.cg.n;
  T.nsites = C1.cg.V;
  while ((int)L.levels.size() <= level) L.levels.emplace_back(new CoarseLevel());
  CoarseLevel& C2 = *L.levels[level];
  C2.bg = T.bg;
  C2.nvec = T.nvec;
  C2.cg = make_coarse_geom(T.bg, T.nvec);
  build_coarse_tables(C2);
  // block membership of the level-1 sites (internal orders on both levels)
  const int V1 = C1.cg.V, V2 = C2.cg.V, bvol = T.bg.bvol;
  std::vector<int> lex1(V1), blk(V1), members((size_t)V2 * bvol), fill(V2, 0);
  for (int l = 0; l < V1; ++l) lex1[C1.perm_host[l]] = l;
  for (int i = 0; i < V1; ++i) {
    int l = lex1[i];
    int x[4];
    for (int k = 0; k < 4; ++k) {
      x[k] = l % C1.cg.L[k];
      l /= C1.cg.L[k];
    }
    const int b2 = (((x[3] / T.bg.b[3]) * T.bg.nb[2] + x[2] / T.bg.b[2]) * T.bg.nb[1] + x[1] / T.bg.b[1]) * T.bg.nb[0] +
                   x[0] / T.bg.b[0];
    const int c2 = C2.perm_host[b2];
    blk[i] = c2;
    members[(size_t)c2 * bvol + fill[c2]++] = i;
  }
  T.blk.alloc(V1 * sizeof(int));
  T.members.alloc(members.size() * sizeof(int));
  HIPCHK(hipMemcpy(T.blk.p, blk.data(), V1 * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(T.members.p, members.data(), members.size() * sizeof(int), hipMemcpyHostToDevice));
  // P2: block x chirality orthonormalisation
  const size_t vbytes = T.vstride() * 16;
  T.v64.alloc((size_t)T.nvec * vbytes);
  HIPCHK(hipMemcpyAsync(T.v64.p, T.raw.p, (size_t)T.nvec * vbytes, hipMemcpyDeviceToDevice, st));
  int* flag = (int*)c.scratch_buf(12, 64);
  HIPCHK(hipMemsetAsync(flag, 0, 64, st));
  launch_ctr_block_ortho(T.v64.p, T.vstride(), T.members.as<int>(), V2, bvol, T.nf, T.nvec, flag, st);
  int hflag = 0;
  HIPCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hflag) fail(WCMG_ERANK, "coarse-level null vectors are linearly dependent on a block");
  T.v32.alloc((size_t)T.nvec * T.vstride() * 8);
  launch_reals_convert(WCMG_F32, T.v32.p, T.v64.as<double>(), (size_t)T.nvec * T.vstride() * 2, st);
  T.orth = true;
  // Y9 column by column
  const int n1 = C1.cg.n, n2 = C2.cg.n;
  const size_t nn2 = (size_t)n2 * n2;
  C2.Y9.alloc((size_t)V2 * 9 * nn2 * 16);
  const size_t b1 = (size_t)V1 * n1 * 16;
  void* bucket[9];
  for (int k = 0; k < 9; ++k) bucket[k] = c.scratch_buf(20 + k, b1);
  void* vcol = c.scratch_buf(30, b1);
  void* u = c.scratch_buf(31, b1);
  void* e = c.scratch_buf(32, (size_t)V2 * n2 * 16);
  for (int j = 0; j < n2; ++j) {
    launch_unit_fill(e, V2, n2, j, st);
    launch_ctr_prolong(WCMG_F64, vcol, 0, e, 0, T.v64.p, T.vstride(), T.blk.as<int>(), V1, n1, T.nvec, 1, st);
    launch_coarse_local(WCMG_F64, u, vcol, C1.Xinv[0].p, -1, C1.cg, st);
    launch_chop_split(bucket, vcol, u, C1.Yhop[0].p, C1.nbr.as<int>(), T.blk.as<int>(), V1, n1, st);
    for (int slot = 0; slot < 9; ++slot) {
      void* out = (char*)C2.Y9.p + ((size_t)slot * n2 + j) * n2 * 16;
      launch_ctr_restrict(WCMG_F64, out, 9 * nn2, 0, bucket[slot], 0, T.v64.p, T.vstride(), T.members.as<int>(), V2,
                          bvol, n1, T.nvec, 1, st);
    }
  }
  finalize_coarse(c, C2, flag);
  C2.built = true;
  for (size_t l = level + 1; l < L.levels.size(); ++l) L.levels[l]->built = false;
  if (level + 1 == p.nlevels && p.coarsest == 1) build_dense(c, L, level);
  if (level + 1 == p.nlevels && p.coarsest == 2) build_deflation(c, L, level);
  L.mg.reset();
}

void mg_build_coarse(Ctx& c, LatticeState& L, int level) {
  if (level >= 1) return mg_build_coarse_next(c, L, level);
  if (level != 0) fail(WCMG_EINVAL, "level out of range");
  if (!L.F.have_clover) fail(WCMG_ESTATE, "clover not set");
  if (!L.have_params) fail(WCMG_ESTATE, "multigrid parameters not set");
  if (!L.T0.have_vecs) fail(WCMG_ESTATE, "null vectors not set");
  const wcmg_mg_params& p = L.params;
  const Geom& g = L.F.g;
  hipStream_t st = c.st;
  const int nvec = p.nvec[0];
  const size_t hb64 = spinor_bytes(WCMG_F64, g.Vh);
  const size_t hb32 = spinor_bytes(WCMG_F32, g.Vh);
  FineTransfer& T = L.T0;
  T.bg = make_block_geom(g.L, p.block[0]);
  T.nvec = nvec;
  // P: block x chirality orthonormalisation
  T.v64.alloc((size_t)nvec * 2 * hb64);
  HIPCHK(hipMemcpyAsync(T.v64.p, T.raw.p, (size_t)nvec * 2 * hb64, hipMemcpyDeviceToDevice, st));
  int* flag = (int*)c.scratch_buf(12, 64);
  HIPCHK(hipMemsetAsync(flag, 0, 64, st));
  launch_block_orthonormalize(T.v64.p, nvec, g, T.bg, flag, st);
  int hflag[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hflag[0]) fail(WCMG_ERANK, "null vectors are linearly dependent on a block");
  T.v32.alloc((size_t)nvec * 2 * hb32);
  for (int k = 0; k < 2 * nvec; ++k)
    spinor_convert(WCMG_F32, (char*)T.v32.p + (size_t)k * hb32, WCMG_F64, (const char*)T.v64.p + (size_t)k * hb64,
                   g.Vh, st);
  T.vbm32.alloc((size_t)nvec * 2 * hb32);
  launch_vec_blockmajor(T.vbm32.p, T.v32.p, nvec, g, T.bg, st);
  {
    // FP16 copies for the cycle's transfers (transfer_fp16): four halves per float4 chunk
    const size_t nch = (size_t)nvec * 2 * hb32 / 16;
    T.v16.alloc(nch * 8);
    T.vbm16.alloc(nch * 8);
    launch_chunks_to_half(T.v16.p, T.v32.p, nch, st);
    launch_chunks_to_half(T.vbm16.p, T.vbm32.p, nch, st);
  }
  T.orth = true;

  if (L.levels.empty()) L.levels.emplace_back(new CoarseLevel());
  CoarseLevel& C = *L.levels[0];
  C.bg = T.bg;
  C.nvec = nvec;
  C.cg = make_coarse_geom(T.bg, nvec);
  build_coarse_tables(C);
  const int n = C.cg.n, V = C.cg.V;
  const size_t nn = (size_t)n * n;
  C.Y9.alloc((size_t)V * 9 * nn * 16);

  FineOp op{&c, &L.F, WCMG_F64, &c.fw[0], st};
  void* bucket[9];
  for (int s = 0; s < 9; ++s) bucket[s] = c.scratch_buf(20 + s, 2 * hb64);
  void* vcol = c.scratch_buf(30, 2 * hb64);
  void* u = c.scratch_buf(31, 2 * hb64);
  for (int s = 0; s < 2; ++s)
    for (int k = 0; k < nvec; ++k) {
      const int j = s * nvec + k;
      const char* vk = (const char*)T.v64.p + (size_t)k * 2 * hb64;
      spinor_chiral_project(WCMG_F64, vcol, vk, g.Vh, s, st);
      spinor_chiral_project(WCMG_F64, (char*)vcol + hb64, vk + hb64, g.Vh, s, st);
      op.clover(u, vcol, 0, 1);
      op.clover((char*)u + hb64, (char*)vcol + hb64, 1, 1);
      launch_hop_split(bucket, vcol, u, L.F.gauge[WCMG_F64].p, g, T.bg, st);
      for (int slot = 0; slot < 9; ++slot) {
        void* out = (char*)C.Y9.p + ((size_t)slot * n + j) * n * 16;
        launch_restrict(WCMG_F64, out, 9 * nn, 1, bucket[slot], T.v64.p, nvec, 0, g, T.bg, false, st);
        launch_restrict(WCMG_F64, out, 9 * nn, 1, (char*)bucket[slot] + hb64, T.v64.p, nvec, 1, g, T.bg, true, st);
      }
    }
  finalize_coarse(c, C, flag);
  C.built = true;
  if (p.nlevels == 1 && p.coarsest == 1) build_dense(c, L, 0);
  if (p.nlevels == 1 && p.coarsest == 2) build_deflation(c, L, 0);
  L.mg.reset();
}

// ---------------------------------------------------------------------------
// adaptive refinement of the null vectors (Setup section: the alphaSA idea of
// relaxing with a cycle built from the vectors already available, and the
// hybrid of that with inverse iteration)
// ---------------------------------------------------------------------------
// With the hierarchy built from the current vectors, every fine null vector v
// is relaxed by `iters` steps of the multigrid-preconditioned GCR on the
// homogeneous reduced system D_r y = 0 started from y = v_e: the error that
// survives is what the present cycle resolves worst.  The odd half follows
// from D_p v = 0 (v_o = -H_oe A_ee^-1 v_e), the vectors are orthonormalised
// against each other (twice, in order), and P and the coarse operator are
// rebuilt; `passes` rounds.
void mg_refine_null_vectors(Ctx& c, LatticeState& L, int passes, int iters) {
  require_hierarchy(L);
  if (passes < 1 || iters < 1) fail(WCMG_EINVAL, "passes and iters must be >= 1");
  const wcmg_mg_params& p = L.params;
  const Geom& g = L.F.g;
  hipStream_t st = c.st;
  const int nvec = L.T0.nvec;
  const size_t hb = spinor_bytes(WCMG_F64, g.Vh);
  const size_t ne = (size_t)12 * g.Vh, nf = 2 * ne;
  FineOp op{&c, &L.F, WCMG_F64, &c.fw[0], st};
  void* zero = c.scratch_buf(53, hb);
  void* z = c.scratch_buf(54, hb);
  std::vector<double> cf(2 * nvec);
  for (int pass = 0; pass < passes; ++pass) {
    if (!L.mg) L.mg = std::make_shared<MGSolver>(c, L);
    MGSolver& mg = *L.mg;
    OpFn Dr = [&](void* o, const void* i) { op.Dr(o, i); };
    OpFn K = [&](void* o, const void* i) { mg.precondition(o, i); };
    GcrSpace& S64 = c.outer;
    S64.prec = WCMG_F64;
    S64.n = ne;
    S64.bytes = hb;
    blas_zero(WCMG_F64, zero, ne, st);
    std::vector<const void*> done;
    for (int k = 0; k < nvec; ++k) {
      char* v = (char*)L.T0.raw.p + (size_t)k * 2 * hb;
      gcr(c, S64, Dr, &K, v, zero, false, 0.0, 1.0, std::min(kMaxRestart, std::max(p.outer_restart, iters)), iters,
          true);
      mg.collect_device_stats();
      op.clover(z, v, 0, 1);                           // A_ee^-1 v_e
      op.hop(v + hb, z, nullptr, 1, 0, false, -1.0);   // v_o = -H_oe A_ee^-1 v_e
      for (int rep = 0; rep < 2 && k > 0; ++rep) {
        blas_multi_cdot(WCMG_F64, done.data(), k, v, nf, c.red.out(), st);
        const double* d = c.red.fetch(2 * k);
        for (int j = 0; j < 2 * k; ++j) cf[j] = -d[j];
        blas_multi_axpy(WCMG_F64, cf.data(), done.data(), k, v, nf, st);
      }
      const double nv = std::sqrt(norm2(c, WCMG_F64, v, nf));
      if (!(nv > 0.0) || !finite(nv)) fail(WCMG_ENAN, "refined null vector vanished");
      blas_axpby(WCMG_F64, 0.0, 0.0, v, 1.0 / nv, 0.0, v, nf, st);
      done.push_back(v);
    }
    HIPCHK(hipStreamSynchronize(st));
    L.T0.orth = false;
    for (auto& lv : L.levels) lv->built = false;
    L.mg.reset();
    for (int l = 0; l < p.nlevels; ++l) mg_build_coarse(c, L, l);
  }
}

// ---------------------------------------------------------------------------
// one right-hand side:  b_r (Eq.(4)), solve D_r y = b_r, reconstruct x
// ---------------------------------------------------------------------------
void solve_rhs(Ctx& c, LatticeState& L, int solver, void* x_e, void* x_o, const void* b_e, const void* b_o,
               bool x_zero, double tol, wcmg_stats* stats) {
  auto t0 = std::chrono::steady_clock::now();
  const Geom& g = L.F.g;
  hipStream_t st = c.st;
  const size_t hb = spinor_bytes(WCMG_F64, g.Vh);
  const size_t n = (size_t)12 * g.Vh;
  FineOp op{&c, &L.F, WCMG_F64, &c.fw[0], st};
  double bn2 = norm2(c, WCMG_F64, b_e, n) + norm2(c, WCMG_F64, b_o, n);
  wcmg_stats s{};
  if (!finite(bn2)) fail(WCMG_ENAN, "right-hand side is not finite");
  if (bn2 == 0.0) {
    blas_zero(WCMG_F64, x_e, n, st);
    blas_zero(WCMG_F64, x_o, n, st);
    if (stats) *stats = s;
    return;
  }
  const double bn = std::sqrt(bn2);
  void* br = c.scratch_buf(0, hb);
  void* y = c.scratch_buf(1, hb);
  op.reduced_source(br, b_e, b_o);
  if (!x_zero) op.clover(y, x_e, 0, 0);  // y_e = D_ee x_e
  OpFn Dr = [&](void* o, const void* i) { op.Dr(o, i); };
  const wcmg_mg_params& p = L.params;
  const int restart = L.have_params ? p.outer_restart : 16;
  const int maxiter = L.have_params ? p.outer_max_iter : 100000;
  // cap of the unpreconditioned solvers
  const int plain_cap = L.have_params && p.plain_max_iter > 0 ? p.plain_max_iter : 100000;
  KrylovResult kr;
  if (solver == WCMG_BICGSTAB) {
    if (x_zero) blas_zero(WCMG_F64, y, n, st);
    kr = bicgstab(c, WCMG_F64, n, Dr, y, br, tol, bn, plain_cap);
  } else if (solver == WCMG_MP_BICGSTAB) {
    int cycles = 0;
    const double itol = L.have_params && p.mp_inner_tol > 0 ? p.mp_inner_tol : 1e-3;
    kr = mp_bicgstab(c, L, y, br, x_zero, tol, bn, plain_cap, itol, &cycles);
    s.inner_iters[0] = cycles;
  } else if (solver == WCMG_CGNR) {
    kr = cgnr(c, L, y, br, x_zero, tol, bn, plain_cap);
  } else {
    GcrSpace& S64 = c.outer;
    S64.prec = WCMG_F64;
    S64.n = n;
    S64.bytes = hb;
    if (solver == WCMG_GCR) {
      kr = gcr(c, S64, Dr, nullptr, y, br, x_zero, tol, bn, restart, plain_cap);
    } else {
      require_hierarchy(L);
      if (!L.mg) L.mg = std::make_shared<MGSolver>(c, L);
      MGSolver& mg = *L.mg;
      mg.calls = 0;
      for (auto& lvl : mg.lv) lvl.calls = lvl.iters = 0;
      OpFn K = [&](void* o, const void* i) { mg.precondition(o, i); };
      kr = gcr(c, S64, Dr, &K, y, br, x_zero, tol, bn, restart, maxiter);
      s.inner_status = mg.collect_device_stats();
      for (size_t l = 0; l < mg.lv.size() && l < WCMG_MAX_LEVELS; ++l)
        s.inner_iters[l] = mg.lv[l].calls ? (double)mg.lv[l].iters / mg.lv[l].calls : 0.0;
    }
  }
  op.reconstruct(x_e, x_o, y, b_o);
  // true residual of the full system in FP64
  void* te = c.scratch_buf(2, hb);
  void* to = c.scratch_buf(3, hb);
  op.D(te, to, x_e, x_o);
  blas_axpby(WCMG_F64, 1.0, 0.0, b_e, -1.0, 0.0, te, n, st);
  blas_axpby(WCMG_F64, 1.0, 0.0, b_o, -1.0, 0.0, to, n, st);
  double rr = norm2(c, WCMG_F64, te, n) + norm2(c, WCMG_F64, to, n);
  s.iters = kr.iters;
  s.true_rel_res = std::sqrt(rr) / bn;
  s.status = kr.status;
  if (s.status == WCMG_OK && !(s.true_rel_res <= tol * 1.0000001)) s.status = WCMG_ENOCONV;
  s.t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = s;
}

// Multigrid solve of a batch of right-hand sides in lockstep: one FP64 outer
// GCR per right-hand side, every operator and preconditioner application done
// for the whole batch at once (links, clover and coarse matrices read once per
// kernel for all right-hand sides of a group).
void solve_batch(Ctx& c, LatticeState& L, void* x_e, void* x_o, const void* b_e, const void* b_o, int nrhs,
                 bool x_zero, double tol, wcmg_stats* stats) {
  auto t0 = std::chrono::steady_clock::now();
  if (nrhs < 1 || nrhs > kMaxBatch) fail(WCMG_EINVAL, "batch size out of range");
  require_hierarchy(L);
  const Geom& g = L.F.g;
  hipStream_t st = c.st;
  const size_t hb = spinor_bytes(WCMG_F64, g.Vh);
  const size_t n = (size_t)12 * g.Vh;
  FineOp op{&c, &L.F, WCMG_F64, &c.fw[0], st};
  std::vector<double> bn(nrhs);
  blas_norm2_b(WCMG_F64, b_e, n, n, nrhs, c.red.outb(c.red.dres(), 1), st);
  blas_norm2_b(WCMG_F64, b_o, n, n, nrhs, c.red.outb(c.red.dres() + 32, 1), st);
  {
    const double* h = c.red.fetch(64);
    for (int i = 0; i < nrhs; ++i) bn[i] = std::sqrt(h[i] + h[32 + i]);
  }
  for (int i = 0; i < nrhs; ++i)
    if (!finite(bn[i])) fail(WCMG_ENAN, "right-hand side is not finite");
  void* br = c.scratch_buf(0, hb * nrhs);
  void* y = c.scratch_buf(1, hb * nrhs);
  op.reduced_source(br, b_e, b_o, nrhs);
  if (!x_zero) op.clover(y, x_e, 0, 0, nrhs);  // y_e = D_ee x_e
  const wcmg_mg_params& p = L.params;
  if (!L.mg) L.mg = std::make_shared<MGSolver>(c, L);
  MGSolver& mg = *L.mg;
  mg.calls = 0;
  for (auto& lvl : mg.lv) lvl.calls = lvl.iters = 0;
  OpFn Dr = [&](void* o, const void* i) { op.Dr(o, i, nrhs); };
  OpFn K = [&](void* o, const void* i) { mg.precondition_b(o, i, nrhs); };
  GcrSpaceB& outer = c.outer_b;
  outer.prec = WCMG_F64;
  outer.n = n;
  outer.vs = n;
  outer.nrhs = nrhs;
  // a zero right-hand side has a zero solution; give it a unit target so the
  // batch does not wait for it
  std::vector<double> tn(bn);
  for (double& v : tn)
    if (v == 0.0) v = 1.0;
  std::vector<KrylovResult> kr = gcr_b(c, outer, Dr, &K, y, br, x_zero, tol, tn.data(), p.outer_restart,
                                       p.outer_max_iter);
  const int inner_status = mg.collect_device_stats();
  op.reconstruct(x_e, x_o, y, b_o, nrhs);
  // true residuals of the full system in FP64
  void* te = c.scratch_buf(2, hb * nrhs);
  void* to = c.scratch_buf(3, hb * nrhs);
  op.D(te, to, x_e, x_o, nrhs);
  blas_axpby(WCMG_F64, 1.0, 0.0, b_e, -1.0, 0.0, te, n * nrhs, st);
  blas_axpby(WCMG_F64, 1.0, 0.0, b_o, -1.0, 0.0, to, n * nrhs, st);
  blas_norm2_b(WCMG_F64, te, n, n, nrhs, c.red.outb(c.red.dres(), 1), st);
  blas_norm2_b(WCMG_F64, to, n, n, nrhs, c.red.outb(c.red.dres() + 32, 1), st);
  const double* h = c.red.fetch(64);
  const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int i = 0; i < nrhs; ++i) {
    wcmg_stats s{};
    s.iters = kr[i].iters;
    s.status = kr[i].status;
    s.inner_status = inner_status;
    s.true_rel_res = bn[i] > 0 ? std::sqrt(h[i] + h[32 + i]) / bn[i] : 0.0;
    for (size_t l = 0; l < mg.lv.size() && l < WCMG_MAX_LEVELS; ++l)
      s.inner_iters[l] = mg.lv[l].calls ? (double)mg.lv[l].iters / mg.lv[l].calls : 0.0;
    if (s.status == WCMG_OK && !(s.true_rel_res <= tol * 1.0000001)) s.status = WCMG_ENOCONV;
    s.t_solve_s = dt;
    if (stats) stats[i] = s;
  }
}

}  // namespace wcmg
