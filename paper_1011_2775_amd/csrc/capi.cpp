// C ABI of the wcmg library: argument validation, canonical <-> internal
// layout conversion, and dispatch to the runtime.  No exception crosses the
// boundary; every entry point returns a status code.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "random.h"
#include "runtime.h"

using namespace wcmg;

namespace {

thread_local std::string g_err;

int set_err(int code, const std::string& m) {
  g_err = m;
  return code;
}

template <typename F>
int guarded(F&& f) {
  try {
    f();
    return WCMG_OK;
  } catch (const Error& e) {
    return set_err(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return set_err(WCMG_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return set_err(WCMG_EINVAL, e.what());
  } catch (...) {
    return set_err(WCMG_EINVAL, "unknown error");
  }
}

#define CHECK(cond, code, msg) \
  do {                         \
    if (!(cond)) return set_err((code), (msg)); \
  } while (0)

Ctx* as_ctx(void* p) { return reinterpret_cast<Ctx*>(p); }

bool valid_prec(int p) { return p == WCMG_F64 || p == WCMG_F32 || p == WCMG_F16; }
bool valid_op(int o) { return o == WCMG_OP_FULL || o == WCMG_OP_SCHUR || o == WCMG_OP_DP || o == WCMG_OP_SCHUR_X; }

// copies `bytes` of host or device data into a device scratch slot
const void* to_device(Ctx& c, int slot, const void* src, size_t bytes, int on_device) {
  if (on_device) return src;
  void* d = c.scratch_buf(slot, bytes);
  HIPCHK(hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, c.st));
  return d;
}

// per plane: csw_s on the spatial planes, csw_t on the planes with time
CloverCoef clover_coef(double csw_s, double csw_t) {
  // chiral gamma basis: gamma_k = [[0,-i s_k],[i s_k,0]], gamma_4 = [[0,1],[1,0]]
  typedef double cd[2];
  auto cm = [](const cd a, const cd b, cd o) {
    o[0] = a[0] * b[0] - a[1] * b[1];
    o[1] = a[0] * b[1] + a[1] * b[0];
  };
  static const double sig[3][2][2][2] = {{{{0, 0}, {1, 0}}, {{1, 0}, {0, 0}}},
                                         {{{0, 0}, {0, -1}}, {{0, 1}, {0, 0}}},
                                         {{{1, 0}, {0, 0}}, {{0, 0}, {-1, 0}}}};
  double G[4][4][4][2];
  std::memset(G, 0, sizeof(G));
  for (int k = 0; k < 3; ++k)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        // upper-right block -i sigma_k, lower-left i sigma_k
        const double* s = sig[k][a][b];
        G[k][a][2 + b][0] = s[1];
        G[k][a][2 + b][1] = -s[0];
        G[k][2 + a][b][0] = -s[1];
        G[k][2 + a][b][1] = s[0];
      }
  for (int a = 0; a < 2; ++a) {
    G[3][a][2 + a][0] = 1;
    G[3][2 + a][a][0] = 1;
  }
  CloverCoef cc;
  int plane = 0;
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = mu + 1; nu < 4; ++nu, ++plane) {
      const double csw = nu == 3 ? csw_t : csw_s;
      // sigma = (i/2)(g_mu g_nu - g_nu g_mu); coefficient csw (i/2) -> -csw/4 (g g - g g)
      double C[4][4][2];
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          double s1[2] = {0, 0}, s2[2] = {0, 0};
          for (int k = 0; k < 4; ++k) {
            double t[2];
            cm(G[mu][i][k], G[nu][k][j], t);
            s1[0] += t[0];
            s1[1] += t[1];
            cm(G[nu][i][k], G[mu][k][j], t);
            s2[0] += t[0];
            s2[1] += t[1];
          }
          C[i][j][0] = -0.25 * csw * (s1[0] - s2[0]);
          C[i][j][1] = -0.25 * csw * (s1[1] - s2[1]);
        }
      for (int chi = 0; chi < 2; ++chi)
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) {
            cc.s[plane][chi][a * 2 + b][0] = C[2 * chi + a][2 * chi + b][0];
            cc.s[plane][chi][a * 2 + b][1] = C[2 * chi + a][2 * chi + b][1];
          }
    }
  return cc;
}

// A buffer the header marks "device" must be device (or managed) memory of
// the context's GPU, with at least `bytes` bytes from p to the end of its
// allocation; anything else (a host pointer, another GPU's memory, a buffer
// too short for the shape the call implies) is rejected before any launch.
int check_dev(Ctx* c, const void* p, size_t bytes, const char* what) {
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return set_err(WCMG_EINVAL, std::string(what) + ": not a device pointer");
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
    return set_err(WCMG_EINVAL, std::string(what) + ": host memory where device memory is required");
  if (at.device != c->device)
    return set_err(WCMG_EINVAL, std::string(what) + ": memory of another device than the context's");
  void* base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) == hipSuccess && base) {
    if ((const char*)p + bytes > (const char*)base + size)
      return set_err(WCMG_EINVAL, std::string(what) + ": device buffer shorter than the call requires");
  } else {
    (void)hipGetLastError();
  }
  return WCMG_OK;
}
#define CHECK_DEV(c, p, bytes, what) \
  do {                               \
    if (int r_ = check_dev((c), (p), (bytes), (what))) return r_; \
  } while (0)

int check_lat(Ctx* c, int lat) {
  if (!c) return set_err(WCMG_EINVAL, "null context");
  if (lat < 0 || lat >= (int)c->lats.size()) return set_err(WCMG_EINVAL, "lattice index out of range");
  return WCMG_OK;
}

}  // namespace

extern "C" {

const char* wcmg_last_error(void) { return g_err.c_str(); }

int wcmg_mg_params_default(wcmg_mg_params* p) {
  CHECK(p, WCMG_EINVAL, "null params");
  std::memset(p, 0, sizeof(*p));
  p->nlevels = 1;
  for (int l = 0; l < WCMG_MAX_LEVELS; ++l) {
    for (int k = 0; k < 4; ++k) p->block[l][k] = l == 0 ? 4 : 2;
    p->nvec[l] = l == 0 ? 24 : 32;
    p->tol[l] = 0.1;
    p->max_iter[l] = 50;
    p->restart[l] = 10;
  }
  p->nu_post = 4;
  p->outer_restart = 16;
  p->outer_max_iter = 1000;
  p->smoother_prec = WCMG_F32;
  p->setup_prec = WCMG_F32;
  p->setup_relax = 10;
  p->setup_max_steps = 10;
  p->setup_rq_tol = 0.05;
  p->seed = 0;
  p->coarsest = 0;
  return WCMG_OK;
}

int wcmg_create(const wcmg_lattice* lats, int nlat, void* hip_stream, void** out) {
  CHECK(out, WCMG_EINVAL, "null output handle");
  *out = nullptr;
  CHECK(lats && nlat > 0, WCMG_EINVAL, "need at least one lattice");
  for (int l = 0; l < nlat; ++l) {
    for (int k = 0; k < 4; ++k) {
      int L = lats[l].dims[k];
      CHECK(L >= 2 && L % 2 == 0, WCMG_EDIM, "lattice extents must be even and >= 2");
    }
    CHECK(lats[l].t_bc == 1 || lats[l].t_bc == -1, WCMG_EINVAL, "t_bc must be +1 or -1");
    double v = 1;
    for (int k = 0; k < 4; ++k) v *= lats[l].dims[k];
    CHECK(v < 2.0e9, WCMG_EDIM, "lattice too large");
  }
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return set_err(WCMG_ENODEV, "no HIP device available");
  }
  return guarded([&] {
    auto c = new Ctx();
    try {
      HIPCHK(hipGetDevice(&c->device));
      c->st = reinterpret_cast<hipStream_t>(hip_stream);
      c->timer.st = c->st;
      c->red.init(c->st);
      (void)noalloc_scratch(c->device);  // the allocation-free entry point's array on this GPU
      for (int l = 0; l < nlat; ++l) {
        auto L = new LatticeState();
        L->F.g = make_geom(lats[l].dims, lats[l].t_bc);
        c->lats.emplace_back(L);
      }
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
  });
}

int wcmg_destroy(void* ctx) {
  CHECK(ctx, WCMG_EINVAL, "null context");
  return guarded([&] {
    Ctx* c = as_ctx(ctx);
    (void)hipStreamSynchronize(c->st);
    delete c;
  });
}

int wcmg_set_gauge(void* ctx, int lat, const void* U, int on_device) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  CHECK(U, WCMG_EINVAL, "null gauge field");
  if (on_device) CHECK_DEV(c, U, (size_t)c->lats[lat]->F.g.V * 4 * 9 * 16, "gauge field");
  return guarded([&] {
    LatticeState& L = *c->lats[lat];
    const Geom& g = L.F.g;
    const void* src = to_device(*c, 40, U, (size_t)g.V * 4 * 9 * 16, on_device);
    for (int p = 0; p < 3; ++p) {
      L.F.gauge[p].alloc(gauge_bytes(p, g.V));
      gauge_to_internal(p, L.F.gauge[p].p, src, g, c->st);
    }
    HIPCHK(hipStreamSynchronize(c->st));
    L.F.have_gauge = true;
    L.F.have_clover = false;
    L.clear_hierarchy();
  });
}

static int set_clover_impl(void* ctx, int lat, double m0, double hop_s, double csw, double csw_t, const void* A,
                           int on_device) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  CHECK(std::isfinite(m0) && std::isfinite(csw) && std::isfinite(csw_t), WCMG_EINVAL,
        "m0 and the clover coefficients must be finite");
  CHECK(std::isfinite(hop_s) && hop_s > 0.0, WCMG_EINVAL, "the spatial hop coefficient must be positive");
  CHECK(!A || hop_s == 1.0, WCMG_EINVAL, "a caller-supplied clover matrix goes with isotropic hops");
  LatticeState& L = *c->lats[lat];
  CHECK(A || L.F.have_gauge, WCMG_ESTATE, "gauge field not set");
  if (A && on_device) CHECK_DEV(c, A, (size_t)L.F.g.V * 144 * 16, "clover matrix");
  return guarded([&] {
    const Geom& g = L.F.g;
    DBuf c64;
    c64.alloc(clover_bytes(WCMG_F64, g.V));
    int* flag = (int*)c->scratch_buf(12, 64);
    HIPCHK(hipMemsetAsync(flag, 0, 64, c->st));
    if (A) {
      const void* src = to_device(*c, 40, A, (size_t)g.V * 144 * 16, on_device);
      clover_from_matrix(c64.p, src, g, flag, c->st);
    } else {
      Geom ga = L.F.g;
      ga.hs = hop_s;
      clover_compute(c64.p, L.F.gauge[WCMG_F64].p, ga, m0, clover_coef(csw, csw_t), flag, c->st);
    }
    int hf = 0;
    HIPCHK(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (hf) fail(WCMG_ECLOVER_NOT_PD, "clover block not positive definite");
    size_t nreal = (size_t)g.V * 144;
    L.F.clov[WCMG_F64] = std::move(c64);
    for (int p = 1; p < 3; ++p) {
      L.F.clov[p].alloc(clover_bytes(p, g.V));
      clover_relayout(p, L.F.clov[p].p, L.F.clov[WCMG_F64].as<double>(), g.Vh, c->st);
    }
    HIPCHK(hipStreamSynchronize(c->st));
    L.F.g.hs = A ? 1.0 : hop_s;  // the spatial hops of every kernel on this lattice from now on
    L.F.m0 = m0;
    L.F.csw = csw;
    L.F.csw_t = csw_t;
    L.F.clover_from_u = (A == nullptr);
    L.F.have_clover = true;
    L.mg.reset();  // the preconditioner (and any captured graph) holds the old clover
    for (auto& lv : L.levels) lv->built = false;
    L.mg.reset();
  });
}

int wcmg_set_clover(void* ctx, int lat, double m0, double csw, const void* A, int on_device) {
  return set_clover_impl(ctx, lat, m0, 1.0, csw, csw, A, on_device);
}

int wcmg_set_clover_aniso(void* ctx, int lat, double m0, double hop_s, double csw_s, double csw_t) {
  return set_clover_impl(ctx, lat, m0, hop_s, csw_s, csw_t, nullptr, 1);
}

int wcmg_set_mg_params(void* ctx, int lat, const wcmg_mg_params* p) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  CHECK(p, WCMG_EINVAL, "null params");
  CHECK(p->nlevels >= 1 && p->nlevels <= WCMG_MAX_LEVELS, WCMG_EINVAL, "nlevels out of range");
  CHECK(p->nlevels <= WCMG_MAX_LEVELS - 1, WCMG_EINVAL,
        "at most three coarse levels (nvec[nlevels] holds the deflation count)");
  LatticeState& L = *c->lats[lat];
  const Geom& g = L.F.g;
  for (int k = 0; k < 4; ++k) {
    int b = p->block[0][k];
    CHECK(b >= 2 && b % 2 == 0, WCMG_EDIM, "block extents must be even and >= 2");
    CHECK(g.L[k] % b == 0, WCMG_EDIM, "block does not divide the lattice");
  }
  int bvol = p->block[0][0] * p->block[0][1] * p->block[0][2] * p->block[0][3];
  CHECK(bvol <= 1024, WCMG_EDIM, "block volume above 1024");
  CHECK(p->nvec[0] >= 1 && p->nvec[0] <= 64, WCMG_EDIM, "nvec must be in 1..64");
  CHECK(p->nvec[0] <= 6 * bvol, WCMG_EDIM, "nvec exceeds the block's degrees of freedom per chirality");
  CHECK(p->tol[0] > 0 && p->tol[0] < 1, WCMG_EINVAL, "inner tolerance must be in (0,1)");
  CHECK(p->max_iter[0] >= 1 && p->restart[0] >= 1, WCMG_EINVAL, "inner max_iter and restart must be >= 1");
  CHECK(p->outer_restart >= 1 && p->outer_max_iter >= 1, WCMG_EINVAL, "outer restart and max_iter must be >= 1");
  CHECK(p->outer_restart <= 64 && p->restart[0] <= 64 && p->setup_relax <= 64, WCMG_EINVAL,
        "restart lengths are limited to 64");
  CHECK(p->nu_post >= 0, WCMG_EINVAL, "nu_post must be >= 0");
  CHECK(p->smoother_prec == WCMG_F64 || p->smoother_prec == WCMG_F32 || p->smoother_prec == WCMG_F16, WCMG_EINVAL,
        "smoother precision must be F64, F32 or F16 (FP16 fields, FP32 arithmetic)");
  CHECK(p->setup_relax >= 1 && p->setup_max_steps >= 1, WCMG_EINVAL, "setup iteration counts must be >= 1");
  CHECK(p->coarsest >= 0 && p->coarsest <= 2, WCMG_EINVAL,
        "coarsest must be 0 (GCR), 1 (dense FP64 inverse) or 2 (deflated FP64 GCR)");
  CHECK(p->cycle_mode >= 0 && p->cycle_mode <= 3, WCMG_EINVAL, "cycle_mode must be 0, 1, 2 or 3");
  CHECK(p->coarse_launch >= 0 && p->coarse_launch <= 2, WCMG_EINVAL, "coarse_launch must be 0, 1 or 2");
  CHECK(p->coarse_fp16 == 0 || p->coarse_fp16 == 1, WCMG_EINVAL, "coarse_fp16 must be 0 or 1");
  CHECK(p->transfer_fp16 == 0 || p->transfer_fp16 == 1, WCMG_EINVAL, "transfer_fp16 must be 0 or 1");
  CHECK(p->plain_max_iter >= 0, WCMG_EINVAL, "plain_max_iter must be >= 0");
  CHECK(p->mp_inner_tol >= 0 && p->mp_inner_tol < 1, WCMG_EINVAL, "mp_inner_tol must be in [0,1)");
  CHECK(p->setup_prec == WCMG_F64 || p->setup_prec == WCMG_F32 || p->setup_prec == WCMG_F16, WCMG_EINVAL,
        "setup precision must be F64, F32 or F16 (FP16 fields, FP32 arithmetic)");
  // coarse extents and degrees of freedom of every level
  int ext[4], nf = 2 * p->nvec[0];
  for (int k = 0; k < 4; ++k) ext[k] = g.L[k] / p->block[0][k];
  long vc = (long)ext[0] * ext[1] * ext[2] * ext[3];
  for (int l = 1; l < p->nlevels; ++l) {
    long bv = 1;
    for (int k = 0; k < 4; ++k) {
      int b = p->block[l][k];
      CHECK(b >= 1 && ext[k] % b == 0, WCMG_EDIM, "coarse block does not divide the coarse lattice");
      ext[k] /= b;
      bv *= b;
    }
    CHECK(bv >= 2 && bv <= 1024, WCMG_EDIM, "coarse block volume must be in 2..1024");
    CHECK(p->nvec[l] >= 1 && p->nvec[l] <= 64, WCMG_EDIM, "nvec must be in 1..64");
    CHECK(p->nvec[l] <= bv * (nf / 2), WCMG_EDIM, "nvec exceeds the block's degrees of freedom per chirality");
    CHECK(p->tol[l] > 0 && p->tol[l] < 1, WCMG_EINVAL, "inner tolerance must be in (0,1)");
    CHECK(p->max_iter[l] >= 1 && p->restart[l] >= 1 && p->restart[l] <= 64, WCMG_EINVAL,
          "inner max_iter and restart must be >= 1 (restart <= 64)");
    vc = (long)ext[0] * ext[1] * ext[2] * ext[3];
    nf = 2 * p->nvec[l];
  }
  if (p->coarsest == 1)
    CHECK(vc * nf <= kMaxDense, WCMG_EDIM, "coarsest level too large for the dense solve");
  if (p->coarsest == 2) {
    const int K = p->nvec[p->nlevels];
    CHECK(K >= 1 && K <= 48, WCMG_EINVAL, "deflation vectors (nvec[nlevels]) must be in 1..48");
    CHECK(K + p->restart[p->nlevels - 1] <= 64, WCMG_EINVAL,
          "deflation vectors plus the coarsest restart length must not exceed 64");
    CHECK((long)K * 4 <= vc * nf, WCMG_EDIM, "too many deflation vectors for the coarsest dimension");
  }
  return guarded([&] {
    bool same_shape = L.have_params && L.params.nlevels == p->nlevels;
    for (int l = 0; same_shape && l < p->nlevels; ++l)
      same_shape = L.params.nvec[l] == p->nvec[l] &&
                   std::memcmp(L.params.block[l], p->block[l], sizeof(p->block[l])) == 0;
    const bool same_coarsest = L.have_params && L.params.coarsest == p->coarsest &&
                               (p->coarsest != 2 || L.params.nvec[p->nlevels] == p->nvec[p->nlevels]);
    L.params = *p;
    L.have_params = true;
    if (!same_shape) {
      L.clear_hierarchy();
    } else if (!same_coarsest) {
      L.dense.release();
      L.dense_n = 0;
      L.defl_k = 0;
      for (auto& lv : L.levels) lv->built = false;
    }
    L.mg.reset();
  });
}

static int check_level(Ctx* c, int lat, int level) {
  LatticeState& L = *c->lats[lat];
  CHECK(L.have_params, WCMG_ESTATE, "multigrid parameters not set");
  CHECK(level >= 0 && level < L.params.nlevels, WCMG_EINVAL, "level out of range");
  return WCMG_OK;
}

int wcmg_build_null_vectors(void* ctx, int lat, int level) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  if (int r = check_level(c, lat, level)) return r;
  return guarded([&] { mg_setup_null_vectors(*c, *c->lats[lat], level); });
}

int wcmg_set_null_vectors(void* ctx, int lat, int level, const void* v, int nvec, int on_device) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  CHECK(v, WCMG_EINVAL, "null vectors pointer");
  if (int r = check_level(c, lat, level)) return r;
  LatticeState& L = *c->lats[lat];
  CHECK(nvec == L.params.nvec[level], WCMG_EINVAL, "nvec differs from the parameters");
  if (level >= 1) {
    CHECK((int)L.levels.size() >= level && L.levels[level - 1]->built, WCMG_ESTATE, "coarse level not built");
    if (on_device)
      CHECK_DEV(c, v, (size_t)nvec * L.levels[level - 1]->cg.V * L.levels[level - 1]->cg.n * 16, "null vectors");
    return guarded([&] {
      CoarseLevel& C1 = *L.levels[level - 1];
      const size_t one = (size_t)C1.cg.V * C1.cg.n * 16;
      while ((int)L.ctr.size() < level) L.ctr.emplace_back(new CoarseTransfer());
      CoarseTransfer& T = *L.ctr[level - 1];
      T.nf = C1.cg.n;
      T.nsites = C1.cg.V;
      T.raw.alloc((size_t)nvec * one);
      for (int k = 0; k < nvec; ++k) {
        const void* src = to_device(*c, 41, (const char*)v + (size_t)k * one, one, on_device);
        launch_coarse_canon(WCMG_F64, (char*)T.raw.p + (size_t)k * one, const_cast<void*>(src), C1.perm.as<int>(),
                            C1.cg.V, C1.cg.n, true, c->st);
        if (!on_device) HIPCHK(hipStreamSynchronize(c->st));
      }
      HIPCHK(hipStreamSynchronize(c->st));
      T.nvec = nvec;
      T.have_vecs = true;
      T.orth = false;
      for (size_t l = level; l < L.levels.size(); ++l) L.levels[l]->built = false;
      L.dense_n = 0;
      L.mg.reset();
    });
  }
  if (on_device) CHECK_DEV(c, v, (size_t)nvec * L.F.g.V * 12 * 16, "null vectors");
  return guarded([&] {
    const Geom& g = L.F.g;
    const size_t hb = spinor_bytes(WCMG_F64, g.Vh);
    const size_t one = (size_t)g.V * 12 * 16;
    L.T0.raw.alloc((size_t)nvec * 2 * hb);
    for (int k = 0; k < nvec; ++k) {
      const void* src = to_device(*c, 41, (const char*)v + (size_t)k * one, one, on_device);
      char* dst = (char*)L.T0.raw.p + (size_t)k * 2 * hb;
      spinor_to_internal(WCMG_F64, dst, dst + hb, src, g, false, c->st);
      if (!on_device) HIPCHK(hipStreamSynchronize(c->st));
    }
    HIPCHK(hipStreamSynchronize(c->st));
    L.T0.nvec = nvec;
    L.T0.have_vecs = true;
    L.T0.orth = false;
    for (auto& lv : L.levels) lv->built = false;
    L.mg.reset();
  });
}

int wcmg_get_null_vectors(void* ctx, int lat, int level, void* v, int on_device) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  CHECK(v, WCMG_EINVAL, "null vectors pointer");
  if (int r = check_level(c, lat, level)) return r;
  LatticeState& L = *c->lats[lat];
  if (level >= 1) {
    CHECK((int)L.ctr.size() >= level && L.ctr[level - 1]->have_vecs && (int)L.levels.size() >= level, WCMG_ESTATE,
          "null vectors not available");
    if (on_device)
      CHECK_DEV(c, v, (size_t)L.ctr[level - 1]->nvec * L.levels[level - 1]->cg.V * L.levels[level - 1]->cg.n * 16,
                "null vectors");
    return guarded([&] {
      CoarseLevel& C1 = *L.levels[level - 1];
      CoarseTransfer& T = *L.ctr[level - 1];
      const size_t one = (size_t)C1.cg.V * C1.cg.n * 16;
      for (int k = 0; k < T.nvec; ++k) {
        void* dst = on_device ? (char*)v + (size_t)k * one : c->scratch_buf(41, one);
        launch_coarse_canon(WCMG_F64, (char*)T.raw.p + (size_t)k * one, dst, C1.perm.as<int>(), C1.cg.V, C1.cg.n,
                            false, c->st);
        if (!on_device)
          HIPCHK(hipMemcpyAsync((char*)v + (size_t)k * one, dst, one, hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
      }
    });
  }
  CHECK(L.T0.have_vecs, WCMG_ESTATE, "null vectors not available");
  if (on_device) CHECK_DEV(c, v, (size_t)L.T0.nvec * L.F.g.V * 12 * 16, "null vectors");
  return guarded([&] {
    const Geom& g = L.F.g;
    const size_t hb = spinor_bytes(WCMG_F64, g.Vh);
    const size_t one = (size_t)g.V * 12 * 16;
    for (int k = 0; k < L.T0.nvec; ++k) {
      const char* src = (const char*)L.T0.raw.p + (size_t)k * 2 * hb;
      void* dst = on_device ? (char*)v + (size_t)k * one : c->scratch_buf(41, one);
      spinor_from_internal(WCMG_F64, dst, src, src + hb, g, false, c->st);
      if (!on_device)
        HIPCHK(hipMemcpyAsync((char*)v + (size_t)k * one, dst, one, hipMemcpyDeviceToHost, c->st));
    }
    HIPCHK(hipStreamSynchronize(c->st));
  });
}

int wcmg_setup_start_vectors(void* ctx, int lat, int level, uint64_t seed, int k0, int nvec, void* out) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  CHECK(out, WCMG_EINVAL, "null output");
  CHECK(k0 >= 0 && nvec >= 1, WCMG_EINVAL, "k0 must be >= 0 and nvec >= 1");
  LatticeState& L = *c->lats[lat];
  const Geom& g = L.F.g;
  if (level == 0) {
    CHECK_DEV(c, out, (size_t)nvec * g.V * 12 * 16, "start vectors");
    return guarded([&] {
      const size_t hb = spinor_bytes(WCMG_F64, g.Vh);
      char* v = (char*)c->scratch_buf(41, 2 * hb);
      for (int k = 0; k < nvec; ++k) {
        random_fine_vector(v, seed, k0 + k, 0, g, c->st);
        spinor_from_internal(WCMG_F64, (char*)out + (size_t)k * g.V * 12 * 16, v, v + hb, g, false, c->st);
      }
    });
  }
  CHECK(level >= 1 && (int)L.levels.size() >= level && L.levels[level - 1]->built, WCMG_ESTATE,
        "coarse level not built");
  const CoarseLevel& C = *L.levels[level - 1];
  CHECK_DEV(c, out, (size_t)nvec * C.cg.V * C.cg.n * 16, "start vectors");
  return guarded([&] {
    const size_t one = (size_t)C.cg.V * C.cg.n * 16;
    void* v = c->scratch_buf(41, one);
    for (int k = 0; k < nvec; ++k) {
      random_coarse_vector(v, seed, k0 + k, level, C.perm.as<int>(), C.cg.V, C.cg.n, c->st);
      launch_coarse_canon(WCMG_F64, v, (char*)out + (size_t)k * one, C.perm.as<int>(), C.cg.V, C.cg.n, false, c->st);
    }
  });
}

int wcmg_refine_null_vectors(void* ctx, int lat, int passes, int iters) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  CHECK(passes >= 1 && iters >= 1 && iters <= 1000, WCMG_EINVAL, "passes must be >= 1 and iters in 1..1000");
  LatticeState& L = *c->lats[lat];
  CHECK(L.have_params && !L.levels.empty() && L.levels[0]->built && L.T0.have_vecs, WCMG_ESTATE,
        "multigrid hierarchy not built");
  return guarded([&] { mg_refine_null_vectors(*c, L, passes, iters); });
}

int wcmg_build_coarse(void* ctx, int lat, int level) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  if (int r = check_level(c, lat, level)) return r;
  return guarded([&] { mg_build_coarse(*c, *c->lats[lat], level); });
}

int wcmg_get_coarse(void* ctx, int lat, int level, void* Y, int on_device) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  CHECK(Y, WCMG_EINVAL, "null output");
  if (int r = check_level(c, lat, level)) return r;
  LatticeState& L = *c->lats[lat];
  CHECK((int)L.levels.size() > level && L.levels[level]->built, WCMG_ESTATE, "coarse operator not built");
  if (on_device)
    CHECK_DEV(c, Y, (size_t)L.levels[level]->cg.V * 9 * L.levels[level]->cg.n * L.levels[level]->cg.n * 16,
              "coarse operator");
  return guarded([&] {
    CoarseLevel& C = *L.levels[level];
    const int n = C.cg.n, V = C.cg.V;
    const size_t nn = (size_t)n * n;
    std::vector<double> h((size_t)V * 9 * nn * 2), o(h.size());
    HIPCHK(hipMemcpyAsync(h.data(), C.Y9.p, h.size() * 8, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    for (int l = 0; l < V; ++l) {
      const int ci = C.perm_host[l];
      for (int s = 0; s < 9; ++s)
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) {
            size_t src = (((size_t)ci * 9 + s) * n + j) * n + i;  // column-major
            size_t dst = (((size_t)l * 9 + s) * n + i) * n + j;   // row-major
            o[2 * dst] = h[2 * src];
            o[2 * dst + 1] = h[2 * src + 1];
          }
    }
    if (on_device)
      HIPCHK(hipMemcpyAsync(Y, o.data(), o.size() * 8, hipMemcpyHostToDevice, c->st));
    else
      std::memcpy(Y, o.data(), o.size() * 8);
    HIPCHK(hipStreamSynchronize(c->st));
  });
}

// Every lattice of the context at once (lat = -1): buffers hold, in lattice
// order, nrhs canonical spinors of each lattice; for each right-hand side
// every kernel of the operator is one launch over all lattices (a work list
// of per-lattice block ranges).  D^dag = gamma5 D gamma5 and
// D_r^dag = gamma5 (1 - A_ee^-1 H_eo A_oo^-1 H_oe) gamma5 (red-black
// paragraph, with the gamma5-hermiticity of Eq.(1)); D_p = D A^-1 and
// D_p^dag = A^-1 gamma5 D gamma5.
static int apply_all_lattices(Ctx* c, int op, int prec, void* out, const void* in, int nrhs, bool dag) {
  const int nl = (int)c->lats.size();
  CHECK(nl <= kMaxMulti, WCMG_EINVAL, "too many lattices for one launch");
  for (auto& L : c->lats) CHECK(L->F.have_clover, WCMG_ESTATE, "clover not set");
  size_t total = 0;
  for (auto& L : c->lats) total += (size_t)nrhs * L->F.g.V * 12 * 16;
  CHECK_DEV(c, in, total, "input spinors");
  CHECK_DEV(c, out, total, "output spinors");
  return guarded([&] {
    std::vector<char*> ie(nl), io(nl), oe(nl), oo(nl), t1(nl), t2(nl);
    std::vector<size_t> off(nl + 1, 0);
    for (int l = 0; l < nl; ++l) {
      const Geom& g = c->lats[l]->F.g;
      const size_t hb = spinor_bytes(prec, g.Vh);
      char** bufs[6] = {&ie[l], &io[l], &oe[l], &oo[l], &t1[l], &t2[l]};
      for (int k = 0; k < 6; ++k) *bufs[k] = (char*)c->scratch_buf(60 + 6 * l + k, hb);
      off[l + 1] = off[l] + (size_t)nrhs * g.V * 12 * 16;
    }
    auto args = [&](int l, void* o, const void* i, const void* x, int parity, double coeff) {
      FineFields& F = c->lats[l]->F;
      DslashArgs a;
      a.out = o;
      a.in = i;
      a.x = x;
      a.gauge = F.gauge[prec].p;
      a.clov = F.clov[prec].p;
      a.g = dgeom(F.g);
      a.parity = parity;
      a.nblocks = 0;
      a.coeff = coeff;
      return a;
    };
    auto clover_all = [&](std::vector<char*>& o, std::vector<char*>& i, int parity) {
      CloverMulti cm{};
      cm.nl = nl;
      cm.parity = parity;
      cm.kind = 1;
      for (int l = 0; l < nl; ++l) {
        cm.out[l] = o[l];
        cm.in[l] = i[l];
        cm.clov[l] = c->lats[l]->F.clov[prec].p;
        cm.Vh[l] = c->lats[l]->F.g.Vh;
      }
      launch_clover_multi(prec, cm, c->st);  // A_p^-1 on parity p
    };
    DslashMulti m{};
    m.nl = nl;
    // input converted with gamma5 for the adjoint of FULL and DP; output flipped for FULL
    const bool g5_in = dag && op != WCMG_OP_SCHUR, g5_out = dag && (op == WCMG_OP_FULL || op == WCMG_OP_SCHUR_X);
    for (int r = 0; r < nrhs; ++r) {
      for (int l = 0; l < nl; ++l) {
        const Geom& g = c->lats[l]->F.g;
        spinor_to_internal(prec, ie[l], io[l], (const char*)in + off[l] + (size_t)r * g.V * 12 * 16, g, g5_in,
                           c->st);
        if (dag && op == WCMG_OP_SCHUR) spinor_gamma5(prec, ie[l], g.Vh, c->st);
      }
      std::vector<char*>* re = &oe;
      std::vector<char*>* ro = &oo;
      if (op == WCMG_OP_FULL || (op == WCMG_OP_DP && dag)) {
        for (int l = 0; l < nl; ++l) m.a[l] = args(l, oe[l], io[l], ie[l], 0, 1.0);
        launch_dslash_multi(prec, 2, false, m, c->st);
        for (int l = 0; l < nl; ++l) m.a[l] = args(l, oo[l], ie[l], io[l], 1, 1.0);
        launch_dslash_multi(prec, 2, false, m, c->st);
        if (op == WCMG_OP_DP) {
          // D_p^dag = A^-1 gamma5 D gamma5
          for (int l = 0; l < nl; ++l) {
            spinor_gamma5(prec, oe[l], c->lats[l]->F.g.Vh, c->st);
            spinor_gamma5(prec, oo[l], c->lats[l]->F.g.Vh, c->st);
          }
          clover_all(t1, oe, 0);
          clover_all(t2, oo, 1);
          re = &t1;
          ro = &t2;
        }
      } else if (op == WCMG_OP_SCHUR_X) {
        // D_ee x - H_eo D_oo^-1 H_oe x (the adjoint: the same between gamma5s)
        for (int l = 0; l < nl; ++l) m.a[l] = args(l, t2[l], ie[l], nullptr, 1, 1.0);
        launch_dslash_multi(prec, 0, true, m, c->st);  // w = A_oo^-1 H_oe x
        for (int l = 0; l < nl; ++l) m.a[l] = args(l, oe[l], t2[l], ie[l], 0, -1.0);
        launch_dslash_multi(prec, 2, false, m, c->st);  // out = A_ee x - H_eo w
        ro = nullptr;
      } else if (op == WCMG_OP_DP) {
        clover_all(t1, ie, 0);
        clover_all(t2, io, 1);
        for (int l = 0; l < nl; ++l) m.a[l] = args(l, oe[l], t2[l], ie[l], 0, 1.0);
        launch_dslash_multi(prec, 1, false, m, c->st);  // out_e = ie + H A_oo^-1 io
        for (int l = 0; l < nl; ++l) m.a[l] = args(l, oo[l], t1[l], io[l], 1, 1.0);
        launch_dslash_multi(prec, 1, false, m, c->st);
      } else if (!dag) {
        clover_all(t1, ie, 0);  // z = A_ee^-1 y
        for (int l = 0; l < nl; ++l) m.a[l] = args(l, t2[l], t1[l], nullptr, 1, 1.0);
        launch_dslash_multi(prec, 0, true, m, c->st);  // w = A_oo^-1 H_oe z
        for (int l = 0; l < nl; ++l) m.a[l] = args(l, oe[l], t2[l], ie[l], 0, -1.0);
        launch_dslash_multi(prec, 1, false, m, c->st);  // out = y - H_eo w
        ro = nullptr;
      } else {
        for (int l = 0; l < nl; ++l) m.a[l] = args(l, t2[l], ie[l], nullptr, 1, 1.0);
        launch_dslash_multi(prec, 0, true, m, c->st);  // A_oo^-1 H_oe (gamma5 y)
        for (int l = 0; l < nl; ++l) m.a[l] = args(l, oe[l], t2[l], ie[l], 0, -1.0);
        launch_dslash_multi(prec, 1, true, m, c->st);  // gamma5 y - A_ee^-1 H_eo (...)
        for (int l = 0; l < nl; ++l) spinor_gamma5(prec, oe[l], c->lats[l]->F.g.Vh, c->st);
        ro = nullptr;
      }
      for (int l = 0; l < nl; ++l) {
        const Geom& g = c->lats[l]->F.g;
        spinor_from_internal(prec, (char*)out + off[l] + (size_t)r * g.V * 12 * 16, (*re)[l], ro ? (*ro)[l] : nullptr,
                             g, g5_out, c->st);
      }
    }
  });
}

static int apply_common(void* ctx, int lat, int op, int prec, void* out, const void* in, int nrhs, bool dag) {
  Ctx* c = as_ctx(ctx);
  if (lat == -1 && c) {
    CHECK(out && in && out != in, WCMG_EINVAL, "null or aliased buffer");
    CHECK(valid_op(op) && valid_prec(prec), WCMG_EINVAL, "bad operator or precision");
    CHECK(nrhs >= 1, WCMG_EINVAL, "nrhs must be >= 1");
    return apply_all_lattices(c, op, prec, out, in, nrhs, dag);
  }
  if (int r = check_lat(c, lat)) return r;
  CHECK(out && in, WCMG_EINVAL, "null buffer");
  CHECK(valid_op(op), WCMG_EINVAL, "bad operator");
  CHECK(valid_prec(prec), WCMG_EINVAL, "bad precision");
  CHECK(nrhs >= 1, WCMG_EINVAL, "nrhs must be >= 1");
  CHECK(out != in, WCMG_EINVAL, "out and in must not alias");
  LatticeState& L = *c->lats[lat];
  CHECK(L.F.have_clover, WCMG_ESTATE, "clover not set");
  CHECK_DEV(c, in, (size_t)nrhs * L.F.g.V * 12 * 16, "input spinors");
  CHECK_DEV(c, out, (size_t)nrhs * L.F.g.V * 12 * 16, "output spinors");
  return guarded([&] {
    const Geom& g = L.F.g;
    const size_t hb = spinor_bytes(prec, g.Vh);
    const size_t one = (size_t)g.V * 12 * 16;
    // all right-hand sides go through each kernel in one batched launch
    char* ie = (char*)c->scratch_buf(42, hb * nrhs);
    char* io = (char*)c->scratch_buf(43, hb * nrhs);
    char* oe = (char*)c->scratch_buf(44, hb * nrhs);
    char* oo = (char*)c->scratch_buf(45, hb * nrhs);
    FineOp fo{c, &L.F, prec, &c->fw[prec], c->st};
    for (int r = 0; r < nrhs; ++r)
      spinor_to_internal(prec, ie + r * hb, io + r * hb, (const char*)in + (size_t)r * one, g,
                         dag && op != WCMG_OP_SCHUR, c->st);
    bool flip_out = false;
    char* re = oe;
    char* ro = oo;
    if (op == WCMG_OP_FULL) {
      fo.D(oe, oo, ie, io, nrhs);
      flip_out = dag;
    } else if (op == WCMG_OP_DP) {
      if (!dag) {
        fo.Dp(oe, oo, ie, io, nrhs);
      } else {
        // D_p^dag = A^-1 gamma5 D gamma5
        fo.D(oe, oo, ie, io, nrhs);
        for (int r = 0; r < nrhs; ++r) {
          spinor_gamma5(prec, oe + r * hb, g.Vh, c->st);
          spinor_gamma5(prec, oo + r * hb, g.Vh, c->st);
        }
        fo.clover(ie, oe, 0, 1, nrhs);
        fo.clover(io, oo, 1, 1, nrhs);
        re = ie;
        ro = io;
      }
    } else if (op == WCMG_OP_SCHUR_X) {
      fo.Mx(oe, ie, nrhs);  // adjoint: input converted with gamma5 above, output flipped below
      flip_out = dag;
      ro = nullptr;
    } else {
      if (!dag)
        fo.Dr(oe, ie, nrhs);
      else
        fo.Dr_dag(oe, ie, nrhs);
      ro = nullptr;
    }
    for (int r = 0; r < nrhs; ++r)
      spinor_from_internal(prec, (char*)out + (size_t)r * one, re + r * hb, ro ? ro + r * hb : nullptr, g, flip_out,
                           c->st);
  });
}

int wcmg_apply_D(void* ctx, int lat, int op, int prec, void* out, const void* in, int nrhs) {
  return apply_common(ctx, lat, op, prec, out, in, nrhs, false);
}

int wcmg_apply_Ddag(void* ctx, int lat, int op, int prec, void* out, const void* in, int nrhs) {
  return apply_common(ctx, lat, op, prec, out, in, nrhs, true);
}

// restrict (to_coarse) or prolong between coarse level `level` (>= 1) and
// coarse level level + 1, canonical layouts
static int transfer_coarse(Ctx* c, LatticeState& L, int level, int prec, void* out, const void* in, int nrhs,
                           bool to_coarse) {
  CHECK(prec == WCMG_F64 || prec == WCMG_F32, WCMG_EINVAL, "coarse transfer precision must be F64 or F32");
  CHECK((int)L.levels.size() > level && L.levels[level]->built && (int)L.ctr.size() >= level &&
            L.ctr[level - 1]->orth,
        WCMG_ESTATE, "next coarse level not built");
  {
    const CoarseLevel& C1 = *L.levels[level - 1];
    const CoarseLevel& C2 = *L.levels[level];
    const size_t b1 = (size_t)nrhs * C1.cg.V * C1.cg.n * 16, b2 = (size_t)nrhs * C2.cg.V * C2.cg.n * 16;
    CHECK_DEV(c, in, to_coarse ? b1 : b2, "input vectors");
    CHECK_DEV(c, out, to_coarse ? b2 : b1, "output vectors");
  }
  return guarded([&] {
    CoarseLevel& C1 = *L.levels[level - 1];
    CoarseLevel& C2 = *L.levels[level];
    CoarseTransfer& T = *L.ctr[level - 1];
    const size_t one1 = (size_t)C1.cg.V * C1.cg.n, one2 = (size_t)C2.cg.V * C2.cg.n;
    const size_t cs = 16;  // canonical side is complex128
    void* a = c->scratch_buf(46, one1 * 16);
    void* b = c->scratch_buf(47, one2 * 16);
    const void* P = prec == WCMG_F64 ? T.v64.p : T.v32.p;
    for (int r = 0; r < nrhs; ++r) {
      if (to_coarse) {
        launch_coarse_canon(prec, a, (char*)const_cast<void*>(in) + r * one1 * cs, C1.perm.as<int>(), C1.cg.V,
                            C1.cg.n, true, c->st);
        launch_ctr_restrict(prec, b, C2.cg.n, 0, a, 0, P, T.vstride(), T.members.as<int>(), C2.cg.V, T.bg.bvol,
                            C1.cg.n, T.nvec, 1, c->st);
        launch_coarse_canon(prec, b, (char*)out + r * one2 * cs, C2.perm.as<int>(), C2.cg.V, C2.cg.n, false, c->st);
      } else {
        launch_coarse_canon(prec, b, (char*)const_cast<void*>(in) + r * one2 * cs, C2.perm.as<int>(), C2.cg.V,
                            C2.cg.n, true, c->st);
        launch_ctr_prolong(prec, a, 0, b, 0, P, T.vstride(), T.blk.as<int>(), C1.cg.V, C1.cg.n, T.nvec, 1, c->st);
        launch_coarse_canon(prec, a, (char*)out + r * one1 * cs, C1.perm.as<int>(), C1.cg.V, C1.cg.n, false, c->st);
      }
    }
    HIPCHK(hipStreamSynchronize(c->st));
  });
}

int wcmg_restrict(void* ctx, int lat, int level, int prec, void* coarse_out, const void* fine_in, int nrhs) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  CHECK(coarse_out && fine_in, WCMG_EINVAL, "null buffer");
  if (int r = check_level(c, lat, level)) return r;
  CHECK(valid_prec(prec), WCMG_EINVAL, "bad precision");
  CHECK(nrhs >= 1, WCMG_EINVAL, "nrhs must be >= 1");
  LatticeState& L = *c->lats[lat];
  if (level >= 1) return transfer_coarse(c, L, level, prec, coarse_out, fine_in, nrhs, true);
  CHECK(!L.levels.empty() && L.levels[0]->built, WCMG_ESTATE, "coarse operator not built");
  CHECK_DEV(c, fine_in, (size_t)nrhs * L.F.g.V * 12 * 16, "fine vectors");
  CHECK_DEV(c, coarse_out, (size_t)nrhs * L.levels[0]->cg.V * L.levels[0]->cg.n * 16, "coarse vectors");
  return guarded([&] {
    const Geom& g = L.F.g;
    CoarseLevel& C = *L.levels[0];
    const int cprec = prec == WCMG_F64 ? WCMG_F64 : WCMG_F32;
    const size_t hb = spinor_bytes(prec, g.Vh);
    void* fe = c->scratch_buf(42, hb);
    void* fo = c->scratch_buf(43, hb);
    void* cv = c->scratch_buf(46, (size_t)C.cg.V * C.cg.n * 16);
    const void* vecs = L.T0.v64.p;
    DBuf v16;
    if (prec == WCMG_F32) vecs = L.T0.v32.p;
    if (prec == WCMG_F16) {
      const size_t h64 = spinor_bytes(WCMG_F64, g.Vh), h16 = spinor_bytes(WCMG_F16, g.Vh);
      v16.alloc((size_t)2 * L.T0.nvec * h16);
      for (int k = 0; k < 2 * L.T0.nvec; ++k)
        spinor_convert(WCMG_F16, (char*)v16.p + k * h16, WCMG_F64, (const char*)L.T0.v64.p + k * h64, g.Vh, c->st);
      vecs = v16.p;
    }
    const size_t one = (size_t)g.V * 12 * 16, cone = (size_t)C.cg.V * C.cg.n * 16;
    for (int r = 0; r < nrhs; ++r) {
      spinor_to_internal(prec, fe, fo, (const char*)fine_in + r * one, g, false, c->st);
      const void* vbm = prec == WCMG_F32 ? L.T0.vbm32.p : nullptr;
      launch_restrict(prec, cv, C.cg.n, 1, fe, vecs, L.T0.nvec, 0, g, L.T0.bg, false, c->st, vbm);
      launch_restrict(prec, cv, C.cg.n, 1, fo, vecs, L.T0.nvec, 1, g, L.T0.bg, true, c->st, vbm);
      launch_coarse_canon(cprec, cv, (char*)coarse_out + r * cone, C.perm.as<int>(), C.cg.V, C.cg.n, false, c->st);
    }
    HIPCHK(hipStreamSynchronize(c->st));
  });
}

int wcmg_prolong(void* ctx, int lat, int level, int prec, void* fine_out, const void* coarse_in, int nrhs) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  CHECK(fine_out && coarse_in, WCMG_EINVAL, "null buffer");
  if (int r = check_level(c, lat, level)) return r;
  CHECK(valid_prec(prec), WCMG_EINVAL, "bad precision");
  CHECK(nrhs >= 1, WCMG_EINVAL, "nrhs must be >= 1");
  LatticeState& L = *c->lats[lat];
  if (level >= 1) return transfer_coarse(c, L, level, prec, fine_out, coarse_in, nrhs, false);
  CHECK(!L.levels.empty() && L.levels[0]->built, WCMG_ESTATE, "coarse operator not built");
  CHECK_DEV(c, fine_out, (size_t)nrhs * L.F.g.V * 12 * 16, "fine vectors");
  CHECK_DEV(c, coarse_in, (size_t)nrhs * L.levels[0]->cg.V * L.levels[0]->cg.n * 16, "coarse vectors");
  return guarded([&] {
    const Geom& g = L.F.g;
    CoarseLevel& C = *L.levels[0];
    const int cprec = prec == WCMG_F64 ? WCMG_F64 : WCMG_F32;
    const size_t hb = spinor_bytes(prec, g.Vh);
    void* fe = c->scratch_buf(42, hb);
    void* fo = c->scratch_buf(43, hb);
    void* cv = c->scratch_buf(46, (size_t)C.cg.V * C.cg.n * 16);
    const void* vecs = L.T0.v64.p;
    DBuf v16;
    if (prec == WCMG_F32) vecs = L.T0.v32.p;
    if (prec == WCMG_F16) {
      const size_t h64 = spinor_bytes(WCMG_F64, g.Vh), h16 = spinor_bytes(WCMG_F16, g.Vh);
      v16.alloc((size_t)2 * L.T0.nvec * h16);
      for (int k = 0; k < 2 * L.T0.nvec; ++k)
        spinor_convert(WCMG_F16, (char*)v16.p + k * h16, WCMG_F64, (const char*)L.T0.v64.p + k * h64, g.Vh, c->st);
      vecs = v16.p;
    }
    const size_t one = (size_t)g.V * 12 * 16, cone = (size_t)C.cg.V * C.cg.n * 16;
    for (int r = 0; r < nrhs; ++r) {
      launch_coarse_canon(cprec, cv, (char*)coarse_in + r * cone, C.perm.as<int>(), C.cg.V, C.cg.n, true, c->st);
      launch_prolong(prec, fe, cv, vecs, L.T0.nvec, 0, g, L.T0.bg, c->st);
      launch_prolong(prec, fo, cv, vecs, L.T0.nvec, 1, g, L.T0.bg, c->st);
      spinor_from_internal(prec, (char*)fine_out + r * one, fe, fo, g, false, c->st);
    }
    HIPCHK(hipStreamSynchronize(c->st));
  });
}

int wcmg_apply_coarse(void* ctx, int lat, int level, int op, int prec, void* out, const void* in, int nrhs) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  CHECK(out && in, WCMG_EINVAL, "null buffer");
  CHECK(out != in, WCMG_EINVAL, "out and in must not alias");
  CHECK(valid_op(op) && op != WCMG_OP_SCHUR_X, WCMG_EINVAL, "bad operator for a coarse level");
  CHECK(prec == WCMG_F64 || prec == WCMG_F32, WCMG_EINVAL, "coarse precision must be F64 or F32");
  CHECK(nrhs >= 1, WCMG_EINVAL, "nrhs must be >= 1");
  LatticeState& L = *c->lats[lat];
  CHECK(L.have_params && level >= 1 && level <= L.params.nlevels, WCMG_EINVAL, "level out of range");
  CHECK((int)L.levels.size() >= level && L.levels[level - 1]->built, WCMG_ESTATE, "coarse operator not built");
  CoarseLevel& C = *L.levels[level - 1];
  CHECK(op != WCMG_OP_SCHUR || C.cg.split, WCMG_EDIM, "coarse lattice has an odd extent: no red-black form");
  CHECK_DEV(c, in, (size_t)nrhs * C.cg.V * C.cg.n * 16, "input vectors");
  CHECK_DEV(c, out, (size_t)nrhs * C.cg.V * C.cg.n * 16, "output vectors");
  return guarded([&] {
    // all right-hand sides in one batched application (FP32 red-black batches
    // run on the matrix cores)
    const size_t cs = prec == WCMG_F64 ? 16 : 8;
    const size_t nall = (size_t)C.cg.V * C.cg.n;
    char* vi = (char*)c->scratch_buf(46, nall * 16 * nrhs);
    char* vo = (char*)c->scratch_buf(47, nall * 16 * nrhs);
    blas_zero(prec, vo, nall * nrhs, c->st);
    CoarseOp cop{&C, prec, &c->cw[prec == WCMG_F64 ? 0 : 1], c->st};
    const size_t cone = nall * 16;
    for (int r = 0; r < nrhs; ++r)
      launch_coarse_canon(prec, vi + r * nall * cs, (char*)const_cast<void*>(in) + r * cone, C.perm.as<int>(),
                          C.cg.V, C.cg.n, true, c->st);
    if (op == WCMG_OP_FULL)
      cop.Dfull(vo, vi, nrhs);
    else if (op == WCMG_OP_DP)
      cop.Dp(vo, vi, nrhs);
    else
      cop.Dr(vo, vi, nrhs);
    for (int r = 0; r < nrhs; ++r)
      launch_coarse_canon(prec, vo + r * nall * cs, (char*)out + r * cone, C.perm.as<int>(), C.cg.V, C.cg.n, false,
                          c->st);
  });
}

int wcmg_coarse_solve(void* ctx, int lat, int level, int prec, void* x, const void* b, double tol, int max_iter,
                      int restart, int launch, wcmg_stats* stats) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  CHECK(x && b, WCMG_EINVAL, "null buffer");
  CHECK(x != b, WCMG_EINVAL, "x and b must not alias");
  CHECK(prec == WCMG_F64 || prec == WCMG_F32, WCMG_EINVAL, "coarse precision must be F64 or F32");
  CHECK(tol > 0 && tol < 1, WCMG_EINVAL, "tol must be in (0,1)");
  CHECK(max_iter >= 1 && restart >= 1 && restart <= kMaxRestart, WCMG_EINVAL,
        "max_iter must be >= 1 and restart in 1..64");
  CHECK(launch >= 0 && launch <= 4, WCMG_EINVAL, "launch must be 0..4");
  CHECK(launch < 3 || prec == WCMG_F32, WCMG_EINVAL, "FP16 hop blocks (launch 3, 4) go with F32");
  LatticeState& L = *c->lats[lat];
  CHECK(L.have_params && level >= 1 && level <= L.params.nlevels, WCMG_EINVAL, "level out of range");
  CHECK((int)L.levels.size() >= level && L.levels[level - 1]->built, WCMG_ESTATE, "coarse operator not built");
  CoarseLevel& C = *L.levels[level - 1];
  CHECK(C.cg.split, WCMG_EDIM, "coarse lattice has an odd extent: no red-black form");
  CHECK_DEV(c, b, (size_t)C.cg.V * C.cg.n * 16, "right-hand side");
  CHECK_DEV(c, x, (size_t)C.cg.V * C.cg.n * 16, "solution");
  return guarded([&] {
    const size_t cs = prec == WCMG_F64 ? 16 : 8;
    const size_t nall = (size_t)C.cg.V * C.cg.n;
    void* vb = c->scratch_buf(40, nall * cs);
    void* vx = c->scratch_buf(41, nall * cs);
    void* t = c->scratch_buf(42, nall * cs);
    void* y = c->scratch_buf(43, nall * cs);
    void* r = c->scratch_buf(44, nall * cs);
    void* br = c->scratch_buf(45, nall * cs);
    launch_coarse_canon(prec, vb, const_cast<void*>(b), C.perm.as<int>(), C.cg.V, C.cg.n, true, c->st);
    wcmg_stats s{};
    auto t0 = std::chrono::steady_clock::now();
    CoarseOp op{&C, prec, &c->cw[prec == WCMG_F64 ? 0 : 1], c->st};
    if (launch != 1) {
      PersistWork pw;
      if (!persistent_available(pw, prec, C, restart))
        fail(WCMG_ENODEV, "the device cannot run the persistent coarse solve");
      persistent_launch(*c, pw, C, prec, vx, vb, t, y, r, br, tol, restart, max_iter, false,
                        launch == 2 || launch == 4, launch >= 3);
      int code = WCMG_OK;
      s.iters = (int)persistent_collect(*c, pw, &code);
      s.status = code;
    } else {
      op.reduced_source(br, vb);
      const double bn = std::sqrt(norm2(*c, prec, br, op.neven()));
      GcrSpace S;
      S.prec = prec;
      S.n = op.neven();
      S.bytes = S.n * cs;
      OpFn A = [&](void* o, const void* i) { op.Dr(o, i); };
      KrylovResult kr = gcr(*c, S, A, nullptr, y, br, true, tol, bn, restart, max_iter, false);
      op.reconstruct(vx, y, vb);
      s.iters = kr.iters;
      s.status = kr.status;
    }
    HIPCHK(hipStreamSynchronize(c->st));
    s.t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    launch_coarse_canon(prec, vx, x, C.perm.as<int>(), C.cg.V, C.cg.n, false, c->st);
    // ||b - Yhat x|| / ||b|| of the full coarse system
    op.Dfull(t, vx);
    blas_axpby(prec, 1.0, 0.0, vb, -1.0, 0.0, t, nall, c->st);
    const double rr = norm2(*c, prec, t, nall), bb = norm2(*c, prec, vb, nall);
    s.true_rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    if (stats) *stats = s;
  });
}

int wcmg_coarse_solve_noalloc(void* ctx, int lat, int level, int prec, void* x, const void* b, double tol,
                              int max_iter, int restart, wcmg_stats* stats) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  CHECK(x && b, WCMG_EINVAL, "null buffer");
  CHECK(x != b, WCMG_EINVAL, "x and b must not alias");
  CHECK(prec == WCMG_F64 || prec == WCMG_F32, WCMG_EINVAL, "coarse precision must be F64 or F32");
  CHECK(tol > 0 && tol < 1, WCMG_EINVAL, "tol must be in (0,1)");
  CHECK(max_iter >= 1 && restart >= 1 && restart <= kMaxRestart, WCMG_EINVAL,
        "max_iter must be >= 1 and restart in 1..64");
  LatticeState& L = *c->lats[lat];
  CHECK(L.have_params && level >= 1 && level <= L.params.nlevels, WCMG_EINVAL, "level out of range");
  CHECK((int)L.levels.size() >= level && L.levels[level - 1]->built, WCMG_ESTATE, "coarse operator not built");
  CoarseLevel& C = *L.levels[level - 1];
  CHECK(C.cg.split, WCMG_EDIM, "coarse lattice has an odd extent: no red-black form");
  CHECK_DEV(c, b, (size_t)C.cg.V * C.cg.n * 16, "right-hand side");
  CHECK_DEV(c, x, (size_t)C.cg.V * C.cg.n * 16, "solution");
  int grid = 0;
  size_t need = 0;
  if (int r = guarded([&] {
        grid = coarse_gcr_persistent_grid(prec, C.cg.n, C.cg.Vh);
        if (grid > 0) need = coarse_solve_noalloc_bytes(C, prec, std::min(restart, max_iter), grid);
      }))
    return r;
  CHECK(grid > 0, WCMG_ENODEV, "the device cannot run the persistent coarse solve");
  if (need > kNoAllocScratchBytes)
    return set_err(WCMG_EINVAL, "the solve needs " + std::to_string(need) + " bytes of work space; the static scratch holds " +
                                    std::to_string(kNoAllocScratchBytes) + " (use wcmg_coarse_solve)");
  return guarded([&] {
    wcmg_stats s{};
    coarse_solve_noalloc(*c, C, prec, noalloc_scratch(c->device), grid, x, b, tol, max_iter, restart, &s);
    if (stats) *stats = s;
  });
}

static int solve_lattice(void* ctx, int lat, int solver, void* x, const void* b, int nrhs, double tol,
                         wcmg_stats* stats, bool dag) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  CHECK(x && b, WCMG_EINVAL, "null buffer");
  CHECK(x != b, WCMG_EINVAL, "x and b must not alias");
  CHECK(solver >= WCMG_MG_GCR && solver <= WCMG_CGNR, WCMG_EINVAL, "bad solver");
  CHECK(nrhs >= 1, WCMG_EINVAL, "nrhs must be >= 1");
  CHECK(tol > 0 && tol < 1, WCMG_EINVAL, "tol must be in (0,1)");
  LatticeState& L = *c->lats[lat];
  CHECK(L.F.have_clover, WCMG_ESTATE, "clover not set");
  if (solver == WCMG_MG_GCR)
    CHECK(L.have_params && !L.levels.empty() && L.levels[0]->built, WCMG_ESTATE, "multigrid hierarchy not built");
  CHECK_DEV(c, b, (size_t)nrhs * L.F.g.V * 12 * 16, "right-hand sides");
  CHECK_DEV(c, x, (size_t)nrhs * L.F.g.V * 12 * 16, "solutions");
  int worst = WCMG_OK;
  int rc = guarded([&] {
    const Geom& g = L.F.g;
    const size_t hb = spinor_bytes(WCMG_F64, g.Vh);
    const size_t one = (size_t)g.V * 12 * 16;
    if (solver == WCMG_MG_GCR && nrhs > 1) {
      // lockstep batches of up to kMaxBatch right-hand sides
      const int bmax = std::min(nrhs, kMaxBatch);
      char* be = (char*)c->scratch_buf(48, hb * bmax);
      char* bo = (char*)c->scratch_buf(49, hb * bmax);
      char* xe = (char*)c->scratch_buf(50, hb * bmax);
      char* xo = (char*)c->scratch_buf(51, hb * bmax);
      for (int r0 = 0; r0 < nrhs; r0 += kMaxBatch) {
        const int nb = std::min(kMaxBatch, nrhs - r0);
        bool x_zero = true;
        for (int i = 0; i < nb; ++i) {
          const void* bs = (const char*)b + (size_t)(r0 + i) * one;
          void* xs = (char*)x + (size_t)(r0 + i) * one;
          spinor_to_internal(WCMG_F64, be + i * hb, bo + i * hb, bs, g, false, c->st);
          spinor_to_internal(WCMG_F64, xe + i * hb, xo + i * hb, xs, g, false, c->st);
          if (dag)
            for (char* v : {be, bo, xe, xo}) spinor_gamma5(WCMG_F64, v + i * hb, g.Vh, c->st);
          x_zero = x_zero && norm2(*c, WCMG_F64, xe + i * hb, (size_t)12 * g.Vh) +
                                     norm2(*c, WCMG_F64, xo + i * hb, (size_t)12 * g.Vh) ==
                                 0.0;
        }
        std::vector<wcmg_stats> s(nb);
        solve_batch(*c, L, xe, xo, be, bo, nb, x_zero, tol, s.data());
        for (int i = 0; i < nb; ++i) {
          if (dag) {
            spinor_gamma5(WCMG_F64, xe + i * hb, g.Vh, c->st);
            spinor_gamma5(WCMG_F64, xo + i * hb, g.Vh, c->st);
          }
          spinor_from_internal(WCMG_F64, (char*)x + (size_t)(r0 + i) * one, xe + i * hb, xo + i * hb, g, false,
                               c->st);
          if (stats) stats[r0 + i] = s[i];
          if (s[i].status != WCMG_OK && worst == WCMG_OK) worst = s[i].status;
        }
      }
      HIPCHK(hipStreamSynchronize(c->st));
      return;
    }
    void* be = c->scratch_buf(48, hb);
    void* bo = c->scratch_buf(49, hb);
    void* xe = c->scratch_buf(50, hb);
    void* xo = c->scratch_buf(51, hb);
    for (int r = 0; r < nrhs; ++r) {
      const void* bs = (const char*)b + (size_t)r * one;
      void* xs = (char*)x + (size_t)r * one;
      spinor_to_internal(WCMG_F64, be, bo, bs, g, false, c->st);
      spinor_to_internal(WCMG_F64, xe, xo, xs, g, false, c->st);
      if (dag) {
        // D^dag x = b  <=>  D (gamma5 x) = gamma5 b
        for (void* v : {be, bo, xe, xo}) spinor_gamma5(WCMG_F64, v, g.Vh, c->st);
      }
      double xn = norm2(*c, WCMG_F64, xe, (size_t)12 * g.Vh) + norm2(*c, WCMG_F64, xo, (size_t)12 * g.Vh);
      wcmg_stats s{};
      solve_rhs(*c, L, solver, xe, xo, be, bo, xn == 0.0, tol, &s);
      if (dag) {
        spinor_gamma5(WCMG_F64, xe, g.Vh, c->st);
        spinor_gamma5(WCMG_F64, xo, g.Vh, c->st);
      }
      spinor_from_internal(WCMG_F64, xs, xe, xo, g, false, c->st);
      if (stats) stats[r] = s;
      if (s.status != WCMG_OK && worst == WCMG_OK) worst = s.status;
    }
    HIPCHK(hipStreamSynchronize(c->st));
  });
  if (rc != WCMG_OK) return rc;
  if (worst != WCMG_OK) return set_err(worst, "solver did not reach the tolerance for every right-hand side");
  return WCMG_OK;
}

// lat = -1: every lattice of the context in lattice order, nrhs right-hand
// sides each (buffers and stats concatenated); a lattice whose solve does not
// converge does not stop the others, and the worst status is returned.
static int solve_impl(void* ctx, int lat, int solver, void* x, const void* b, int nrhs, double tol, wcmg_stats* stats,
                      bool dag) {
  Ctx* c = as_ctx(ctx);
  if (lat != -1) return solve_lattice(ctx, lat, solver, x, b, nrhs, tol, stats, dag);
  CHECK(c, WCMG_EINVAL, "null context");
  CHECK(x && b && x != b, WCMG_EINVAL, "null or aliased buffer");
  CHECK(nrhs >= 1, WCMG_EINVAL, "nrhs must be >= 1");
  size_t total = 0;
  for (auto& L : c->lats) {
    CHECK(L->F.have_clover, WCMG_ESTATE, "clover not set");
    if (solver == WCMG_MG_GCR)
      CHECK(L->have_params && !L->levels.empty() && L->levels[0]->built, WCMG_ESTATE,
            "multigrid hierarchy not built");
    total += (size_t)nrhs * L->F.g.V * 12 * 16;
  }
  CHECK_DEV(c, b, total, "right-hand sides");
  CHECK_DEV(c, x, total, "solutions");
  int worst = WCMG_OK;
  std::string msg;
  size_t off = 0;
  for (int l = 0; l < (int)c->lats.size(); ++l) {
    const int rc = solve_lattice(ctx, l, solver, (char*)x + off, (const char*)b + off, nrhs, tol,
                                 stats ? stats + (size_t)l * nrhs : nullptr, dag);
    if (rc != WCMG_OK && rc != WCMG_ENOCONV && rc != WCMG_EBREAKDOWN && rc != WCMG_ENAN) return rc;
    if (rc != WCMG_OK && worst == WCMG_OK) {
      worst = rc;
      msg = "lattice " + std::to_string(l) + ": " + g_err;
    }
    off += (size_t)nrhs * c->lats[l]->F.g.V * 12 * 16;
  }
  return worst == WCMG_OK ? WCMG_OK : set_err(worst, msg);
}

int wcmg_solve(void* ctx, int lat, int solver, void* x, const void* b, int nrhs, double tol, wcmg_stats* stats) {
  return solve_impl(ctx, lat, solver, x, b, nrhs, tol, stats, false);
}

int wcmg_solve_dag(void* ctx, int lat, int solver, void* x, const void* b, int nrhs, double tol,
                   wcmg_stats* stats) {
  return solve_impl(ctx, lat, solver, x, b, nrhs, tol, stats, true);
}

int wcmg_force(void* ctx, int lat, void* dU, const void* psi, const void* lam, int nrhs, int include_clover) {
  Ctx* c = as_ctx(ctx);
  if (int r = check_lat(c, lat)) return r;
  CHECK(dU && psi && lam, WCMG_EINVAL, "null buffer");
  CHECK(nrhs >= 1, WCMG_EINVAL, "nrhs must be >= 1");
  LatticeState& L = *c->lats[lat];
  CHECK(L.F.have_gauge, WCMG_ESTATE, "gauge field not set");
  if (include_clover)
    CHECK(L.F.have_clover && L.F.clover_from_u, WCMG_ESTATE,
          "the clover force needs a clover term computed from the gauge field");
  CHECK_DEV(c, psi, (size_t)nrhs * L.F.g.V * 12 * 16, "psi");
  CHECK_DEV(c, lam, (size_t)nrhs * L.F.g.V * 12 * 16, "lam");
  CHECK_DEV(c, dU, (size_t)L.F.g.V * 4 * 9 * 16, "gauge gradient");
  return guarded([&] {
    const Geom& g = L.F.g;
    const bool clov = include_clover && (L.F.csw != 0.0 || L.F.csw_t != 0.0);
    const CloverCoef cc = clover_coef(L.F.csw, L.F.csw_t);
    void* z = clov ? c->scratch_buf(52, (size_t)g.V * 54 * 16) : nullptr;
    force_compute(dU, psi, lam, nrhs, L.F.gauge[WCMG_F64].p, g, clov ? &cc : nullptr, z, c->st);
  });
}

int wcmg_dot(void* ctx, int prec, const void* x, const void* y, long n, double* out) {
  CHECK(ctx, WCMG_EINVAL, "null context");
  CHECK(x && y && out, WCMG_EINVAL, "null buffer");
  CHECK(prec == WCMG_F64 || prec == WCMG_F32, WCMG_EINVAL, "precision must be F64 or F32");
  CHECK(n >= 1, WCMG_EINVAL, "n must be >= 1");
  CHECK_DEV(as_ctx(ctx), x, (size_t)n * (prec == WCMG_F64 ? 16 : 8), "x");
  CHECK_DEV(as_ctx(ctx), y, (size_t)n * (prec == WCMG_F64 ? 16 : 8), "y");
  return guarded([&] {
    Ctx* c = as_ctx(ctx);
    blas_cdot(prec, x, y, (size_t)n, c->red.out(), c->st);
    const double* h = c->red.fetch(2);
    out[0] = h[0];
    out[1] = h[1];
  });
}

int wcmg_autotune(void* ctx, int on) {
  CHECK(ctx, WCMG_EINVAL, "null context");
  return guarded([&] { as_ctx(ctx)->tuner.on = on != 0; });
}

int wcmg_autotune_report(void* ctx, char* buf, int len) {
  CHECK(ctx, WCMG_EINVAL, "null context");
  CHECK(buf && len > 0, WCMG_EINVAL, "null buffer");
  return guarded([&] {
    std::string out;
    for (const auto& kv : as_ctx(ctx)->tuner.best) {
      char line[160];
      std::snprintf(line, sizeof(line), "%d %d %d %d %d %d %d %.3f\n", kv.first[0], kv.first[1], kv.first[2],
                    kv.first[3], kv.first[4], kv.second.threads, kv.second.group, kv.second.us);
      out += line;
    }
    std::snprintf(buf, (size_t)len, "%s", out.c_str());
  });
}

int wcmg_timer_enable(void* ctx, int on) {
  CHECK(ctx, WCMG_EINVAL, "null context");
  CHECK(on >= 0 && on <= 2, WCMG_EINVAL, "timer mode must be 0, 1 or 2");
  return guarded([&] {
    Ctx* c = as_ctx(ctx);
    c->timer.reset();
    c->timer.on = on != 0;
    c->timer.only_persistent = on == 2;
  });
}

int wcmg_timer_read(void* ctx, int which, long* count, double* total_ms) {
  CHECK(ctx, WCMG_EINVAL, "null context");
  CHECK(which >= 0 && which < KernelTimer::kIds, WCMG_EINVAL, "bad timer id");
  CHECK(count && total_ms, WCMG_EINVAL, "null output");
  return guarded([&] {
    Ctx* c = as_ctx(ctx);
    c->timer.drain();
    *count = c->timer.count[which];
    *total_ms = c->timer.ms[which];
  });
}

}  // extern "C"
