// Host-side state of a wcmg context: per-lattice fields, the multigrid
// hierarchy, the operator wrappers that sequence kernel launches, and the
// solvers.
#pragma once

#include <array>
#include <functional>
#include <map>
#include <memory>

#include "kernels.h"

namespace wcmg {

// ------------------------------------------------------------------ timers
// HIP-event timing of selected kernel classes on the context stream.
struct KernelTimer {
  bool on = false;
  bool only_persistent = false;  // record only the persistent coarse solves (ids 28-30)
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;  // (class, (start, stop))
  static constexpr int kIds = 128;
  long count[kIds] = {};
  double ms[kIds] = {};
  hipEvent_t get();
  void begin(int cls, hipEvent_t* a);
  void end(int cls, hipEvent_t a);
  void drain();  // synchronises and accumulates
  void reset();
  ~KernelTimer();
};

// ------------------------------------------------------------------ autotuner
// Launch shape of the fine hop kernels (threads per block, right-hand sides
// per thread), chosen by timing every candidate on the first launch of each
// (precision, kernel variant, lattice, batch) and kept for the context.  All
// candidates compute bitwise the same result.
struct Tuner {
  bool on = false;
  struct Choice {
    int threads, group;
    double us;
  };
  std::map<std::array<int, 5>, Choice> best;
};

// ------------------------------------------------------------------ reductions
struct Reducer {
  hipStream_t st = nullptr;
  DBuf partial, res, counter;
  DBuf part_b;  // per-block partials of the batched reductions
  double* host = nullptr;  // pinned staging buffer for results read on the host
  void init(hipStream_t s);
  double* dres() { return res.as<double>(); }
  // reduction result to the device buffer `dst` (default: res)
  RedOut out(double* dst = nullptr) {
    return RedOut{dst ? dst : res.as<double>(), partial.as<double>(), counter.as<unsigned>(), nullptr};
  }
  // copy n results (from res, or from any device address) to the host and synchronise
  const double* fetch(int n) { return fetch_from(res.as<double>(), n); }
  const double* fetch_from(const double* dev, int n);
  // rows doubles at dev + r * pitch (r < rows), `width` each, packed to host[r * width]
  const double* fetch_rows(const double* dev, size_t pitch, int width, int rows);
  // two-slot asynchronous form: the copy of n <= 8 doubles is ordered on the
  // stream and completes while later work runs; fetch_wait blocks for it
  double* host2 = nullptr;
  hipEvent_t ev2[2] = {nullptr, nullptr};
  void fetch_async(const double* dev, int n, int slot);
  const double* fetch_wait(int slot);
  RedB outb(double* dst, size_t rs) { return RedB{dst, rs, part_b.as<double>()}; }
  ~Reducer();
};

struct Ctx;

// ------------------------------------------------------------------ fine level
struct FineFields {
  Geom g;
  bool have_gauge = false, have_clover = false;
  bool clover_from_u = false;  // clover computed from the gauge field (not a caller matrix)
  double m0 = 0.0, csw = 0.0, csw_t = 0.0;  // csw: spatial planes (all planes when isotropic)
  DBuf gauge[3];   // per precision
  DBuf clov[3];    // per precision, packed A and A^-1
};

// temporaries of one precision on the fine lattice
struct FineWork {
  int prec = -1;
  size_t hb = 0;
  DBuf t1, t2, t3;  // parity halves (nrhs of them when batched)
  void ensure(int p, const Geom& g, int nrhs = 1);
};

struct FineOp {
  Ctx* ctx;
  FineFields* F;
  int prec;
  FineWork* w;
  hipStream_t st;
  int fprec = -1;  // storage of links and clover (-1: prec; F16 with F32 spinors)
  int fp() const { return fprec < 0 ? prec : fprec; }
  const Geom& g() const { return F->g; }
  size_t hb() const { return spinor_bytes(prec, F->g.Vh); }
  size_t nelem() const { return (size_t)12 * F->g.Vh; }
  // every operator below acts on nrhs parity halves stored hb() bytes apart
  void hop(void* out, const void* in, const void* x, int parity, int diag, bool postinv, double coeff,
           int nrhs = 1);
  void clover(void* out, const void* in, int parity, int kind, int nrhs = 1);
  // reduced operator D_r y = y - H_eo A_oo^-1 H_oe A_ee^-1 y on even halves
  void Dr(void* out, const void* y, int nrhs = 1);
  // Dr with <out, y> and ||out||^2 reduced into o by its last launch; false
  // (nothing launched) where the fused launch does not apply
  // With e and coef, the first launch also applies the pending minimal-residual
  // update e += a y, y -= a out (a from coef, out still holding the previous
  // D_r result) before D_r is applied to the updated y.
  bool Dr_red(void* out, void* y, const RedOut& o, void* e = nullptr, const double* coef = nullptr);
  void Dr_dag(void* out, const void* y, int nrhs = 1);
  // the same reduced system in the variable x = A_ee^-1 y: out = A_ee x - H_eo A_oo^-1 H_oe x
  // (two launches; its adjoint is gamma5 Mx gamma5)
  void Mx(void* out, const void* x, int nrhs = 1);
  // full-lattice operators on (even, odd) halves
  void D(void* oe, void* oo, const void* ie, const void* io, int nrhs = 1);
  void Dp(void* oe, void* oo, const void* ie, const void* io, int nrhs = 1);
  void reduced_source(void* br, const void* be, const void* bo, int nrhs = 1);
  void reconstruct(void* xe, void* xo, const void* ye, const void* bo, int nrhs = 1);
};

// ------------------------------------------------------------------ coarse level
struct CoarseLevel {
  CoarseGeom cg{};
  BlockGeom bg{};       // blocking of the finer level that produced it
  int nvec = 0;
  bool built = false;
  std::vector<int> perm_host;  // lex -> internal
  DBuf nbr, perm;              // device int arrays
  DBuf Y9;                     // FP64 [site][9][n][n]
  DBuf X[2], Xinv[2], Yhop[2], Yt[2];  // [0] FP64, [1] FP32
  DBuf Yt16;                           // FP16 copy of Yt for the persistent coarsest solve (coarse_fp16)
  DBuf frag;              // FP16 matrix-core fragments of Yt (batched stencil)
  bool has_frag = false;
};

struct CoarseWork {
  DBuf t1, t2;
  void ensure(size_t bytes);
};

struct CoarseOp {
  CoarseLevel* C;
  int prec;     // F64 or F32
  CoarseWork* w;
  hipStream_t st;
  KernelTimer* timer = nullptr;  // times the red-black hop launches (ids timer_base + 0 F64, + 1 F32)
  int timer_base = 20;
  int pi() const { return prec == WCMG_F64 ? 0 : 1; }
  size_t csize() const { return prec == WCMG_F64 ? 16 : 8; }
  size_t nall() const { return (size_t)C->cg.V * C->cg.n; }
  size_t neven() const { return (size_t)C->cg.Vh * C->cg.n; }
  // nrhs right-hand sides of nall() elements each, stored back to back
  void Dfull(void* out, const void* in, int nrhs = 1);
  void Dp(void* out, const void* in, int nrhs = 1);
  void Dr(void* out, const void* y, int nrhs = 1);  // full-size buffers, even half meaningful
  void reduced_source(void* br, const void* b, int nrhs = 1);
  void reconstruct(void* c, const void* y, const void* b, int nrhs = 1);
};

// ------------------------------------------------------------------ hierarchy
struct FineTransfer {
  BlockGeom bg{};
  int nvec = 0;
  bool have_vecs = false, orth = false;
  DBuf raw;       // FP64 full spinors (as given / found by the setup)
  DBuf v64, v32;  // block-orthonormalised copies
  DBuf vbm32;     // v32 in block-major order for the restriction
  DBuf v16, vbm16;  // FP16 copies of v32 and vbm32 (the cycle's transfers with transfer_fp16)
};

// transfer between coarse level l (>= 1) and level l+1; vectors in the
// finer level's internal site order, [k][site][nf]
struct CoarseTransfer {
  BlockGeom bg{};  // blocking of the finer coarse lattice
  int nvec = 0;    // vectors (Nv of the coarser level)
  int nf = 0;      // components per site of the finer level
  int nsites = 0;  // sites of the finer level
  bool have_vecs = false, orth = false;
  DBuf raw, v64, v32;
  DBuf blk;      // int [nsites]: coarser internal site of each finer internal site
  DBuf members;  // int [coarser sites][bvol]: finer internal sites of each block
  size_t vstride() const { return (size_t)nsites * nf; }
};

struct MGSolver;

struct LatticeState {
  std::shared_ptr<MGSolver> mg;  // preconditioner buffers, rebuilt with the hierarchy
  FineFields F;
  bool have_params = false;
  wcmg_mg_params params{};
  FineTransfer T0;
  std::vector<std::unique_ptr<CoarseLevel>> levels;  // levels[0] = coarse level 1
  std::vector<std::unique_ptr<CoarseTransfer>> ctr;  // ctr[0]: coarse level 1 -> level 2
  DBuf dense;       // coarsest level: augmented [N][2N] FP64, right half = inverse (coarsest == 1)
  int dense_n = 0;  // N (0: not built)
  // coarsest == 2: K deflation pairs (Q_j = A Z_j, Q orthonormal) of the coarsest
  // operator A (reduced red-black form where the extents allow), FP64 full-size
  // buffers; qa: the pairs' GCR coefficient slots; tmp: scratch coefficients
  DBuf defl_q, defl_z, defl_qa, defl_tmp;
  int defl_k = 0;  // K (0: not built)
  void clear_hierarchy() {
    T0 = FineTransfer();
    levels.clear();
    ctr.clear();
    dense.release();
    dense_n = 0;
    defl_q.release();
    defl_z.release();
    defl_k = 0;
    mg.reset();
  }
};

// flexible restarted GCR on flat vectors of n complex elements in `prec`
struct GcrSpace {
  int prec;
  size_t n;      // complex elements
  size_t bytes;  // bytes per vector
  std::vector<DBuf> Z, Q;
  DBuf r;
  DBuf scal;  // device-resident GCR coefficients
  void ensure(int restart);
};
constexpr int kMaxRestart = 64;
// per right-hand side coefficient block of the batched GCR: beta then qa
constexpr size_t kGcrCoefs = 2 * (kMaxRestart + 16) + 4 * kMaxRestart;

// lockstep GCR over nrhs right-hand sides: vectors of n complex elements,
// vs elements apart (vs >= n)
struct GcrSpaceB {
  int prec = WCMG_F64;
  size_t n = 0, vs = 0;
  int nrhs = 0;
  std::vector<DBuf> Z, Q;
  DBuf r, scal;
  DBuf cm;  // per right-hand side: orthogonalisation coefficients [slot][slot], then update coefficients
  size_t bytes() const { return (size_t)nrhs * vs * (prec == WCMG_F64 ? 16 : 8); }
  void ensure(int restart);
};
constexpr int kMaxDense = 16384;  // largest coarsest dimension for the dense solve
// ------------------------------------------------------------------ context
struct Ctx {
  hipStream_t st = nullptr;
  int device = 0;
  std::vector<std::unique_ptr<LatticeState>> lats;
  Reducer red;
  KernelTimer timer;
  Tuner tuner;
  FineWork fw[3];
  CoarseWork cw[2];
  GcrSpace outer{};  // Krylov basis of the outer FP64 solver
  GcrSpaceB outer_b{};  // the same for batches of right-hand sides
  // scratch pools reused across calls (keyed by purpose)
  std::vector<DBuf> scratch;
  void* scratch_buf(int slot, size_t bytes);
};

// ------------------------------------------------------------------ solvers
using OpFn = std::function<void(void* out, const void* in)>;

struct KrylovResult {
  int iters = 0;
  int status = WCMG_OK;
  double rel_res = 0.0;
};

// A fixed set of K direction pairs (Q_j = A Z_j, the Q_j orthonormal) kept at
// the head of the GCR basis through every restart: GCR then never explores
// those directions again (deflation of the modes they span).  qa holds the
// 4K coefficient slots of the pairs ({1, 0, 0, 0} each) to copy into the
// solver's slots.
struct GcrDeflation {
  std::vector<const void*> Q, Z;
  const double* qa = nullptr;
  int K() const { return (int)Q.size(); }
};
KrylovResult gcr(Ctx& c, GcrSpace& S, const OpFn& A, const OpFn* K, void* x, const void* b, bool x_zero,
                 double tol, double target_norm, int restart, int maxiter, bool fixed_iters = false,
                 const GcrDeflation* defl = nullptr);
// The unpreconditioned red-black GCR of a coarse level in one cooperative
// launch: buffers of its own, iterations and failures counted on the device
// and read back by persistent_collect (one host synchronisation).
struct PersistWork {
  DBuf q, z, t, qraw, part, ctl;  // Krylov bases, odd-site hops of q, partial sums, barrier lines + info
  DBuf tags;                      // tagged slots of t, q and the step sums (cleared with ctl)
  int grid = -1;         // workgroups (0: not available; -1: not yet queried)
  bool pending = false;  // device counters not yet read back
};
bool persistent_available(PersistWork& w, int prec, const CoarseLevel& C, int restart);
// out = approximate Dhat^-1 in (full coarse vectors); t: full scratch, y, r, br: >= half vectors
void persistent_launch(Ctx& c, PersistWork& w, CoarseLevel& C, int prec, void* out, const void* in, void* t, void* y,
                       void* r, void* br, double tol, int restart, int maxiter, bool fixed,
                       bool general = false, bool mat16 = false, bool trust = false);
// iterations since the last collect; status (optional) gets the first failure code
long persistent_collect(Ctx& c, PersistWork& w, int* status = nullptr);
// the persistent launch on caller-provided buffers (sizes as for launch_coarse_gcr_persistent;
// ctl: kPersistCtlBytes, zeroed before its first use)
struct PersistBufs {
  void *Q, *Z, *T, *qraw;
  double* part;
  void* ctl;
  void* tags = nullptr;  // coarse_gcr_persistent_tag_bytes, zeroed with ctl (nullptr: no tagged steps)
  size_t tag_bytes = 0;
};
void persistent_launch_bufs(Ctx& c, int grid, const PersistBufs& B, CoarseLevel& C, int prec, void* out,
                            const void* in, void* t, void* y, void* r, void* br, double tol, int restart,
                            int maxiter, bool fixed, bool general, bool mat16 = false, bool trust = false);

// ------------------------------------------------------------------ allocation-free coarse solve
// One static device array per GPU (noalloc.hip) holds every work buffer of
// wcmg_coarse_solve_noalloc.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
// device address of that GPU's array (looked up once per device, with it current)
void* noalloc_scratch(int device);
// zero `bytes` (a multiple of 4) with a fill kernel on st
void noalloc_zero(void* p, size_t bytes, hipStream_t st);
// bytes of the array a coarse solve of level C needs (grid: persistent workgroups)
size_t coarse_solve_noalloc_bytes(const CoarseLevel& C, int prec, int restart, int grid);
// the persistent coarse solve (wcmg_coarse_solve, launch 0) with every buffer carved
// from `base` (at least coarse_solve_noalloc_bytes); x, b canonical complex128 [Vc][n]
void coarse_solve_noalloc(Ctx& c, CoarseLevel& C, int prec, void* base, int grid, void* x, const void* b,
                          double tol, int max_iter, int restart, wcmg_stats* s);
KrylovResult bicgstab(Ctx& c, int prec, size_t n, const OpFn& A, void* x, const void* b, double tol,
                      double target_norm, int maxiter);
// batched flexible GCR: A and K act on S.nrhs right-hand sides at once
std::vector<KrylovResult> gcr_b(Ctx& c, GcrSpaceB& S, const OpFn& A, const OpFn* K, void* x, const void* b,
                                bool x_zero, double tol, const double* target_norm, int restart, int maxiter,
                                bool fixed = false);

// vector helpers
double norm2(Ctx& c, int prec, const void* x, size_t n);

// multigrid driver
void mg_setup_null_vectors(Ctx& c, LatticeState& L, int level);
void mg_build_coarse(Ctx& c, LatticeState& L, int level);
void mg_refine_null_vectors(Ctx& c, LatticeState& L, int passes, int iters);
struct MGSolver;
void solve_rhs(Ctx& c, LatticeState& L, int solver, void* x_e, void* x_o, const void* b_e, const void* b_o,
               bool x_zero, double tol, wcmg_stats* st);
// multigrid solve of nrhs (<= kMaxBatch) right-hand sides in lockstep; halves
// stored contiguously (nrhs even halves, then nrhs odd halves in separate buffers)
void solve_batch(Ctx& c, LatticeState& L, void* x_e, void* x_o, const void* b_e, const void* b_o, int nrhs,
                 bool x_zero, double tol, wcmg_stats* st);

CoarseGeom make_coarse_geom(const BlockGeom& bg, int nvec);
BlockGeom make_block_geom(const int L[4], const int b[4]);

}  // namespace wcmg
