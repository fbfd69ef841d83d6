/*
 * wcmg.h -- C ABI of the Wilson-clover adaptive-multigrid library for AMD
 * Instinct MI355X (gfx950).
 *
 * The library solves the lattice Dirac equation of Osborn et al.,
 * "Multigrid solver for clover fermions" (Lattice 2010), Eq.(1):
 *
 *     [D(U) + m] psi = eta        for varying sources eta and gauge fields U,
 *
 * with GCR preconditioned by an adaptive multigrid cycle built on the
 * red-black preconditioned operator of Eqs.(2)-(4).  All arithmetic runs in
 * hand-written HIP kernels on one GPU; the host code only sequences kernels.
 *
 * Conventions (the paper leaves them open; these are the library's choice):
 *   D psi(x) = (4+m0) psi(x)
 *            - 1/2 sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu)
 *                         + (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
 *            + csw (i/4) sum_{mu!=nu} sigma_mu_nu Fhat_mu_nu(x) psi(x)
 *   sigma_mu_nu = (i/2)[gamma_mu, gamma_nu], Fhat = (Q - Q^dag)/8 with Q the
 *   sum of the four plaquette leaves; chiral gamma basis with
 *   gamma5 = diag(1,1,-1,-1); directions mu = x,y,z,t; periodic in space,
 *   time boundary phase t_bc (-1 antiperiodic, +1 periodic).
 *
 * Canonical layouts (interleaved complex, little endian):
 *   gauge   complex128 [Lt][Lz][Ly][Lx][4 mu][3][3]
 *   spinor  complex128 [nrhs][Lt][Lz][Ly][Lx][4 spin][3 colour]
 *   coarse  complex128 [nrhs][Vc][2*Nv]   coarse site lex order, component
 *           s*Nv + k (s = 0: gamma5 = +1 chirality, s = 1: -1)
 *   coarse operator complex128 [Vc][9][2Nv][2Nv]: slot 0 the site block X,
 *           slot 1+d the hop to direction d = 2*mu (+mu) or 2*mu+1 (-mu).
 *
 * Ownership: every buffer argument belongs to the caller.  Pointers marked
 * "device" must be device memory of the context's GPU; "host" pointers are
 * read or written before the call returns.  The library keeps its own
 * copies (in its internal even-odd layouts) of everything it is given and
 * never retains a caller pointer.  Work is enqueued on the stream given to
 * wcmg_create; apply/restrict/prolong return without synchronising, solve
 * and the setup calls synchronise the stream before returning.
 *
 * Errors: every call returns an int status, 0 = WCMG_OK.  No exception or
 * abort crosses the ABI.  Arguments are validated before any device call;
 * on error wcmg_last_error() returns a message (thread-local).
 */
#ifndef WCMG_H
#define WCMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  WCMG_OK = 0,
  WCMG_EINVAL = 1,          /* bad argument (null pointer, bad enum, range) */
  WCMG_EDIM = 2,            /* odd extent, block does not divide, Nv too large */
  WCMG_ESTATE = 3,          /* call made before its prerequisites */
  WCMG_ENOCONV = 4,         /* solver hit max_iter; x holds the last iterate */
  WCMG_EBREAKDOWN = 5,      /* Krylov breakdown (rho or omega = 0) */
  WCMG_ENAN = 6,            /* NaN/Inf met in a residual norm */
  WCMG_ECLOVER_NOT_PD = 7,  /* clover block not positive definite */
  WCMG_ERANK = 8,           /* null vectors linearly dependent on a block */
  WCMG_ENOMEM = 9,          /* device allocation failed */
  WCMG_EHIP = 10,           /* HIP runtime error */
  WCMG_ENODEV = 11          /* no usable GPU */
};

typedef enum { WCMG_F64 = 0, WCMG_F32 = 1, WCMG_F16 = 2 } wcmg_prec;

/* operator forms (red-black paragraph, Eqs.(2)-(3)):
 *   FULL     D of Eq.(1), both parities;
 *   SCHUR    D_r = 1 - D_eo D_oo^-1 D_oe D_ee^-1 acting on even sites (odd
 *            sites of the input are ignored, odd sites of the output are
 *            zero); three launches (A_ee^-1, then the two hops);
 *   DP       D_p = D diag(D_ee, D_oo)^-1, both parities;
 *   SCHUR_X  D_r D_ee = D_ee - D_eo D_oo^-1 D_oe, the same reduced system in
 *            the variable x_e = D_ee^-1 y_e of Eq.(3) (fine operators only);
 *            two launches, each field read once: the odd hop with D_oo^-1
 *            fused, then the even hop with D_ee x fused. */
typedef enum { WCMG_OP_FULL = 0, WCMG_OP_SCHUR = 1, WCMG_OP_DP = 2, WCMG_OP_SCHUR_X = 3 } wcmg_op;

/* MG_GCR: FP64 GCR on D_r preconditioned by the multigrid cycle (adaptive
 * multigrid paragraph); GCR, BICGSTAB: unpreconditioned FP64 on D_r;
 * MP_BICGSTAB: the paper's comparison solver (Implementation paragraph),
 * BiCGStab in FP32 inside FP64 iterative refinement; CGNR: conjugate
 * gradients on the normal equations D_r^dag D_r y = D_r^dag b_r, FP64. */
typedef enum {
  WCMG_MG_GCR = 0,
  WCMG_GCR = 1,
  WCMG_BICGSTAB = 2,
  WCMG_MP_BICGSTAB = 3,
  WCMG_CGNR = 4
} wcmg_solver;

typedef struct {
  int dims[4]; /* Lx, Ly, Lz, Lt; each even and >= 2 */
  int t_bc;    /* -1 antiperiodic (default), +1 periodic */
} wcmg_lattice;

#define WCMG_MAX_LEVELS 4

/* Multigrid parameters (Implementation paragraph, Table 1, Setup section).
 * Level l = 0 is the fine lattice; coarse level l+1 is built from level l
 * with block[l] and nvec[l]. */
typedef struct {
  int nlevels;                      /* number of coarse levels: 1 (two-level), 2 (three-level) or 3
                                       (four-level; the fourth level the Results section anticipates
                                       for large volumes) */
  int block[WCMG_MAX_LEVELS][4];    /* aggregate (block) extents per level */
  int nvec[WCMG_MAX_LEVELS];        /* null vectors per level (coarse dim 2*nvec) */
  double tol[WCMG_MAX_LEVELS];      /* relative tolerance of the GCR on coarse level l+1 */
  int max_iter[WCMG_MAX_LEVELS];    /* cap of that GCR */
  int restart[WCMG_MAX_LEVELS];     /* its restart length */
  int nu_post;                      /* MR smoothing steps after the coarse correction */
  int outer_restart;                /* restart length of the outer FP64 GCR */
  int outer_max_iter;               /* cap of the outer GCR */
  wcmg_prec smoother_prec;          /* precision of the preconditioner: F64, F32, or F16 (FP32
                                       vectors and arithmetic, half-precision links and clover in
                                       the fine smoother; coarse levels FP32) */
  int setup_relax;                  /* GCR steps per relaxation in the setup */
  int setup_max_steps;              /* max relaxations per vector */
  double setup_rq_tol;              /* stop when |d rho| / rho < this */
  uint64_t seed;                    /* Philox4x32-10 key for the random start vectors */
  int coarsest;                     /* 0: unpreconditioned GCR (paper); 1: direct solve with the
                                       dense FP64 inverse of the coarsest full operator (Gauss-Jordan
                                       with partial pivoting; dimension <= 16384); 2: deflated FP64
                                       GCR: nvec[nlevels] (1..48) low modes of the coarsest
                                       (red-black where possible) operator, found by inverse
                                       iteration when the coarsest level is built, stay at the head
                                       of the GCR basis (nvec[nlevels] + restart <= 64) */
  int cycle_mode;                   /* 0: inner GCRs stop at their tolerance (paper); 1: every inner
                                       GCR runs exactly max_iter[l] steps with no host round trip;
                                       2: as 1, with the whole preconditioner captured once into a
                                       HIP graph and replayed at every outer iteration; 3: as 0, with
                                       the preconditioner captured and replayed as in 2 when it is a
                                       pure sequence of kernels (one coarse level solved by the
                                       persistent launch, whose tolerance test runs on the device),
                                       eagerly otherwise or where the capture is refused */
  wcmg_prec setup_prec;             /* arithmetic of the null-vector setup (inverse iteration, Setup
                                       section): F32 (default), F64, or F16 (FP32 vectors and
                                       arithmetic with half-precision links and clover); the
                                       vectors are block-orthonormalised in FP64 afterwards */
  int coarse_launch;                /* unpreconditioned GCR on the coarsest level: 0 (default) the
                                       whole solve in one cooperative launch with grid barriers,
                                       where the device supports it and cycle_mode != 2 (the
                                       one-site kernel where it applies, as wcmg_coarse_solve
                                       launch 0); 2 the same with the strided kernel always; 1
                                       one launch per kernel of every step */
  int plain_max_iter;               /* iteration cap of the solvers without multigrid (GCR,
                                       BiCGStab, MP_BICGSTAB (FP32 iterations), CGNR); 0: 100000 */
  double mp_inner_tol;              /* MP_BICGSTAB: relative tolerance of each FP32 BiCGStab solve of
                                       the residual equation; 0: 1e-3 */
  int coarse_fp16;                  /* 1: the persistent coarsest solve reads its red-black hop blocks
                                       in FP16 (FP32 vectors and arithmetic; with one site per
                                       workgroup the even site's blocks stay in LDS for the whole
                                       solve); 0: FP32 blocks */
  int transfer_fp16;                /* 1: the FP32 cycle restricts and prolongs with FP16 copies of
                                       the first level's null vectors (FP32 arithmetic, half the
                                       bytes of P; the coarse operator is still built from the FP64
                                       vectors); 0: FP32 copies */
} wcmg_mg_params;

typedef struct {
  int iters;               /* outer iterations (GCR) or BiCGStab iterations */
  double inner_iters[WCMG_MAX_LEVELS]; /* MG_GCR: mean inner GCR iterations per call, coarse level
                                          l+1; MP_BICGSTAB: [0] = refinement cycles */
  double true_rel_res;     /* ||b - D x|| / ||b|| recomputed in FP64 after the solve */
  double t_solve_s;        /* wall time of the solve on the host clock */
  int status;              /* WCMG_OK or the failure code for this right-hand side */
  int inner_status;        /* first failure an inner (coarse-level) solve of the preconditioner reported
                              during this solve (e.g. EBREAKDOWN when the FP32 persistent coarse GCR lost
                              its Pythagorean step norm, ENAN), else WCMG_OK; informational: the outer
                              FP64 GCR and the true residual decide `status` */
} wcmg_stats;

/* Fill *p with the library defaults (2 levels, 4^4 blocks, Nv = 24,
 * tol 0.1, MR(4) post-smoothing, FP32 preconditioner). */
int wcmg_mg_params_default(wcmg_mg_params* p);

/* Create a context for nlat lattices on the current HIP device.
 * lats: host array of nlat descriptors.  hip_stream: a hipStream_t or NULL
 * for the null stream.  *out receives the handle.  Fails with ENODEV when
 * no GPU is visible, EDIM for an odd or too small extent. */
int wcmg_create(const wcmg_lattice* lats, int nlat, void* hip_stream, void** out);
int wcmg_destroy(void* ctx);

/* Gauge field U of Eq.(1) in the canonical layout (host or device per
 * on_device).  The library converts it to its internal layouts in every
 * precision.  Invalidates clover and multigrid state of that lattice. */
int wcmg_set_gauge(void* ctx, int lat, const void* U, int on_device);

/* Site-diagonal part D_ee / D_oo (red-black paragraph): (4+m0) + clover.
 * A == NULL: computed on the GPU from the gauge field with coefficient csw.
 * Otherwise A is complex128 [V][12][12] (host/device per on_device) and
 * csw is ignored.  The inverse comes from a per-chirality Cholesky; fails
 * with ECLOVER_NOT_PD if a block is not positive definite. */
int wcmg_set_clover(void* ctx, int lat, double m0, double csw, const void* A, int on_device);

/* Anisotropic Wilson-clover (the Results section's lattices have a finer
 * temporal than spatial spacing): every spatial hop of Eq.(1) carries the
 * coefficient hop_s (the bare speed of light over the bare anisotropy, > 0;
 * temporal hops keep 1), the site-diagonal constant becomes
 * m0 + 1 + 3 hop_s (4 + m0 when hop_s = 1), and the clover term weights the
 * spatial planes with csw_s and the planes containing time with csw_t:
 *   D = (m0 + 1 + 3 hop_s) - 1/2 sum_mu c_mu [hops of Eq.(1)]
 *     + (i/4) sum_{mu != nu} c_munu sigma_mu_nu Fhat_mu_nu,
 * c_mu = hop_s (mu spatial), 1 (t); c_munu = csw_s (both spatial), csw_t.
 * Computed from the gauge field; every operator, solver, the multigrid setup
 * and the force of this lattice use it from then on (wcmg_set_clover goes
 * back to the isotropic form).  Errors as wcmg_set_clover. */
int wcmg_set_clover_aniso(void* ctx, int lat, double m0, double hop_s, double csw_s, double csw_t);

/* Fix the multigrid shape (blocks, Nv, tolerances) for a lattice. EDIM if
 * a block does not divide its level, Nv exceeds the block's degrees of
 * freedom per chirality, or (coarsest = 1) the coarsest dimension exceeds
 * 16384.  With nlevels = 2 each intermediate level runs GCR preconditioned
 * by the next level's correction followed by MR smoothing (the recursive
 * cycle of the Implementation paragraph). */
int wcmg_set_mg_params(void* ctx, int lat, const wcmg_mg_params* p);

/* Setup section: for each vector, repeated relaxation (inverse iteration)
 * on a Philox random start vector while the Rayleigh quotient
 * ||D_p v||^2/||v||^2 is monitored, keeping v globally orthogonal to the
 * vectors already found.  Level 0 relaxes on the fine D_p; level l > 0 on
 * the coarse D_p of level l (which must be built).  Synchronises. */
int wcmg_build_null_vectors(void* ctx, int lat, int level);

/* Import or export raw null vectors of a level (saved setups, Results
 * section).  Level 0: nvec fine spinors in the canonical spinor layout;
 * level l > 0: nvec coarse vectors of level l.  nvec must equal the
 * parameters' nvec[level]. */
int wcmg_set_null_vectors(void* ctx, int lat, int level, const void* v, int nvec, int on_device);
int wcmg_get_null_vectors(void* ctx, int lat, int level, void* v, int on_device);

/* The random start vectors of the setup (Setup section) as the library draws
 * them: entry m of vector k on level l is one complex Gaussian (re, im) by
 * Box-Muller from Philox4x32-10 with counter (m mod 2^32, m div 2^32, k, l)
 * and key (seed mod 2^32, seed div 2^32); m = lex_site * 12 + spin * 3 +
 * colour on the fine level, lex_site * 2Nv + component on coarse level l.
 * Vectors k0 .. k0 + nvec - 1 go to out (device): canonical fine spinors for
 * level 0, coarse vectors of level l (which must be built) otherwise.  For
 * parity checks of the setup, and for callers running their own relaxation.
 * Asynchronous. */
int wcmg_setup_start_vectors(void* ctx, int lat, int level, uint64_t seed, int k0, int nvec, void* out);

/* Adaptive refinement of the fine null vectors (Setup section: relaxing with
 * a multigrid cycle built from the vectors already found, as in adaptive
 * smoothed aggregation, combined with the inverse-iteration setup -- the
 * hybrid the paper plans for the clover case).  Needs a built hierarchy.
 * Each of `passes` rounds relaxes every fine null vector v with `iters` steps
 * of the multigrid-preconditioned FP64 GCR on the homogeneous reduced system
 * D_r y = 0 from y = v_e, completes the odd half from D_p v = 0, orthonormalises
 * the vectors in order (twice) and rebuilds P and every coarse operator (the
 * coarse levels' own vectors are kept).  Synchronises. */
int wcmg_refine_null_vectors(void* ctx, int lat, int passes, int iters);

/* Coarse operator of level+1: block x chirality split and orthonormalise
 * the level's vectors (P), then Yhat = R D_p P with R = P^dag gamma5
 * (red-black paragraph), its site-block inverses and the red-black
 * preconditioned hops.  Synchronises. */
int wcmg_build_coarse(void* ctx, int lat, int level);
/* Copy Yhat of coarse level level+1 (canonical coarse-operator layout). */
int wcmg_get_coarse(void* ctx, int lat, int level, void* Y, int on_device);

/* out = op(in) or op^dag(in) for nrhs canonical spinors (device).  prec is
 * the storage/arithmetic precision of the internal apply (F16 stores
 * fields in half precision with FP32 arithmetic).  All right-hand sides go
 * through each kernel in one batched launch.  lat = -1 (any op, D or
 * D^dag): every lattice of the context (at most 4, of any volumes), buffers
 * holding nrhs spinors of each lattice, concatenated in lattice order; for
 * each right-hand side every kernel is one launch over all lattices (a work
 * list of per-lattice block ranges).  Asynchronous. */
int wcmg_apply_D(void* ctx, int lat, int op, int prec, void* out, const void* in, int nrhs);
int wcmg_apply_Ddag(void* ctx, int lat, int op, int prec, void* out, const void* in, int nrhs);

/* Transfer operators between level and level+1 (device buffers):
 * restrict: coarse = R fine = P^dag gamma5 fine;  prolong: fine = P coarse.
 * Level 0 fine vectors are canonical spinors (both parities); coarse
 * vectors of level l >= 1 are complex128 [Vc][2 Nv] in lexicographic
 * coarse-site order.  prec (F64/F32 on coarse levels) is the arithmetic. */
int wcmg_restrict(void* ctx, int lat, int level, int prec, void* coarse_out, const void* fine_in, int nrhs);
int wcmg_prolong(void* ctx, int lat, int level, int prec, void* fine_out, const void* coarse_in, int nrhs);

/* Coarse stencil of coarse level `level` (>= 1) in form op (FULL: Yhat,
 * SCHUR: 1 - Yhat_eo X_oo^-1 Yhat_oe X_ee^-1, DP: Yhat X^-1). */
int wcmg_apply_coarse(void* ctx, int lat, int level, int op, int prec, void* out, const void* in, int nrhs);

/* Approximate solve of coarse level `level` (>= 1), as inside the cycle
 * (coarse even-odd paragraph, GCR of the solver paragraph): red-black GCR
 * with restart length `restart` (1..64) on the reduced coarse operator from
 * a zero start, stopping when ||r_r|| <= tol ||b_r|| (true reduced residual
 * recomputed at the end of every cycle) or after max_iter steps, then the
 * odd half reconstructed.  b and x: one complex128 [Vc][2 Nv] device vector
 * each (lexicographic coarse sites).  prec: F64 or F32 arithmetic and
 * storage.  launch 0: the whole solve in one cooperative launch with grid
 * barriers (WCMG_ENODEV if the device cannot run the grid at once): with at
 * most one even site per workgroup the one-site kernel (Krylov basis in LDS,
 * a neighbour wait in place of the second grid barrier of a step), else sites
 * strided over the workgroups; launch 2: the strided kernel always (the same
 * bits); launch 1: one launch per kernel of every step; launch 3 and 4: as 0
 * and 2 with the hop blocks read in FP16 (prec F32; FP32 arithmetic; the
 * one-site kernel keeps its even site's blocks in LDS for the whole solve
 * when they fit; 3 and 4 give the same bits).  stats (optional):
 * iters, status, and
 * true_rel_res = ||b - Yhat x|| / ||b|| of the full coarse system in prec.
 * Requires a lattice with every coarse extent even (EDIM otherwise). */
int wcmg_coarse_solve(void* ctx, int lat, int level, int prec, void* x, const void* b, double tol, int max_iter,
                      int restart, int launch, wcmg_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture of its own streams, tight serving loops, harnesses that forbid
 * hipMalloc): wcmg_coarse_solve with launch 0, allocation-free.  Every work
 * buffer (Krylov bases q, z and their odd-site hops, the reduced vectors,
 * the layout staging of b and x, the partial sums and the grid barrier's
 * control block) is carved from one static device array of
 * WCMG_NOALLOC_SCRATCH_BYTES (32 MiB) per GPU, reserved with the library's
 * code object and held until the process ends; its device address is looked
 * up when a context is created on that GPU.  No hipMalloc, hipFree or other
 * allocating call is made.  Arguments, result and stats as for
 * wcmg_coarse_solve (launch 0).  EINVAL, before any launch, when the solve
 * needs more than the array holds: 68 KiB + 16 * grid * 136 bytes + 6 full
 * coarse vectors + (4 restart + 1) half vectors, each rounded up to 256
 * bytes (about 14 MB for a 4^3x8 coarse lattice, Nv = 24, restart 30, FP32;
 * twice that in FP64).  Every call on one GPU shares that GPU's array and
 * finds the previous call's contents; the control block is cleared at every
 * call.  Calls that overlap in time on one GPU (two host threads, or two
 * streams) race: serialise them.  Synchronises the context stream. */
#define WCMG_NOALLOC_SCRATCH_BYTES (32u << 20)
int wcmg_coarse_solve_noalloc(void* ctx, int lat, int level, int prec, void* x, const void* b, double tol,
                              int max_iter, int restart, wcmg_stats* stats);

/* Solve D x = b for nrhs canonical right-hand sides (device).  lat = -1:
 * every lattice of the context in one call, x, b holding nrhs spinors of
 * each lattice in lattice order and stats nlat * nrhs entries in the same
 * order; each lattice's right-hand sides go through its own hierarchy, and a
 * lattice that does not converge does not stop the others.  x is the
 * initial guess on entry if nonzero.  Stops when ||b - D x|| <= tol ||b||
 * (true residual recomputed in FP64).  stats: host array of nrhs entries
 * or NULL.  MG_GCR: outer FP64 GCR on D_r preconditioned by the cycle;
 * GCR / BICGSTAB: unpreconditioned FP64 on D_r.  Synchronises.  Returns the
 * worst status over the right-hand sides. */
int wcmg_solve(void* ctx, int lat, int solver, void* x, const void* b, int nrhs, double tol, wcmg_stats* stats);

/* Solve the adjoint system D^dag x = b (device, canonical layout), for the
 * backward pass of a loss through x = D^-1 eta.  Uses the gamma5-hermiticity
 * of Eq.(1), D^dag = gamma5 D gamma5: x = gamma5 D^-1 (gamma5 b), so the same
 * solver and multigrid hierarchy serve.  Arguments, initial guess, stopping
 * rule, stats and errors as for wcmg_solve (the residual reported is that of
 * the transformed system, equal in norm to ||b - D^dag x||). */
int wcmg_solve_dag(void* ctx, int lat, int solver, void* x, const void* b, int nrhs, double tol,
                   wcmg_stats* stats);

/* Gauge-link gradient of a real loss L through x = D(U)^-1 eta, given the
 * solutions psi (x) and lam = D^-dag g (g the gradient of L with respect to
 * x), both device arrays of nrhs canonical spinors:
 *   dU[y][mu] = -dRe<lam, D(U) psi>/dU_mu(y), summed over the nrhs pairs,
 * in PyTorch's complex convention (dL = Re sum conj(dU) delta U); canonical
 * complex128 [Lt][Lz][Ly][Lx][4][3][3], overwritten.  The hopping part comes
 * from the hop of Eq.(1) (with the time boundary phase of each link); with
 * include_clover != 0 the clover part (derivative of the plaquette leaves)
 * is added, which needs a clover computed from the gauge field by
 * wcmg_set_clover(A = NULL).  FP64.  Asynchronous on the context stream.
 * Errors: EINVAL (null buffer, nrhs < 1), ESTATE (no gauge field, or the
 * clover part requested for a caller-supplied clover matrix). */
int wcmg_force(void* ctx, int lat, void* dU, const void* psi, const void* lam, int nrhs, int include_clover);

/* Project autotuner (on != 0: enable, 0: disable; choices are kept): the
 * first launch of each fine hop kernel variant for a given lattice,
 * precision and batch size times every candidate launch shape (64/128/256
 * threads per block x 1/2/4 right-hand sides per thread, or -1: one per
 * thread with the workgroups of a site block's right-hand sides adjacent) on the context
 * stream and keeps the fastest.  Every candidate gives bitwise the same
 * result, so tuning never changes an answer.  Not during graph capture. */
int wcmg_autotune(void* ctx, int on);
/* The tuner's choices as text, one line per kernel variant
 * ("prec diag postinv Vh nrhs threads group microseconds"), written to buf
 * (NUL-terminated, truncated to len bytes). */
int wcmg_autotune_report(void* ctx, char* buf, int len);

/* The global sum behind every inner product of the Krylov solvers (the
 * GCR orthogonalisation of the adaptive multigrid paragraph):
 * out[0] + i out[1] = sum_k conj(x_k) y_k over n complex elements of
 * device arrays x, y (prec F64: complex128, F32: complex64), accumulated in
 * FP64 with the same deterministic two-pass reduction the solvers use.
 * out is a host array of 2 doubles.  Synchronises. */
int wcmg_dot(void* ctx, int prec, const void* x, const void* y, long n, double* out);

/* Per-kernel timing with HIP events on the context's stream.
 * wcmg_timer_enable(ctx, 1) resets the counters and starts recording every
 * launch of the timed kernels (2: only the persistent coarse solves, whose
 * launches are long, so that recording them costs the solve almost nothing;
 * 0: off); wcmg_timer_read returns the launch count and
 * the summed duration in milliseconds for kernel id `which` (0..127,
 * synchronising the stream).  Ids: fine hop kernel prec*6 + diag*2 +
 * clover_inverse (prec 0 F64, 1 F32, 2 F16; diag 0 none, 1 x, 2 A x; see
 * the DIAG/POST modes of the Dslash), batched fine hops 32 + the same, FP16
 * fields with FP32 spinors 56 + diag*2 + clover_inverse; site-local clover
 * launches 64 + prec (batched 67 + prec, FP16 fields 70), the smoother's
 * fused update + clover launch 72 + prec; coarse red-black hop b + prec
 * with b = 20 + 2 l for l = 0, 1 and 96 + 2 (l - 2) beyond (l = 0 first
 * coarse level, prec 0 F64 / 1 F32; batches +4), batched red-black hop on
 * the matrix cores b + 30, persistent coarse solve 28 + l. */
int wcmg_timer_enable(void* ctx, int on);
int wcmg_timer_read(void* ctx, int which, long* count, double* total_ms);

const char* wcmg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WCMG_H */
