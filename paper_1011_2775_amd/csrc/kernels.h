// Launchers of the device kernels (one translation unit per kernel family).
#pragma once

#include "wcmg_internal.h"

namespace wcmg {

// ------------------------------------------------------------ fine Dslash
struct DslashArgs {
  void* out;           // output parity spinor
  const void* in;      // opposite-parity spinor (hopping input)
  const void* x;       // same-parity spinor for the DIAG term
  const void* gauge;   // links of this precision
  const void* clov;    // packed clover of this precision
  DGeom g;
  int parity;          // output parity
  int nblocks;         // filled by the launcher
  double coeff;        // multiplies the (post-processed) hopping term
  int nrhs = 1;        // right-hand sides: out, in, x hold nrhs spinors
  size_t rstride = 0;  // bytes between consecutive right-hand sides
  int threads = 0;     // launch shape: threads per block (64, 128, 256; 0 = 256)
  int group = 0;       // right-hand sides per thread (1, 2, 4; 0 = default); -1: one per thread, the
                       // right-hand sides of a site block in consecutive workgroups (fields shared in L2)
  int fprec = -1;      // storage of gauge and clover (-1: as the spinors; F16 with F32 spinors)
  int stream = -1;     // non-temporal field loads: 1 on, 0 off, -1 when the fields exceed the Infinity Cache
};
void launch_dslash(int prec, int diag, bool postinv, const DslashArgs& a, hipStream_t st);
struct RedOut;
// DIAG = 1 hop (out = x + coeff H in, one right-hand side, F64 or F32 spinors)
// that also reduces <out, x> (res[0..2)) and ||out||^2 (res[2]) into o in the
// same launch; false (nothing launched) where it does not apply
bool launch_dslash_red(int prec, const DslashArgs& a, const RedOut& o, hipStream_t st);
// minimal-residual update e += a r, r -= a Ar (a = coef[0..2) / coef[2]) fused
// with out = A_p^-1 r on parity p; false (nothing launched) for other precisions
bool launch_clover_mr(int prec, void* out, void* r, void* e, const void* Ar, const double* coef, const void* clov,
                      int Vh, int p, int fprec, hipStream_t st);
// several lattices (one right-hand side each, same precision and kernel variant) in one launch
constexpr int kMaxMulti = 4;
struct DslashMulti {
  DslashArgs a[kMaxMulti];
  int nl;
  int off[kMaxMulti + 1];  // block offsets, filled by the launcher
};
void launch_dslash_multi(int prec, int diag, bool postinv, const DslashMulti& m, hipStream_t st);
struct CloverMulti {
  void* out[kMaxMulti];
  const void* in[kMaxMulti];
  const void* clov[kMaxMulti];
  int Vh[kMaxMulti];
  int nl, parity, kind;
  int off[kMaxMulti + 1];
};
void launch_clover_multi(int prec, CloverMulti m, hipStream_t st);
// out_r = A^(kind) in_r for nrhs spinors rstride bytes apart
void launch_clover(int prec, void* out, const void* in, const void* clov, int Vh, int p, int kind,
                   hipStream_t st, int nrhs = 1, size_t rstride = 0, int fprec = -1);

// ------------------------------------------------------------ fields
// canonical complex128 gauge [V][4][3][3] (device) -> internal links
void gauge_to_internal(int prec, void* dst, const void* canon, const Geom& g, hipStream_t st);
// canonical complex128 spinor [V][12] (device) <-> two internal parity halves
void spinor_to_internal(int prec, void* even, void* odd, const void* canon, const Geom& g, bool g5,
                        hipStream_t st);
// odd == nullptr writes zeros on odd sites; even == nullptr writes zeros on even sites
void spinor_from_internal(int prec, void* canon, const void* even, const void* odd, const Geom& g, bool g5,
                          hipStream_t st);
// one parity, any precision pair
void spinor_convert(int prec_dst, void* dst, int prec_src, const void* src, int Vh, hipStream_t st);
void spinor_gamma5(int prec, void* v, int Vh, hipStream_t st);
// keep only the components of chirality chi (0: spins 0,1; 1: spins 2,3)
void spinor_chiral_project(int prec, void* dst, const void* src, int Vh, int chi, hipStream_t st);

struct CloverCoef {
  double s[6][2][4][2];  // [plane][chirality][2x2 entry][re,im] = csw (i/2) sigma_mu_nu block
};
// packed A and A^-1 (FP64) for both parities from the gauge field; flag[0]
// is set to 1 if a block is not positive definite
void clover_compute(void* clov64, const void* gauge64, const Geom& g, double m0, const CloverCoef& cc,
                    int* flag, hipStream_t st);
// packed A and A^-1 from a canonical complex128 [V][12][12] matrix
void clover_from_matrix(void* clov64, const void* A, const Geom& g, int* flag, hipStream_t st);
// gauge-link gradient from (x, lambda) pairs in canonical layout; cc = null
// skips the clover part; zbuf holds 6*9*V complex doubles
void force_compute(void* G, const void* x, const void* lam, int nrhs, const void* gauge64, const Geom& g,
                   const CloverCoef* cc, void* zbuf, hipStream_t st);
void reals_convert(int prec_dst, void* dst, const double* src, size_t n, hipStream_t st);
// packed FP64 clover (both parities, A and A^-1) -> the chunked layout of prec (F32, F16)
void clover_relayout(int prec, void* dst, const double* src, int Vh, hipStream_t st);

// ------------------------------------------------------------ BLAS-1
// Flat complex vectors of n elements, storage double (prec F64) or float (F32).
// Reductions accumulate in double and are deterministic (grid fixed by n,
// per-block partials summed in block order by a one-block second pass).
constexpr int kRedBlocks = 512;
struct RedOut {
  double* res;        // device result
  double* partial;    // kRedBlocks * 32 doubles of per-block partials
  unsigned* counter;  // arrival counter of the in-launch finish (zero between launches)
  double* hres;       // optional second destination of the result (nullptr: none)
  RedOut at(int off) const { return RedOut{res + off, partial, counter, hres ? hres + off : nullptr}; }
};
void blas_zero(int prec, void* x, size_t n, hipStream_t st);
// y (storage prec_dst) = x (storage prec_src), n complex elements
void blas_convert(int prec_dst, void* y, int prec_src, const void* x, size_t n, hipStream_t st);
void blas_copy(int prec, void* y, const void* x, size_t n, hipStream_t st);
// y = a*x + b*y (complex a, b)
void blas_axpby(int prec, double ar, double ai, const void* x, double br, double bi, void* y, size_t n,
                hipStream_t st);
// res[0] = ||x||^2
void blas_norm2(int prec, const void* x, size_t n, const RedOut& o, hipStream_t st);
// res[0..1] = <x,y> = sum conj(x) y
void blas_cdot(int prec, const void* x, const void* y, size_t n, const RedOut& o, hipStream_t st);
// res[0..1] = <x,y>, res[2] = ||x||^2
void blas_cdot_norm(int prec, const void* x, const void* y, size_t n, const RedOut& o, hipStream_t st);
// res[2j..2j+1] = <v_j, y> for j < k (writes up to 2*(k rounded up to 16) slots)
void blas_multi_cdot(int prec, const void* const* v, int k, const void* y, size_t n, const RedOut& o,
                     hipStream_t st);
// y += sum_j c_j v_j  (c on host)
void blas_multi_axpy(int prec, const double* c, const void* const* v, int k, void* y, size_t n, hipStream_t st);
// y += a x ; res[0] = ||y||^2
void blas_axpy_norm(int prec, double ar, double ai, const void* x, void* y, size_t n, const RedOut& o,
                    hipStream_t st);
// BiCGStab: x += a p + w s ; r = s - w t ; res = [||r||^2, <rhat, r>]
void blas_bicg_update(int prec, double ar, double ai, double wr, double wi, const void* p, const void* s,
                      const void* t, void* x, void* r, const void* rhat, size_t n, const RedOut& o, hipStream_t st);
// BiCGStab: p = r + b (p - w v)
void blas_bicg_p(int prec, double br, double bi, double wr, double wi, const void* r, const void* v, void* p,
                 size_t n, hipStream_t st);
// MR: x += a r ; r -= a Ar
void blas_mr_update(int prec, double ar, double ai, void* x, void* r, const void* Ar, size_t n, hipStream_t st);

// Device-resident GCR coefficients: slot j of qa holds {||q_j||^2, <q_j,r>, ||r||^2
// after step j}; beta holds the multi-dot <q_j, y>.  No host round trip.
// x += sum_j alpha_j z_j
// qa[4j..4j+3] = {1, dots[2j], dots[2j+1], 0} for j < K (coefficients x += sum_j dots_j z_j
// for blas_gcr_update_x_dev)
void blas_defl_coefs(const double* dots, double* qa, int K, hipStream_t st);
void blas_gcr_update_x_dev(int prec, const void* const* z, int k, void* x, size_t n, const double* qa,
                           hipStream_t st);
// One step of the GCR kept with raw preconditioned directions, after
// blas_multi_cdot of y against {q_0 .. q_{k-1}, y, r} into beta: y -= sum_j
// (beta_j/||q_j||^2) q_j; ||y||^2 by the Pythagorean sum and <y, r> (r is
// orthogonal to every q_j) into qa[4k], qa[4k+1..2]; r -= alpha y; ||r||^2
// into o; the coefficients beta_j/||q_j||^2 into cj[0 .. 2k)
void blas_gcr_step_dev(int prec, const void* const* q, int k, void* y, void* r, size_t n, const double* beta,
                       double* qa, double* cj, const RedOut& o, hipStream_t st);
// x += sum_j alpha_j z~_j for a cycle of kt slots (nf fixed ones first) kept as
// raw z_j: z~_j = z_j - sum_{i<j} c_ij z~_i with c_ij = cmat[2 (j ldc + i) ..];
// y (2 kt doubles of device scratch) receives the coefficients on the raw z_j
void blas_gcr_update_x_raw(int prec, const void* const* z, int nf, int kt, void* x, size_t n, const double* qa,
                           const double* cmat, int ldc, double* y, hipStream_t st);
// MR with alpha = coef[0..1] / coef[2] (the output of blas_cdot_norm(Ar, r))
void blas_mr_update_dev(int prec, const double* coef, void* x, void* r, const void* Ar, size_t n, hipStream_t st);

// ------------------------------------------------------------ batched BLAS-1
// nrhs vectors of n complex elements, vstride elements apart; results of right-hand
// side r at res + r * rs; part: scratch of kMaxBatch * kRedBlocks * 32 doubles
constexpr int kMaxBatch = 16;
struct RedB {
  double* res;
  size_t rs;
  double* part;
};
void blas_norm2_b(int prec, const void* x, size_t vs, size_t n, int nrhs, const RedB& o, hipStream_t st);
void blas_cdot_norm_b(int prec, const void* x, const void* y, size_t vs, size_t n, int nrhs, const RedB& o,
                      hipStream_t st);
void blas_multi_cdot_b(int prec, const void* const* v, int k, const void* y, size_t vs, size_t n, int nrhs,
                       const RedB& o, hipStream_t st);
// blas_gcr_step_dev / blas_gcr_update_x_raw for every right-hand side (rows of
// beta, qa, cj / cmat and y bs, qs, cjs / cms and ys doubles apart)
void blas_gcr_step_b(int prec, const void* const* q, int k, void* y, void* r, size_t vs, size_t n, int nrhs,
                     const double* beta, size_t bs, double* qa, size_t qs, double* cj, size_t cjs, const RedB& o,
                     hipStream_t st);
void blas_gcr_update_x_raw_b(int prec, const void* const* z, int kt, void* x, size_t vs, size_t n, int nrhs,
                             const double* qa, size_t qs, const double* cmat, size_t cms, int ldc, double* y,
                             size_t ys, hipStream_t st);
void blas_mr_update_b(int prec, const double* coef, size_t cs, void* x, void* r, const void* Ar, size_t vs, size_t n,
                      int nrhs, hipStream_t st);

// ------------------------------------------------------------ transfer (fine level)
struct BlockGeom {
  int b[4];    // block extents
  int nb[4];   // coarse extents
  int Vc;      // coarse sites
  int bvol;    // block volume
  int coarse_cb;  // 1 if coarse sites are stored parity-split (all nb even)
};
// coarse internal index of coarse lexicographic site
int coarse_internal_index_host(const BlockGeom& bg, int lex);

// R: coarse[c][s*Nv+k] (+)= sign(s) sum conj(V_k) in over fine sites of parity p
// vecs: Nv full-lattice spinors (precision prec) in internal layout
// out_site_stride/out_row_stride are in complex elements; accumulate: add into out
// vbm (FP32 only, optional): the block-major copy of vecs (launch_vec_blockmajor),
// read instead of vecs with the same arithmetic (coalesced loads); vbm16 (FP32
// only, optional): the FP16 copy of vbm (launch_chunks_to_half), read instead of both
void launch_restrict(int prec, void* out, size_t out_site_stride, size_t out_row_stride, const void* in,
                     const void* vecs, int nvec, int p, const Geom& g, const BlockGeom& bg, bool accumulate,
                     hipStream_t st, const void* vbm = nullptr, const void* vbm16 = nullptr);
// out (same size as v32) = the FP32 vectors v32 block by block: float4 chunk c of
// the l-th site (restriction order) of parity p of block b of vector k at
// (((k 2 + p) Vc + b) 6 + c) (bvol / 2) + l
void launch_vec_blockmajor(void* out, const void* v32, int nvec, const Geom& g, const BlockGeom& bg, hipStream_t st);
// P: out_p(x) = sum_k V_k(x) coarse[c(x)][s*Nv+k]; v16 (FP32 only, optional): the FP16
// copy of the FP32 vectors (launch_chunks_to_half), read instead of vecs
void launch_prolong(int prec, void* out, const void* coarse, const void* vecs, int nvec, int p, const Geom& g,
                    const BlockGeom& bg, hipStream_t st, const void* v16 = nullptr);
// FP16 copy of nchunks float4 chunks (two complex FP32 each): uint2 per chunk
void launch_chunks_to_half(void* out, const void* in32, size_t nchunks, hipStream_t st);
// block x chirality Gram-Schmidt (twice) of Nv full-lattice FP64 spinors in place
void launch_block_orthonormalize(void* vecs, int nvec, const Geom& g, const BlockGeom& bg, int* flag,
                                 hipStream_t st);
// coarse build: nine direction buckets of the D_p hop of u = A^-1 v (both parities)
void launch_hop_split(void* const* buckets /*9 full spinors F64*/, const void* v, const void* u,
                      const void* gauge64, const Geom& g, const BlockGeom& bg, hipStream_t st);

// ------------------------------------------------------------ matrix-core coarse stencil
struct CoarseGeom;
// FP16 operand fragments of Yt (from the FP64 [site][8][n][n] column-major blocks);
// flag[0] = 1 if an entry is outside the FP16 range
bool mfma_coarse_supported(int n);
size_t mfma_fragment_bytes(int nsites, int n);
void build_mfma_fragments(void* frag, const void* Yt64, int nsites, int n, int* flag, hipStream_t st);
// red-black coarse hop of nrhs FP32 right-hand sides (vs elements apart) on the matrix cores:
// out(c) = x(c) (if x) + coeff sum_d Yt_d(c) in(nb(c, d)) over the sites of `parity`
void launch_coarse_hop_mfma(void* out, const void* in, const void* x, const void* frag, double coeff, int parity,
                            const CoarseGeom& cg, const int* nbr, int nrhs, size_t vs, hipStream_t st);

// ------------------------------------------------------------ deeper levels
// transfer between coarse level l and l+1 (vectors [site][nf], V: nvec such
// vectors with stride vstride; members [nblocks][bvol], blk [nsites])
void launch_ctr_restrict(int prec, void* out, size_t out_site_stride, size_t out_rhs_stride, const void* in,
                         size_t in_rhs_stride, const void* V, size_t vstride, const int* members, int nblocks,
                         int bvol, int nf, int nvec, int nrhs, hipStream_t st);
void launch_ctr_prolong(int prec, void* out, size_t out_rhs_stride, const void* in, size_t in_rhs_stride,
                        const void* V, size_t vstride, const int* blk, int nsites, int nf, int nvec, int nrhs,
                        hipStream_t st);
// block x chirality Gram-Schmidt (twice) of FP64 level vectors in place
void launch_ctr_block_ortho(void* V, size_t vstride, const int* members, int nblocks, int bvol, int nf, int nvec,
                            int* flag, hipStream_t st);
// nine direction buckets of the level-l hop of u (Yhop [site][8][n][n] column-major, FP64), bucket 0 += v
void launch_chop_split(void* const* buckets, const void* v, const void* u, const void* Yhop, const int* nbr,
                       const int* blk, int nsites, int n, hipStream_t st);
void launch_unit_fill(void* e, int nsites, int n, int j, hipStream_t st);
// dense FP64 inverse of the full stencil Y9 into the augmented M [N][2N] (right half)
void dense_inverse_build(void* M, const void* Y9, const int* nbr, int nsites, int n, int* piv, void* pval, void* f,
                         int* flag, hipStream_t st);
// x = M^-1 b (b, x in prec F64 or F32)
void dense_inverse_apply(int prec, const void* M, int N, const void* b, void* x, hipStream_t st);

// ------------------------------------------------------------ coarse level
struct CoarseGeom {
  int L[4];
  int V;
  int Vh;      // V/2 when parity split, else V
  int split;   // sites stored parity-split
  int n;       // 2*Nv
};
// out(c) = DIAG + coeff * sum_d M_d(c) in(nb(c, d)) over sites of `parity`
// (parity -1: all sites, requires split == 0 or both halves contiguous)
// M: [site][8][n][n] column-major blocks.  diag 0 none, 1 x, 2 X(c) x with Xmat
void launch_coarse_hop(int prec, void* out, const void* in, const void* x, const void* M, const void* Xmat,
                       int diag, double coeff, int parity, const CoarseGeom& cg, const int* nbr, hipStream_t st,
                       int nrhs = 1, size_t vs = 0, bool rb = false);
// out(c) = M(c) in(c) with M [site][n][n] column-major, sites of `parity` (-1 all)
void launch_coarse_local(int prec, void* out, const void* in, const void* M, int parity, const CoarseGeom& cg,
                         hipStream_t st, int nrhs = 1, size_t vs = 0);
void launch_batched_inverse(double* M, int nmat, int n, int* flag, hipStream_t st);
// Whole approximate coarse solve (red-black reduced operator, GCR(restart)
// from zero, stopping at ||r|| <= tol ||b_r|| or after maxiter steps; fixed:
// exactly min(restart, maxiter) steps) in one cooperative launch of `grid`
// (<= 256) workgroups.  Buffers: b, c, t [V][n]; y, br, r, qraw [Vh][n];
// Q, Z [restart][Vh][n]; T [restart][V][n]; part 2 * grid * coarse_gcr_persistent_part_doubles();
// bar: kPersistCtlBytes of barrier lines (zeroed before the first launch;
// consistent after every completed launch, zeroed again after an abort): the
// grid barrier below 33 KiB, the neighbour flags from kPersistLocalOffset;
// info [3] (at bar + kPersistInfoOffset bytes in the library's use):
// iterations are added to info[0], a failure code goes to info[1], info[2] is
// raised when a barrier wait timed out.  With grid == Vh every workgroup owns
// one even and one odd site and the one-site kernel runs (Krylov basis in
// LDS, neighbour flags instead of a second grid barrier per step) unless
// `general` is set or the basis does not fit; otherwise sites are strided
// over the workgroups.
constexpr size_t kPersistCtlBytes = 68 * 1024;
constexpr size_t kPersistInfoOffset = 34 * 1024;
constexpr size_t kPersistLocalOffset = 36 * 1024;
struct CoarseGcrArgs {
  const void* Yt;
  const void* Xinv;
  const int* nbr;
  const void* b;
  void* c;
  void* t;
  void* y;
  void* r;
  void* br;
  void* Q;
  void* Z;
  void* T;
  void* qraw;
  double* part;
  unsigned* bar;
  int* info;
  double tol;
  int Vh, n, restart, maxiter, fixed, grid;
  int general;  // always the strided kernel
  int trust;    // a cycle that met the tolerance by its recurrence residual ends the solve without
                // recomputing the true residual (for a preconditioner's loose tolerance)
  int mat16;    // Yt holds FP16 hop blocks (FP32 vectors and arithmetic)
  void* tags;   // tagged slots of the one-site FP32 kernel (coarse_gcr_persistent_tag_bytes; zeroed
                // whenever the barrier lines are; nullptr: flags and barriers at every step)
  size_t tag_bytes;
};
size_t coarse_gcr_persistent_part_doubles();
// bytes of the tagged slots for a coarse level of Vh sites per parity, n components, grid workgroups
size_t coarse_gcr_persistent_tag_bytes(int n, int Vh, int grid);
// workgroups of the persistent coarse solve on this device (0: not available)
int coarse_gcr_persistent_grid(int prec, int n, int Vh);
void launch_coarse_gcr_persistent(int prec, const CoarseGcrArgs& a, hipStream_t st);

// Yt[c][d] = Y[c][d] * Xinv[nb(c,d)]   (all column-major n x n)
void launch_coarse_right_mul(double* Yt, const double* Y, const double* Xinv, const int* nbr, int V, int n,
                             hipStream_t st);
// canonical complex128 [lex][n] <-> internal [perm[lex]][n] (F64 or F32)
void launch_coarse_canon(int prec, void* internal, void* canon, const int* perm, int V, int n, bool to_internal,
                         hipStream_t st);
void launch_reals_convert(int prec_dst, void* dst, const double* src, size_t n, hipStream_t st);

}  // namespace wcmg
