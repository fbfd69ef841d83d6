"""Adaptive multigrid pieces in plain FP64 (oracle; test infrastructure only).

Follows the paper's description:
* setup (Setup procedure section): for each vector, repeated relaxation
  (inverse iteration) on a random vector, monitoring the Rayleigh quotient
  v^dag D^dag D v / v^dag v, keeping the vector globally orthogonal to the
  previously converged ones.  The operator relaxed on is D_p, whose low
  modes form P (red-black paragraph).  Counts and thresholds are not given
  in the paper; the readings are: relaxation = n_relax GCR steps on
  D_p x = v from zero, stop when |d rho|/rho < delta or after s_max steps.
* P is split into space-time blocks x 2 chiralities; within every (block,
  chirality) the vectors are orthonormalized (Gram-Schmidt in order, done
  twice: the thin QR with real positive diagonal).
* R = P^dag gamma5, coarse operator Yhat = R D_p P.
* the coarse system is solved with red-black preconditioning again; every
  level runs GCR preconditioned by the next level's cycle and the coarsest
  runs unpreconditioned GCR (Implementation paragraph), to a per-level
  relative tolerance (about 0.1 is reported best).
* the smoother (type not given) is MR on the level's reduced operator,
  applied after the coarse correction.
* the adaptive refinement the Setup section describes as the alphaSA idea
  (relax with a cycle built from the vectors at hand) combined with the
  inverse-iteration setup ("hybrid"); the paper leaves its details open, so
  it is parity unpinned (invariants only, like the setup itself).

Coarse fields are arrays [Vc][2*Nv]; coarse component s*Nv + k has chirality
s (s = 0 for gamma5 = +1).  The coarse operator is stored as
Y[Vc][9][2Nv][2Nv]: slot 0 is the site-local block X, slot 1+d the hop
towards direction d = 2*mu (+mu) or 2*mu+1 (-mu).
"""
import numpy as np

from .krylov import gcr, mr, norm, SolveInfo
from .lattice import Lattice
from .philox import gaussian_vector


class RankError(RuntimeError):
    pass


# ----------------------------------------------------------------------------
# coarse operator
# ----------------------------------------------------------------------------

class CoarseOperator:
    """Stencil X(c) v(c) + sum_d Y_d(c) v(c + d) with red-black pieces."""

    def __init__(self, dims, Y):
        self.lat = Lattice(dims, t_bc=1)
        self.Y = np.asarray(Y, dtype=np.complex128)
        Vc, nine, n, _ = self.Y.shape
        assert Vc == self.lat.V and nine == 9 and n % 2 == 0
        self.n = n
        self.nvec = n // 2
        self.ncomp = n
        self.shape = (Vc, n)
        self.A = self.Y[:, 0]
        self.Ainv = np.linalg.inv(self.A)
        self.chirality = np.repeat([0, 1], self.nvec)
        self.even_dims = all(d % 2 == 0 for d in self.lat.dims)

    def vec(self, v):
        return np.asarray(v, dtype=np.complex128).reshape(self.shape)

    def nbr(self, d):
        mu, back = divmod(d, 2)
        return self.lat.bwd[mu] if back else self.lat.fwd[mu]

    def _diag(self, M, v, sites):
        v = self.vec(v)
        if sites is None:
            return np.einsum("cij,cj->ci", M, v)
        out = np.zeros(self.shape, dtype=np.complex128)
        out[sites] = np.einsum("cij,cj->ci", M[sites], v[sites])
        return out

    def apply_A(self, v, sites=None):
        return self._diag(self.A, v, sites)

    def apply_Ainv(self, v, sites=None):
        return self._diag(self.Ainv, v, sites)

    def apply_H_dir(self, v, d, sites=None):
        v = self.vec(v)
        s = np.arange(self.lat.V) if sites is None else sites
        out = np.zeros(self.shape, dtype=np.complex128)
        out[s] = np.einsum("cij,cj->ci", self.Y[s, 1 + d], v[self.nbr(d)[s]])
        return out

    def apply_H(self, v, sites=None):
        out = np.zeros(self.shape, dtype=np.complex128)
        for d in range(8):
            out += self.apply_H_dir(v, d, sites)
        return out

    def gamma5(self, v):
        v = self.vec(v).copy()
        v[:, self.nvec:] *= -1
        return v

    def apply_D(self, v):
        return self.apply_A(v) + self.apply_H(v)

    def apply_Dp(self, v):
        return self.apply_D(self.apply_Ainv(v))

    def apply_Dr(self, y):
        lat = self.lat
        y = self.vec(y)
        z = self.apply_Ainv(y, lat.even)
        w = self.apply_Ainv(self.apply_H(z, lat.odd), lat.odd)
        out = np.zeros(self.shape, dtype=np.complex128)
        out[lat.even] = y[lat.even] - self.apply_H(w, lat.even)[lat.even]
        return out

    def reduced_source(self, b):
        lat = self.lat
        b = self.vec(b)
        w = self.apply_Ainv(b, lat.odd)
        out = np.zeros(self.shape, dtype=np.complex128)
        out[lat.even] = b[lat.even] - self.apply_H(w, lat.even)[lat.even]
        return out

    def reconstruct(self, y, b):
        lat = self.lat
        b = self.vec(b)
        x = self.apply_Ainv(y, lat.even)
        t = np.zeros(self.shape, dtype=np.complex128)
        t[lat.odd] = b[lat.odd] - self.apply_H(x, lat.odd)[lat.odd]
        x[lat.odd] = self.apply_Ainv(t, lat.odd)[lat.odd]
        return x

    def dense(self):
        """Dense matrix of the full coarse operator (small lattices only)."""
        Vc, n = self.shape
        M = np.zeros((Vc, n, Vc, n), dtype=np.complex128)
        for c in range(Vc):
            M[c, :, c, :] += self.Y[c, 0]
            for d in range(8):
                M[c, :, self.nbr(d)[c], :] += self.Y[c, 1 + d]
        return M.reshape(Vc * n, Vc * n)


# ----------------------------------------------------------------------------
# transfer operators
# ----------------------------------------------------------------------------

def block_map(dims, blocks):
    """Coarse lattice dims and the block (coarse site) of every fine site."""
    dims = tuple(int(d) for d in dims)
    blocks = tuple(int(b) for b in blocks)
    for L, b in zip(dims, blocks):
        if b <= 0 or L % b:
            raise ValueError("block %s does not divide lattice %s" % (blocks, dims))
    cdims = tuple(L // b for L, b in zip(dims, blocks))
    lat = Lattice(dims, t_bc=1)
    cc = lat.coords // np.array(blocks)
    clat = Lattice(cdims, t_bc=1)
    return cdims, clat.index(cc)


def block_orthonormalize(vecs, block_of, chirality, nblocks, rank_tol=1e-12):
    """Per (block, chirality): Gram-Schmidt in order k = 0..Nv-1, twice.

    vecs: [Nv][nsites][ncomp].  Returns the orthonormalized copy.
    """
    vecs = np.array(vecs, dtype=np.complex128, copy=True)
    nv, nsites, ncomp = vecs.shape
    order = np.argsort(block_of, kind="stable")
    bsize = nsites // nblocks
    sites_of_block = order.reshape(nblocks, bsize)
    out = np.zeros_like(vecs)
    for s in (0, 1):
        comps = np.nonzero(chirality == s)[0]
        # M[b][k][rows]: rows = (site in block, component of chirality s)
        M = vecs[:, sites_of_block][:, :, :, comps]           # [Nv][nb][bsize][nc]
        M = np.moveaxis(M, 0, 1).reshape(nblocks, nv, -1)     # [nb][Nv][rows]
        Q = np.zeros_like(M)
        for k in range(nv):
            v = M[:, k].copy()
            n0 = np.sqrt(np.sum(np.abs(v) ** 2, axis=1))
            for _ in range(2):
                if k:
                    coef = np.einsum("bjr,br->bj", np.conj(Q[:, :k]), v)
                    v = v - np.einsum("bj,bjr->br", coef, Q[:, :k])
            nk = np.sqrt(np.sum(np.abs(v) ** 2, axis=1))
            if np.any(nk <= rank_tol * n0) or np.any(nk == 0):
                raise RankError("null vectors are linearly dependent on a block")
            Q[:, k] = v / nk[:, None]
        Q = Q.reshape(nblocks, nv, bsize, len(comps))
        Q = np.moveaxis(Q, 1, 0)                               # [Nv][nb][bsize][nc]
        tmp = out[:, sites_of_block]
        tmp[..., comps] = Q
        out[:, sites_of_block] = tmp
    return out


class Transfer:
    """P (block x chirality split of the null vectors) and R = P^dag gamma5."""

    def __init__(self, op, blocks, vecs):
        self.op = op
        self.blocks = tuple(blocks)
        self.cdims, self.block_of = block_map(op.lat.dims, blocks)
        self.Vc = int(np.prod(self.cdims))
        vecs = np.asarray(vecs, dtype=np.complex128).reshape((-1,) + (op.lat.V, op.ncomp))
        self.nvec = vecs.shape[0]
        self.chi = op.chirality
        self.V = block_orthonormalize(vecs, self.block_of, self.chi, self.Vc)

    def prolong(self, c):
        """e(x, a) = sum_k V_k(x, a) c(block(x), chi(a), k)."""
        c = np.asarray(c, dtype=np.complex128).reshape(self.Vc, 2, self.nvec)
        coef = c[self.block_of][:, self.chi, :]                # [nsites][ncomp][Nv]
        e = np.einsum("kna,nak->na", self.V, coef)
        return e.reshape(self.op.shape)

    def restrict(self, r):
        """c(b, s, k) = (+1 | -1)_s sum_{x in b, chi(a)=s} conj(V_k(x,a)) r(x,a)."""
        r = np.asarray(r, dtype=np.complex128).reshape(self.op.lat.V, self.op.ncomp)
        prod = np.einsum("kna,na->nak", np.conj(self.V), r)
        c = np.zeros((self.Vc, 2, self.nvec), dtype=np.complex128)
        np.add.at(c, (self.block_of[:, None], self.chi[None, :]), prod)
        c[:, 1] *= -1
        return c.reshape(self.Vc, 2 * self.nvec)

    def dense_P(self):
        n_f = self.op.lat.V * self.op.ncomp
        n_c = self.Vc * 2 * self.nvec
        P = np.zeros((n_f, n_c), dtype=np.complex128)
        e = np.zeros(n_c, dtype=np.complex128)
        for j in range(n_c):
            e[j] = 1
            P[:, j] = self.prolong(e).reshape(-1)
            e[j] = 0
        return P


# ----------------------------------------------------------------------------
# coarse-operator construction
# ----------------------------------------------------------------------------

def coarse_operator(op, T):
    """Yhat = R D_p P, direction-resolved.

    For every coarse column j = (s, k) the unit vector is prolonged on all
    blocks at once, D_p = A + H acting on M^-1 P e_j is split by which block
    each hop comes from, and every bucket is restricted.
    """
    n = 2 * T.nvec
    Y = np.zeros((T.Vc, 9, n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros((T.Vc, n), dtype=np.complex128)
        e[:, j] = 1.0
        v = T.prolong(e)
        u = op.apply_Ainv(v)
        buckets = np.zeros((9,) + op.shape, dtype=np.complex128)
        buckets[0] = v                                  # D_p = A A^-1 + H A^-1
        for d in range(8):
            hd = op.apply_H_dir(u, d)
            cross = T.block_of[op.nbr(d)] != T.block_of
            buckets[0][~cross] += hd[~cross]
            buckets[1 + d][cross] += hd[cross]
        for slot in range(9):
            Y[:, slot, :, j] = T.restrict(buckets[slot])
    return Y


def coarse_operator_brute_force(op, T):
    """Dense R D_p P, one single-block column at a time (no direction split)."""
    n_c = T.Vc * 2 * T.nvec
    Yd = np.zeros((n_c, n_c), dtype=np.complex128)
    e = np.zeros(n_c, dtype=np.complex128)
    for j in range(n_c):
        e[j] = 1.0
        Yd[:, j] = T.restrict(op.apply_Dp(T.prolong(e))).reshape(-1)
        e[j] = 0.0
    return Yd


# ----------------------------------------------------------------------------
# setup: inverse iteration with Rayleigh-quotient monitoring
# ----------------------------------------------------------------------------

def setup_null_vectors(op, nvec, seed, level=0, n_relax=10, s_max=10, delta=0.05,
                       stats=None):
    """Near-null vectors of D_p by repeated relaxation on random vectors."""
    dim = op.lat.V * op.ncomp
    found = []
    for k in range(nvec):
        v = gaussian_vector(seed, k, level, dim).reshape(op.shape)
        rho_old = None
        steps = 0
        for _ in range(s_max):
            v = gcr(op.apply_Dp, v, tol=0.0, restart=n_relax, maxiter=n_relax)
            for _pass in range(2):
                for w in found:
                    v = v - np.vdot(w, v) * w
            v = v / norm(v)
            rho = norm(op.apply_Dp(v)) ** 2
            steps += 1
            if rho_old is not None and abs(rho - rho_old) / rho < delta:
                break
            rho_old = rho
        if stats is not None:
            stats.append((steps, rho))
        found.append(v)
    return np.stack(found)


# ----------------------------------------------------------------------------
# recursive GCR / multigrid cycle
# ----------------------------------------------------------------------------

class MGParams:
    def __init__(self, blocks, nvec, tol=0.1, maxiter=50, restart=10, nu_post=4,
                 outer_restart=16, outer_maxiter=500, n_relax=10, s_max=10,
                 delta=0.05, seed=0, coarsest="gcr"):
        self.blocks = [tuple(b) for b in blocks]
        self.nvec = list(nvec)
        self.tol = tol
        self.maxiter = maxiter
        self.restart = restart
        self.nu_post = nu_post
        self.outer_restart = outer_restart
        self.outer_maxiter = outer_maxiter
        self.n_relax = n_relax
        self.s_max = s_max
        self.delta = delta
        self.seed = seed
        self.coarsest = coarsest


class Hierarchy:
    """ops[0] = fine operator, transfers[l] maps level l+1 -> l, ops[l+1] coarse."""

    def __init__(self, op, params, vecs=None):
        self.params = params
        self.ops = [op]
        self.transfers = []
        self.raw = []  # the vectors each level's P was built from
        for l, (blk, nv) in enumerate(zip(params.blocks, params.nvec)):
            cur = self.ops[-1]
            if vecs is not None and vecs[l] is not None:
                v = vecs[l]
            else:
                v = setup_null_vectors(cur, nv, params.seed, level=l,
                                       n_relax=params.n_relax, s_max=params.s_max,
                                       delta=params.delta)
            T = Transfer(cur, blk, v)
            Y = coarse_operator(cur, T)
            self.raw.append(np.asarray(v, dtype=np.complex128).reshape((-1,) + cur.shape))
            self.transfers.append(T)
            self.ops.append(CoarseOperator(T.cdims, Y))
        self.inner_iters = [0] * len(self.ops)
        self.inner_calls = [0] * len(self.ops)

    def precond(self, l, r):
        """K(r_e) = even part of P (coarse solve) R (r_e, 0), then MR smoothing."""
        p = self.params
        op, T = self.ops[l], self.transfers[l]
        c = self.coarse_solve(l + 1, T.restrict(r))
        e = T.prolong(c)
        e[op.lat.odd] = 0
        return mr(op.apply_Dr, r, e, p.nu_post) if p.nu_post else e

    def coarse_solve(self, l, b):
        """Approximate solution of the level-l coarse system Yhat c = b."""
        p = self.params
        op = self.ops[l]
        last = l == len(self.ops) - 1
        info = SolveInfo()
        if last and p.coarsest == "lu":
            return np.linalg.solve(op.dense(), b.reshape(-1)).reshape(op.shape)
        if op.even_dims:
            br = op.reduced_source(b)
            pre = None if last else (lambda r: self.precond(l, r))
            y = gcr(op.apply_Dr, br, tol=p.tol, restart=p.restart, maxiter=p.maxiter,
                    precond=pre, info=info)
            x = op.reconstruct(y, b)
        else:
            x = gcr(op.apply_D, op.vec(b), tol=p.tol, restart=p.restart,
                    maxiter=p.maxiter, info=info)
        self.inner_iters[l] += info.iters
        self.inner_calls[l] += 1
        return x

    def solve(self, b, tol=1e-10, info=None):
        """Solve D x = b: red-black reduced GCR preconditioned by the cycle."""
        p = self.params
        op = self.ops[0]
        b = op.vec(b)
        br = op.reduced_source(b)
        y = gcr(op.apply_Dr, br, tol=tol, target_norm=norm(b), restart=p.outer_restart,
                maxiter=p.outer_maxiter, precond=lambda r: self.precond(0, r), info=info)
        return op.reconstruct(y, b)


def refine_null_vectors(H, passes=1, iters=4):
    """Adaptive refinement of the fine null vectors (Setup section; parity
    unpinned).  Each pass relaxes every vector v with `iters` steps of GCR on
    the homogeneous reduced system D_r y = 0, started from y = v_e and
    preconditioned by the current cycle; the odd half then follows from
    D_p v = 0, i.e. v_o = -D_oe D_ee^-1 v_e; the vectors are orthonormalised
    in order (twice) and the hierarchy is rebuilt on them (coarser levels
    keep their own vectors).  Returns the new Hierarchy."""
    op = H.ops[0]
    lat = op.lat
    for _ in range(passes):
        new = []
        for v in H.raw[0]:
            ye = np.zeros(op.shape, dtype=np.complex128)
            ye[lat.even] = v[lat.even]
            y = gcr(op.apply_Dr, np.zeros(op.shape, dtype=np.complex128), x0=ye, tol=0.0,
                    restart=max(H.params.outer_restart, iters), maxiter=iters,
                    precond=lambda r: H.precond(0, r))
            w = np.zeros(op.shape, dtype=np.complex128)
            w[lat.even] = y[lat.even]
            z = op.apply_Ainv(w, lat.even)
            w[lat.odd] = -op.apply_H(z, lat.odd)[lat.odd]
            for _rep in range(2):
                for u in new:
                    w = w - np.vdot(u, w) * u
            new.append(w / norm(w))
        vecs = [np.stack(new)] + H.raw[1:]
        H = Hierarchy(op, H.params, vecs=vecs)
    return H
