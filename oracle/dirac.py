"""Wilson-clover operator and its red-black split (oracle; test infrastructure only).

Operator of Eq.(1), with the mass absorbed into D as stated after Eq.(2):

    D psi(x) = A(x) psi(x) + (H psi)(x)
    (H psi)(x) = -1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
                             + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
    A(x) = (4 + m0) + csw * (i/4) sum_{mu != nu} sigma_mu_nu (x) Fhat_mu_nu(x)

Fhat_mu_nu = (Q_mu_nu - Q_mu_nu^dag)/8 with Q the sum of the four plaquette
leaves around x (Sheikholeslami-Wohlert clover; the paper names "clover
fermions" without a formula, this is the reading used).  The free-field
symbol of this D is m0 + sum_mu (1 - cos p_mu) + i sum_mu gamma_mu sin p_mu.

Red-black preconditioning (Eq.(2)): D_ee = A_e, D_oo = A_o, D_eo/D_oe = the
hopping blocks; D_p = D diag(D_ee, D_oo)^-1; the reduced operator of Eq.(3)
D_r = 1 - D_eo D_oo^-1 D_oe D_ee^-1, the reduced source of Eq.(4)
b_r = b_e - D_eo D_oo^-1 b_o, and the reconstruction x_e = D_ee^-1 y_e,
x_o = D_oo^-1 (b_o - D_oe x_e).

Anisotropic lattices (the Results section's lattices have a finer temporal
spacing; the paper gives no formula, this is the reading used): the spatial
hops carry a coefficient hop_s, the site-diagonal constant is
m0 + 1 + 3 hop_s, and the clover planes are weighted csw_s (spatial) and
csw_t (with time); hop_s = 1 and csw_s = csw_t give the operator above.

Fields are flat arrays: gauge U[V][4][3][3], spinors psi[V][4][3] (complex128).
Half-lattice (single parity) fields are stored as full-lattice arrays that
are zero on the other parity; every function below works that way.
"""
import numpy as np

from .lattice import GAMMA, GAMMA5, Lattice, sigma_munu

I4 = np.eye(4, dtype=np.complex128)


def dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


# ----------------------------------------------------------------------------
# hopping term
# ----------------------------------------------------------------------------

def hop_dir(lat, U, psi, d, sites, hop_s=1.0):
    """Contribution of hop direction d to (H psi) at `sites`.

    d = 2*mu is the forward hop  -1/2 c_mu (1-gamma_mu) U_mu(x) psi(x+mu),
    d = 2*mu+1 the backward hop  -1/2 c_mu (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu),
    c_mu = hop_s for the spatial directions and 1 for time.
    """
    mu, back = divmod(d, 2)
    if mu < 3 and hop_s != 1.0:
        return hop_s * hop_dir(lat, U, psi, d, sites)
    if not back:
        nb = lat.fwd[mu][sites]
        ph = lat.fwd_phase[mu][sites]
        link = U[sites, mu]
        t = np.einsum("nab,nsb->nsa", link, psi[nb]) * ph[:, None, None]
        return -0.5 * np.einsum("st,nta->nsa", I4 - GAMMA[mu], t)
    nb = lat.bwd[mu][sites]
    ph = lat.bwd_phase[mu][sites]
    link = U[nb, mu]
    t = np.einsum("nba,nsb->nsa", np.conj(link), psi[nb]) * ph[:, None, None]
    return -0.5 * np.einsum("st,nta->nsa", I4 + GAMMA[mu], t)


def hop(lat, U, psi, sites=None, hop_s=1.0):
    """(H psi)(x) for x in `sites` (all sites if None); returns [len(sites)][4][3]."""
    if sites is None:
        sites = np.arange(lat.V)
    out = np.zeros((len(sites), 4, 3), dtype=np.complex128)
    for d in range(8):
        out += hop_dir(lat, U, psi, d, sites, hop_s)
    return out


# ----------------------------------------------------------------------------
# clover term
# ----------------------------------------------------------------------------

def plaquette_sum(lat, U, mu, nu, sites):
    """Q_mu_nu(x): sum of the four same-orientation plaquette leaves at x.

    Leaves (all traversed mu-then-nu sense), using periodic links (the
    antiperiodic time phase cancels inside a closed loop):
      U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
      U_nu(x) U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu)
      U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu)
      U_nu(x-nu)^dag U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^dag
    """
    x = sites
    xpm, xpn = lat.fwd[mu][x], lat.fwd[nu][x]
    xmm, xmn = lat.bwd[mu][x], lat.bwd[nu][x]
    xmm_pn = lat.fwd[nu][xmm]
    xmm_mn = lat.bwd[nu][xmm]
    xpm_mn = lat.bwd[nu][xpm]

    def Um(s):
        return U[s, mu]

    def Un(s):
        return U[s, nu]

    l1 = Um(x) @ Un(xpm) @ dag(Um(xpn)) @ dag(Un(x))
    l2 = Un(x) @ dag(Um(xmm_pn)) @ dag(Un(xmm)) @ Um(xmm)
    l3 = dag(Um(xmm)) @ dag(Un(xmm_mn)) @ Um(xmm_mn) @ Un(xmn)
    l4 = dag(Un(xmn)) @ Um(xmn) @ Un(xpm_mn) @ dag(Um(x))
    return l1 + l2 + l3 + l4


def field_strength(lat, U, mu, nu, sites):
    """Fhat_mu_nu(x) = (Q_mu_nu - Q_mu_nu^dag) / 8 (anti-Hermitian 3x3)."""
    Q = plaquette_sum(lat, U, mu, nu, sites)
    return (Q - dag(Q)) / 8.0


def clover_term(lat, U, csw, sites=None, csw_t=None):
    """(i/4) sum_{mu != nu} c_mu_nu sigma_mu_nu (x) Fhat_mu_nu, as [n][12][12],
    c_mu_nu = csw on spatial planes and csw_t (default csw) on planes with time."""
    if sites is None:
        sites = np.arange(lat.V)
    csw_t = csw if csw_t is None else csw_t
    if csw_t != csw:
        space = [(m, n) for m in range(3) for n in range(3) if m != n]
        C = np.zeros((len(sites), 12, 12), dtype=np.complex128)
        for mu in range(4):
            for nu in range(4):
                if mu == nu:
                    continue
                F = field_strength(lat, U, mu, nu, sites)
                w = csw if (mu, nu) in space else csw_t
                C += w * np.einsum("st,nab->nsatb", sigma_munu(mu, nu), F).reshape(len(sites), 12, 12)
        return 0.25j * C
    C = np.zeros((len(sites), 12, 12), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            F = field_strength(lat, U, mu, nu, sites)
            s = sigma_munu(mu, nu)
            # component index spin*3 + colour  ->  kron(sigma, F)
            C += np.einsum("st,nab->nsatb", s, F).reshape(len(sites), 12, 12)
    return csw * 0.25j * C


def site_matrix(lat, U, m0, csw, sites=None, hop_s=1.0, csw_t=None):
    """A(x) = (m0 + 1 + 3 hop_s) 1 + clover term (4 + m0 when isotropic), per site [n][12][12]."""
    C = clover_term(lat, U, csw, sites, csw_t)
    diag = 4.0 + m0 if hop_s == 1.0 else m0 + 1.0 + 3.0 * hop_s
    return C + diag * np.eye(12)[None]


# ----------------------------------------------------------------------------
# the operator
# ----------------------------------------------------------------------------

class WilsonClover:
    """D = A + H on a lattice, with the red-black pieces of Eqs.(2)-(4)."""

    def __init__(self, dims, U, m0, csw, t_bc=-1, A=None, hop_s=1.0, csw_t=None):
        self.lat = Lattice(dims, t_bc)
        V = self.lat.V
        self.U = np.ascontiguousarray(np.asarray(U).reshape(V, 4, 3, 3))
        self.m0 = float(m0)
        self.csw = float(csw)
        self.csw_t = self.csw if csw_t is None else float(csw_t)
        self.hop_s = float(hop_s)
        self.A = (site_matrix(self.lat, self.U, m0, csw, hop_s=self.hop_s, csw_t=self.csw_t) if A is None
                  else A)
        self.Ainv = np.linalg.inv(self.A)
        self.shape = (V, 4, 3)
        self.ncomp = 12
        self.chirality = np.repeat([0, 0, 1, 1], 3)  # per component: 0 -> gamma5=+1

    # --- pieces ------------------------------------------------------------
    def vec(self, v):
        return np.asarray(v, dtype=np.complex128).reshape(self.shape)

    def diag(self, M, v, sites=None):
        v = self.vec(v)
        if sites is None:
            return np.einsum("nij,nj->ni", M, v.reshape(-1, 12)).reshape(self.shape)
        out = np.zeros(self.shape, dtype=np.complex128)
        out[sites] = np.einsum("nij,nj->ni", M[sites], v[sites].reshape(-1, 12)).reshape(-1, 4, 3)
        return out

    def apply_A(self, v, sites=None):
        return self.diag(self.A, v, sites)

    def apply_Ainv(self, v, sites=None):
        return self.diag(self.Ainv, v, sites)

    def apply_H(self, v, sites=None):
        """Hopping term evaluated at `sites`, zero elsewhere."""
        v = self.vec(v)
        out = np.zeros(self.shape, dtype=np.complex128)
        s = np.arange(self.lat.V) if sites is None else sites
        out[s] = hop(self.lat, self.U, v, s, self.hop_s)
        return out

    def apply_H_dir(self, v, d, sites=None):
        v = self.vec(v)
        out = np.zeros(self.shape, dtype=np.complex128)
        s = np.arange(self.lat.V) if sites is None else sites
        out[s] = hop_dir(self.lat, self.U, v, d, s, self.hop_s)
        return out

    def nbr(self, d):
        mu, back = divmod(d, 2)
        return self.lat.bwd[mu] if back else self.lat.fwd[mu]

    def gamma5(self, v):
        v = self.vec(v)
        return np.einsum("st,nta->nsa", GAMMA5, v)

    # --- full operators ----------------------------------------------------
    def apply_D(self, v):
        """Eq.(1): D psi = A psi + H psi on the whole lattice."""
        return self.apply_A(v) + self.apply_H(v)

    def apply_Ddag(self, v):
        """D^dag psi from the explicit adjoint of every term (A and H)."""
        v = self.vec(v)
        lat = self.lat
        out = np.einsum("nji,nj->ni", np.conj(self.A), v.reshape(-1, 12)).reshape(self.shape)
        acc = np.zeros(self.shape, dtype=np.complex128)
        for mu in range(4):
            c = self.hop_s if mu < 3 else 1.0
            # adjoint of the forward hop: -1/2 c_mu (1-gamma)^dag U_mu(x-mu)^dag psi(x-mu)
            nb = lat.bwd[mu]
            t = np.einsum("nba,nsb->nsa", np.conj(self.U[nb, mu]), v[nb]) * lat.bwd_phase[mu][:, None, None]
            acc += c * np.einsum("st,nta->nsa", dag(I4 - GAMMA[mu]), t)
            nb = lat.fwd[mu]
            t = np.einsum("nab,nsb->nsa", self.U[:, mu], v[nb]) * lat.fwd_phase[mu][:, None, None]
            acc += c * np.einsum("st,nta->nsa", dag(I4 + GAMMA[mu]), t)
        return out - 0.5 * acc

    def apply_Dp(self, v):
        """Left side of Eq.(2): D_p y = D diag(D_ee, D_oo)^-1 y."""
        return self.apply_D(self.apply_Ainv(v))

    # --- red-black (Eqs.(3)-(4)) ------------------------------------------
    def apply_Dr(self, y):
        """D_r y_e = y_e - D_eo D_oo^-1 D_oe D_ee^-1 y_e (zero on odd sites)."""
        lat = self.lat
        y = self.vec(y)
        z = self.apply_Ainv(y, lat.even)
        w = self.apply_Ainv(self.apply_H(z, lat.odd), lat.odd)
        out = np.zeros(self.shape, dtype=np.complex128)
        out[lat.even] = y[lat.even] - self.apply_H(w, lat.even)[lat.even]
        return out

    def apply_Dr_dag(self, y):
        """Adjoint of D_r: 1 - D_ee^-dag D_oe^dag D_oo^-dag D_eo^dag on even sites."""
        lat = self.lat
        y = self.vec(y)
        ye = np.zeros(self.shape, dtype=np.complex128)
        ye[lat.even] = y[lat.even]
        a = self.apply_Ddag(ye)                      # D^dag restricted below
        a_o = np.zeros(self.shape, dtype=np.complex128)
        a_o[lat.odd] = a[lat.odd]                    # D_eo^dag y_e
        b = np.einsum("nji,nj->ni", np.conj(self.Ainv), a_o.reshape(-1, 12)).reshape(self.shape)
        b[lat.even] = 0
        c = self.apply_Ddag(b)                       # D_oe^dag (on even sites)
        c_e = np.zeros(self.shape, dtype=np.complex128)
        c_e[lat.even] = c[lat.even]
        d = np.einsum("nji,nj->ni", np.conj(self.Ainv), c_e.reshape(-1, 12)).reshape(self.shape)
        out = np.zeros(self.shape, dtype=np.complex128)
        out[lat.even] = y[lat.even] - d[lat.even]
        return out

    def reduced_source(self, b):
        """b_r = b_e - D_eo D_oo^-1 b_o (Eq.(4)); zero on odd sites."""
        lat = self.lat
        b = self.vec(b)
        w = self.apply_Ainv(b, lat.odd)
        out = np.zeros(self.shape, dtype=np.complex128)
        out[lat.even] = b[lat.even] - self.apply_H(w, lat.even)[lat.even]
        return out

    def reconstruct(self, y, b):
        """x_e = D_ee^-1 y_e, x_o = D_oo^-1 (b_o - D_oe x_e)."""
        lat = self.lat
        b = self.vec(b)
        x = self.apply_Ainv(y, lat.even)
        t = np.zeros(self.shape, dtype=np.complex128)
        t[lat.odd] = b[lat.odd] - self.apply_H(x, lat.odd)[lat.odd]
        x[lat.odd] = self.apply_Ainv(t, lat.odd)[lat.odd]
        return x

    # --- dense forms (tiny lattices only) ----------------------------------
    def dense(self, apply):
        n = self.lat.V * 12
        M = np.zeros((n, n), dtype=np.complex128)
        e = np.zeros(n, dtype=np.complex128)
        for j in range(n):
            e[j] = 1.0
            M[:, j] = apply(e).reshape(-1)
            e[j] = 0.0
        return M


def gauge_transform_links(lat, U, Om):
    """U^Om_mu(x) = Om(x) U_mu(x) Om(x+mu)^dag (flat [V][4][3][3])."""
    Ut = np.empty_like(U)
    for mu in range(4):
        Ut[:, mu] = Om @ U[:, mu] @ dag(Om[lat.fwd[mu]])
    return Ut
