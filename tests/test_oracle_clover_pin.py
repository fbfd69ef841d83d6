"""Closed-form pins of the oracle's clover term and of its MR relaxation (CPU).

Clover (red-black paragraph: the site-diagonal blocks D_ee, D_oo carry the
clover term; Sheikholeslami-Wohlert reading).  For an abelian field
U_mu(x) = exp(i eps a_mu(x) T), T = diag(1, -1, 0), every plaquette leaf is
exp(i eps Phi T) with Phi the lattice curl of a, so the field strength is
Fhat_mu_nu = (i/4) diag_c(S^{mu nu}_c), S_c = sum over the four leaves of
sin(eps Phi_leaf t_c).  With sigma_mu_nu worked out by hand in the chiral
basis,

    sigma_jk = -eps_jkl diag(s_l, s_l)       (j, k, l spatial)
    sigma_k4 = diag(s_k, -s_k)

(s_l the Pauli matrices), the clover term csw (i/4) sum_{mu != nu}
sigma (x) Fhat reduces to -(csw/8) sum_{mu < nu} sigma_mu_nu (x) diag(S).
For a field in the xy plane alone this is (csw/8) diag(s_3, s_3) (x) diag(S).
The fluxes here come from np.roll on the a-fields, not from the oracle's
neighbour tables or matrix products; the Pauli blocks are typed out, not
taken from the oracle's gamma matrices.  Planted mistakes in the oracle
(a factor of 2, the sign, Q in place of Q^dag, a transposed sigma) must
fail these pins.

MR (the smoother of the adaptive multigrid paragraph, minimal-residual
reading): each step takes the scalar a that minimises ||r - a A r||, so the
new residual is orthogonal to A r and x moves by exactly the least-squares
coefficient times r.
"""
import numpy as np
import pytest

import oracle.dirac as dirac
from oracle.dirac import WilsonClover
from oracle.krylov import mr

S1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
S2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
S3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULI = [S1, S2, S3]
TDIAG = np.array([1.0, -1.0, 0.0])


def _blockdiag(a, b):
    out = np.zeros((4, 4), dtype=np.complex128)
    out[:2, :2] = a
    out[2:, 2:] = b
    return out


def sigma_hand(mu, nu):
    """sigma_mu_nu (mu < nu) in the chiral basis, derived by hand (see module doc)."""
    if nu == 3:
        return _blockdiag(PAULI[mu], -PAULI[mu])
    l = 3 - mu - nu  # the remaining spatial index
    sign = {(0, 1): 1, (1, 2): 1, (0, 2): -1}[(mu, nu)]  # eps_{mu nu l}
    return -sign * _blockdiag(PAULI[l], PAULI[l])


def abelian_links(a, eps):
    """U[t,z,y,x,mu] = exp(i eps a_mu T) from a[t,z,y,x,mu]; canonical flat layout."""
    ph = np.exp(1j * eps * a[..., None] * TDIAG)          # [..., mu, colour]
    U = ph[..., :, None] * np.eye(3)                     # diagonal 3x3
    return U.reshape(-1, 4, 3, 3)


# axis of direction mu in an array indexed [t, z, y, x]
AX = {0: 3, 1: 2, 2: 1, 3: 0}


def shift(f, mu, k):
    """f(x + k mu) on the periodic lattice (np.roll moves content the other way)."""
    return np.roll(f, -k, axis=AX[mu])


def leaf_sin_sum(a, eps, mu, nu):
    """S_c(x) = sum over the four clover leaves at x of sin(eps Phi t_c), shape [t,z,y,x,3]."""
    am, an = a[..., mu], a[..., nu]
    # curl on the plaquette with lower corner y in the (mu, nu) plane
    phi = am + shift(an, mu, 1) - shift(am, nu, 1) - an
    corners = [phi, shift(phi, mu, -1), shift(shift(phi, mu, -1), nu, -1), shift(phi, nu, -1)]
    return sum(np.sin(eps * c[..., None] * TDIAG) for c in corners)


def closed_form_clover(a, eps, csw, planes):
    V = a[..., 0].size
    C = np.zeros((V, 12, 12), dtype=np.complex128)
    for mu, nu in planes:
        S = leaf_sin_sum(a, eps, mu, nu).reshape(V, 3)
        s = sigma_hand(mu, nu)
        C += -(csw / 8.0) * np.einsum("st,nc,cd->nsctd", s, S, np.eye(3)).reshape(V, 12, 12)
    return C


def test_sigma_hand_is_clifford_consistent():
    """sigma_hand reproduces the Clifford relations it was derived from."""
    for mu in range(4):
        for nu in range(mu + 1, 4):
            s = sigma_hand(mu, nu)
            assert np.allclose(s, s.conj().T)
            assert np.allclose(s @ s, np.eye(4))  # each sigma_mu_nu squares to one
    # sigma_xy sigma_zt = -gamma5 in this basis (gamma5 = diag(1,1,-1,-1))
    assert np.allclose(sigma_hand(0, 1) @ sigma_hand(2, 3), -np.diag([1, 1, -1, -1]))


def _single_plane_field(dims, seed):
    Lx, Ly, Lz, Lt = dims
    rng = np.random.default_rng(seed)
    axy = rng.standard_normal((Ly, Lx, 2))
    a = np.zeros((Lt, Lz, Ly, Lx, 4))
    a[..., 0] = axy[None, None, :, :, 0]
    a[..., 1] = axy[None, None, :, :, 1]
    return a


@pytest.mark.parametrize("csw", [1.0, 1.7])
def test_clover_single_plane_closed_form(csw):
    """Only a_x(x, y), a_y(x, y) non-zero: A - (4+m0) = (csw/8) diag(s3, s3) (x) diag(S^{xy})."""
    dims = (4, 6, 2, 4)
    eps, m0 = 0.9, -0.2
    a = _single_plane_field(dims, 5)
    op = WilsonClover(dims, abelian_links(a, eps), m0, csw)
    S = leaf_sin_sum(a, eps, 0, 1).reshape(-1, 3)
    spin_sign = np.array([1.0, -1.0, 1.0, -1.0])  # diag(s3, s3)
    want = (csw / 8.0) * (spin_sign[None, :, None] * S[:, None, :]).reshape(-1, 12)
    got = op.A - (4.0 + m0) * np.eye(12)
    assert np.abs(got - np.einsum("ni,ij->nij", want, np.eye(12))).max() < 1e-14
    assert np.abs(want).max() > 0.1  # the pin is not vacuous


def test_clover_all_planes_closed_form():
    """Arbitrary abelian a_mu(x) in 4D: every plane and sigma_mu_nu at once."""
    dims = (4, 4, 2, 6)
    eps, m0, csw = 0.6, 0.1, 1.3
    rng = np.random.default_rng(17)
    a = rng.standard_normal((dims[3], dims[2], dims[1], dims[0], 4))
    op = WilsonClover(dims, abelian_links(a, eps), m0, csw)
    planes = [(m, n) for m in range(4) for n in range(m + 1, 4)]
    want = closed_form_clover(a, eps, csw, planes)
    got = op.A - (4.0 + m0) * np.eye(12)
    assert np.abs(got - want).max() < 1e-14
    assert np.abs(want).max() > 0.1


def _plant(monkeypatch, kind):
    if kind == "factor2":
        orig = dirac.clover_term
        monkeypatch.setattr(dirac, "clover_term", lambda *a, **k: 2.0 * orig(*a, **k))
    elif kind == "sign":
        orig = dirac.clover_term
        monkeypatch.setattr(dirac, "clover_term", lambda *a, **k: -orig(*a, **k))
    elif kind == "Qdag":
        orig = dirac.plaquette_sum
        monkeypatch.setattr(dirac, "plaquette_sum", lambda *a, **k: dirac.dag(orig(*a, **k)))
    elif kind == "sigmaT":
        orig = dirac.sigma_munu
        monkeypatch.setattr(dirac, "sigma_munu", lambda m, n: orig(m, n).T)
    elif kind == "leaf_missing":
        orig = dirac.plaquette_sum

        def three_leaves(lat, U, mu, nu, sites):
            # drop the first leaf: Q - U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
            x = sites
            l1 = U[x, mu] @ U[lat.fwd[mu][x], nu] @ dirac.dag(U[lat.fwd[nu][x], mu]) @ dirac.dag(U[x, nu])
            return orig(lat, U, mu, nu, sites) - l1
        monkeypatch.setattr(dirac, "plaquette_sum", three_leaves)


@pytest.mark.parametrize("kind", ["factor2", "sign", "Qdag", "sigmaT", "leaf_missing"])
def test_planted_clover_mistakes_fail_the_pins(monkeypatch, kind):
    _plant(monkeypatch, kind)
    dims = (4, 4, 2, 6)
    eps, m0, csw = 0.6, 0.1, 1.3
    rng = np.random.default_rng(17)
    a = rng.standard_normal((dims[3], dims[2], dims[1], dims[0], 4))
    op = WilsonClover(dims, abelian_links(a, eps), m0, csw)
    planes = [(m, n) for m in range(4) for n in range(m + 1, 4)]
    err = np.abs(op.A - (4.0 + m0) * np.eye(12) - closed_form_clover(a, eps, csw, planes)).max()
    assert err > 1e-3, kind


# ---------------------------------------------------------------------------- MR
def _nonhermitian(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return 3.0 * np.eye(n) + 0.4 * M / np.sqrt(n)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mr_steps_are_least_squares_minimisers(seed):
    n = 40
    M = _nonhermitian(n, seed)
    A = lambda v: M @ v
    rng = np.random.default_rng(100 + seed)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    prev_x = x0
    prev_r = b - A(x0)
    for k in range(1, 7):
        x = mr(A, b, x0, k)
        r = b - A(x)
        Ar = A(prev_r)
        # the step is the least-squares coefficient of r_prev against A r_prev ...
        coef = np.linalg.lstsq(Ar[:, None], prev_r, rcond=None)[0][0]
        assert np.abs(x - (prev_x + coef * prev_r)).max() < 1e-12 * max(1.0, np.abs(x).max())
        # ... so the new residual is orthogonal to A r_prev and no longer than r_prev
        assert abs(np.vdot(Ar, r)) < 1e-12 * np.linalg.norm(Ar) * np.linalg.norm(prev_r)
        assert np.linalg.norm(r) <= np.linalg.norm(prev_r) * (1 + 1e-14)
        prev_x, prev_r = x, r


def test_mr_converges_on_a_positive_real_field_of_values():
    """With Re <v, A v> > 0 for all v, MR contracts the residual every step (Saad, Thm. 5.10)."""
    n = 60
    M = _nonhermitian(n, 7)
    A = lambda v: M @ v
    rng = np.random.default_rng(8)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x = mr(A, b, np.zeros(n, dtype=np.complex128), 80)
    assert np.linalg.norm(b - A(x)) < 1e-10 * np.linalg.norm(b)
