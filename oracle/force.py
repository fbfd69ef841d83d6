"""Gradient of a real loss through x = D(U)^-1 eta (oracle; test infrastructure only).

The paper solves D x = eta; differentiating that solve is not part of it.
This module writes the derivative out from the operator definition of Eq.(1)
(hop plus Sheikholeslami-Wohlert clover, with the conventions of dirac.py).

Convention for complex variables (PyTorch's): the gradient of a real loss L
with respect to a complex array z is G = dL/dRe z + i dL/dIm z, so that a
perturbation dz changes the loss by dL = Re sum conj(G) dz.

Given the upstream gradient g = dL/dx of the solution:

    lambda   = D^-dag g                         (adjoint solve)
    grad_eta = lambda
    dL       = -Re <lambda, dD x>                (from dx = -D^-1 dD x)

and grad_U follows term by term from dD:

* hop term, dH x(y) = -1/2 sum_mu [(1-gamma_mu) dU_mu(y) x(y+mu) ph
                                   + (1+gamma_mu) dU_mu(y-mu)^dag x(y-mu) ph']
  gives, for the link U_mu(y) with boundary phase ph,
      grad_U = 1/2 ph sum_s [ lambda(y)_s chi_s^dag + phi_s lambda(y+mu)_s^dag ],
      chi = (1-gamma_mu) x(y+mu),  phi = (1+gamma_mu) x(y)
  (colour outer products summed over spin);

* clover term, dA(y) = csw (i/4) sum_{mu != nu} sigma_mu_nu (x) dF_mu_nu(y),
  F = (Q - Q^dag)/8, Q the sum of the four plaquette leaves: with
      Xi_mu_nu(y)[b, a] = sum_{s,t} sigma_mu_nu[s, t] x(y)_{t b} conj(lambda(y)_{s a})
      W = -csw (i/4) Xi,   Z = (W - W^dag)/8
  the loss changes by dL = Re sum_y sum_{mu != nu} tr(dQ_mu_nu(y) Z_mu_nu(y)),
  and each leaf is a product of four links or adjoints F1 F2 F3 F4; with
  K_k = F_{k+1} ... F_4 Z F_1 ... F_{k-1} the link under F_k = U collects
  K_k^dag, the link under F_k = U^dag collects K_k.

Everything is FP64 and plain NumPy; no blocking or fusion beyond the
definitions above.
"""
import numpy as np

from .dirac import I4, WilsonClover, dag
from .lattice import GAMMA, GAMMA5, sigma_munu


def adjoint_solve_dense(op, g):
    """lambda = D^-dag g by a dense solve (small lattices only)."""
    M = op.dense(op.apply_D)
    lam = np.linalg.solve(dag(M), np.asarray(g, dtype=np.complex128).reshape(-1))
    return lam.reshape(op.shape)


def hop_force(op, x, lam):
    """grad_U of -Re <lam, dH x>, as [V][4][3][3]."""
    lat = op.lat
    x = op.vec(x)
    lam = op.vec(lam)
    G = np.zeros((lat.V, 4, 3, 3), dtype=np.complex128)
    for mu in range(4):
        nb = lat.fwd[mu]
        chi = np.einsum("st,nta->nsa", I4 - GAMMA[mu], x[nb])
        phi = np.einsum("st,nta->nsa", I4 + GAMMA[mu], x)
        m1 = np.einsum("nsa,nsb->nab", lam, np.conj(chi))
        m2 = np.einsum("nsa,nsb->nab", phi, np.conj(lam[nb]))
        c = op.hop_s if mu < 3 else 1.0  # spatial hop coefficient of anisotropic lattices
        G[:, mu] = 0.5 * c * (m1 + m2) * lat.fwd_phase[mu][:, None, None]
    return G


def _leaves(lat, mu, nu):
    """The four leaves of Q_mu_nu(y) as lists of (site array, direction, adjoint).

    Same leaves and order as dirac.plaquette_sum; every site array is
    indexed by y (all sites)."""
    y = np.arange(lat.V)
    ypm, ypn = lat.fwd[mu][y], lat.fwd[nu][y]
    ymm, ymn = lat.bwd[mu][y], lat.bwd[nu][y]
    ymm_pn = lat.fwd[nu][ymm]
    ymm_mn = lat.bwd[nu][ymm]
    ypm_mn = lat.bwd[nu][ypm]
    return [
        [(y, mu, False), (ypm, nu, False), (ypn, mu, True), (y, nu, True)],
        [(y, nu, False), (ymm_pn, mu, True), (ymm, nu, True), (ymm, mu, False)],
        [(ymm, mu, True), (ymm_mn, nu, True), (ymm_mn, mu, False), (ymn, nu, False)],
        [(ymn, nu, True), (ymn, mu, False), (ypm_mn, nu, False), (y, mu, True)],
    ]


def clover_force(op, x, lam):
    """grad_U of -Re <lam, dA x> for A computed from U (csw term only)."""
    lat = op.lat
    U = op.U
    x = op.vec(x)
    lam = op.vec(lam)
    G = np.zeros((lat.V, 4, 3, 3), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            s = sigma_munu(mu, nu)
            xi = np.einsum("st,ntb,nsa->nba", s, x, np.conj(lam))
            w = op.csw if (mu < 3 and nu < 3) else op.csw_t  # plane weight (anisotropic lattices)
            W = -w * 0.25j * xi
            Z = (W - dag(W)) / 8.0
            for leaf in _leaves(lat, mu, nu):
                mats = [dag(U[st, d]) if adj else U[st, d] for st, d, adj in leaf]
                for k in range(4):
                    K = np.broadcast_to(np.eye(3, dtype=np.complex128), (lat.V, 3, 3))
                    for j in range(k + 1, 4):
                        K = K @ mats[j]
                    K = K @ Z
                    for j in range(0, k):
                        K = K @ mats[j]
                    st, d, adj = leaf[k]
                    contrib = K if adj else dag(K)
                    np.add.at(G[:, d], st, contrib)
    return G


def force(op, x, lam, include_clover=True):
    """grad_U = hop part (+ clover part when the clover is computed from U)."""
    G = hop_force(op, x, lam)
    if include_clover and (op.csw != 0.0 or op.csw_t != 0.0):
        G = G + clover_force(op, x, lam)
    return G


def loss_and_grads_dense(dims, U, m0, csw, eta, t_bc=-1):
    """L = ||D^-1 eta||^2 with its gradients (grad_eta, grad_U), all by dense
    solves: x = D^-1 eta, g = 2x, lambda = D^-dag g."""
    op = WilsonClover(dims, U, m0, csw, t_bc)
    M = op.dense(op.apply_D)
    x = np.linalg.solve(M, np.asarray(eta, dtype=np.complex128).reshape(-1)).reshape(op.shape)
    L = float(np.vdot(x, x).real)
    lam = np.linalg.solve(dag(M), (2.0 * x).reshape(-1)).reshape(op.shape)
    return L, lam, force(op, x, lam)


def loss_dense(dims, U, m0, csw, eta, t_bc=-1):
    op = WilsonClover(dims, U, m0, csw, t_bc)
    M = op.dense(op.apply_D)
    x = np.linalg.solve(M, np.asarray(eta, dtype=np.complex128).reshape(-1))
    return float(np.vdot(x, x).real)


def su3_generator_direction(rng):
    """A random traceless Hermitian 3x3 X with unit Frobenius norm."""
    A = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    H = 0.5 * (A + dag(A))
    H -= np.trace(H) / 3.0 * np.eye(3)
    return H / np.linalg.norm(H)


def perturb_link(U, site, mu, X, h):
    """U -> exp(i h X) U on the single link (site, mu); U flat [V][4][3][3]."""
    w, v = np.linalg.eigh(X)
    E = (v * np.exp(1j * h * w)) @ dag(v)
    Up = U.copy()
    Up[site, mu] = E @ U[site, mu]
    return Up


def directional_derivative(G, U, site, mu, X):
    """dL/dh at h = 0 for U -> exp(i h X) U on one link: Re tr(G^dag (i X U))."""
    dU = 1j * X @ U[site, mu]
    return float(np.real(np.sum(np.conj(G[site, mu]) * dU)))


def gamma5_sandwich(op, v):
    """gamma5 v (helper for the D^dag = gamma5 D gamma5 identity)."""
    return np.einsum("st,nta->nsa", GAMMA5, op.vec(v))
