"""Pins of the oracle gradient (adjoint solve + gauge force) of L = ||D^-1 eta||^2.

The force is pinned by central finite differences of the loss computed with
the forward operator only (no shared code with the force), on links in every
direction including the antiperiodic time boundary, with and without the
clover term, and by its covariance under gauge transformations.
"""
import numpy as np
import pytest

import inputs
from oracle import force as F
from oracle.dirac import WilsonClover, dag, gauge_transform_links
from oracle.krylov import bicgstab

DIMS = (4, 4, 4, 4)


def _setup(csw, t_bc, seed=7):
    U = inputs.random_links(DIMS, 0.3, 1000).reshape(-1, 4, 3, 3)
    rng = np.random.default_rng(seed)
    eta = rng.standard_normal((256, 4, 3)) + 1j * rng.standard_normal((256, 4, 3))
    return U, eta, rng


def _solve(op, b):
    return bicgstab(op.apply_D, b, tol=1e-14, maxiter=5000)


def _grads(U, eta, m0, csw, t_bc):
    op = WilsonClover(DIMS, U, m0, csw, t_bc)
    x = _solve(op, eta)
    g = 2.0 * x
    lam = F.gamma5_sandwich(op, _solve(op, F.gamma5_sandwich(op, g)))
    return op, x, lam


def _loss(U, eta, m0, csw, t_bc):
    op = WilsonClover(DIMS, U, m0, csw, t_bc)
    x = _solve(op, eta)
    return float(np.vdot(x, x).real)


def test_adjoint_solve_solves_explicit_adjoint():
    """gamma5 D^-1 gamma5 g solves the explicitly transposed operator."""
    U, eta, _ = _setup(1.0, -1)
    op, x, lam = _grads(U, eta, -0.2, 1.0, -1)
    g = 2.0 * x
    assert np.linalg.norm(op.apply_Ddag(lam) - g) / np.linalg.norm(g) < 1e-12


@pytest.mark.parametrize("csw,t_bc", [(1.0, -1), (0.0, 1)])
def test_force_matches_central_differences(csw, t_bc):
    U, eta, rng = _setup(csw, t_bc)
    m0 = -0.2
    op, x, lam = _grads(U, eta, m0, csw, t_bc)
    G = F.force(op, x, lam)
    h = 1e-4
    t_last = [s for s in range(256) if s // 64 == 3]  # sites on the last time slice
    cases = [(int(rng.integers(256)), mu) for mu in range(4)] + [(t_last[5], 3), (t_last[9], 0)]
    for site, mu in cases:
        X = F.su3_generator_direction(rng)
        an = F.directional_derivative(G, U, site, mu, X)
        fd = (_loss(F.perturb_link(U, site, mu, X, h), eta, m0, csw, t_bc)
              - _loss(F.perturb_link(U, site, mu, X, -h), eta, m0, csw, t_bc)) / (2 * h)
        assert abs(an - fd) <= 1e-6 * abs(fd) + 1e-10, (site, mu, an, fd)


def test_clover_part_is_not_negligible():
    """The clover force carries a sizeable share, so dropping or mis-signing
    it fails the finite-difference pin above."""
    U, eta, _ = _setup(1.0, -1)
    op, x, lam = _grads(U, eta, -0.2, 1.0, -1)
    Gc = F.clover_force(op, x, lam)
    Gh = F.hop_force(op, x, lam)
    assert np.linalg.norm(Gc) > 0.05 * np.linalg.norm(Gh)


def test_source_gradient_matches_differences():
    """L is quadratic in eta, so the central difference is exact up to rounding."""
    U, eta, rng = _setup(1.0, -1)
    m0 = -0.2
    _, _, lam = _grads(U, eta, m0, 1.0, -1)
    d = rng.standard_normal(eta.shape) + 1j * rng.standard_normal(eta.shape)
    h = 1e-3
    fd = (_loss(U, eta + h * d, m0, 1.0, -1) - _loss(U, eta - h * d, m0, 1.0, -1)) / (2 * h)
    an = float(np.real(np.vdot(lam, d)))
    assert abs(an - fd) <= 1e-8 * abs(fd)


def test_force_gauge_covariance():
    """U -> Om U Om(+mu)^dag, x -> Om x, lambda -> Om lambda maps the force as
    G_mu(y) -> Om(y) G_mu(y) Om(y+mu)^dag."""
    U, eta, rng = _setup(1.0, -1)
    op, x, lam = _grads(U, eta, -0.2, 1.0, -1)
    G = F.force(op, x, lam)
    Om = inputs.random_su3(256, 4242)
    Ut = gauge_transform_links(op.lat, U, Om)
    opt = WilsonClover(DIMS, Ut, -0.2, 1.0, -1)
    xt = np.einsum("nab,nsb->nsa", Om, x)
    lt = np.einsum("nab,nsb->nsa", Om, lam)
    Gt = F.force(opt, xt, lt)
    for mu in range(4):
        ref = Om @ G[:, mu] @ dag(Om[op.lat.fwd[mu]])
        assert np.linalg.norm(Gt[:, mu] - ref) <= 1e-12 * np.linalg.norm(ref)
