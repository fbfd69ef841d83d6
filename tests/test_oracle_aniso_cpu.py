"""Pins of the oracle's anisotropic Wilson-clover operator (the Results
section's lattices are anisotropic; reading: spatial hops weighted hop_s,
diagonal m0 + 1 + 3 hop_s, clover planes weighted csw_s / csw_t).

* free field: plane waves are eigenvectors with the symbol
  m0 + sum_mu c_mu (1 - cos p_mu) + i sum_mu c_mu gamma_mu sin p_mu,
  c_mu = hop_s (spatial), 1 (time);
* abelian field: the clover term equals -(1/8) sum_{mu<nu} c_munu sigma_mu_nu
  (x) diag(S^{mu nu}), with the hand-derived sigma's and np.roll fluxes of the
  isotropic closed form, each plane weighted csw_s or csw_t;
* gamma5-hermiticity, gauge covariance and the explicit adjoint;
* the force against central differences of the loss.
"""
import importlib.util
import os

import numpy as np
import pytest

import inputs
from oracle import force as F
from oracle.dirac import WilsonClover, dag, gauge_transform_links
from oracle.krylov import bicgstab
from oracle.lattice import GAMMA, GAMMA5

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("clover_pin", os.path.join(HERE, "test_oracle_clover_pin.py"))
pin = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(pin)

HOP_S, CSW_S, CSW_T = 0.35, 0.8, 1.4


def test_free_field_plane_waves_anisotropic():
    dims = (4, 4, 4, 8)
    m0 = -0.05
    V = inputs.volume(dims)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()
    op = WilsonClover(dims, U, m0, CSW_S, hop_s=HOP_S, csw_t=CSW_T)
    rng = np.random.default_rng(2)
    c = np.array([HOP_S, HOP_S, HOP_S, 1.0])
    for _ in range(5):
        n = [rng.integers(0, L) for L in dims]
        p = 2 * np.pi * np.array([n[0] / dims[0], n[1] / dims[1], n[2] / dims[2], (n[3] + 0.5) / dims[3]])
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * op.lat.coords @ p)
        sym = (m0 + np.sum(c * (1 - np.cos(p)))) * np.eye(4) + 1j * sum(c[m] * GAMMA[m] * np.sin(p[m])
                                                                      for m in range(4))
        got = op.apply_D(phase[:, None, None] * u[None])
        want = phase[:, None, None] * (sym @ u)[None]
        assert np.abs(got - want).max() < 1e-13


def test_clover_per_plane_weights_closed_form():
    dims = (4, 4, 2, 6)
    eps, m0 = 0.6, 0.1
    rng = np.random.default_rng(17)
    a = rng.standard_normal((dims[3], dims[2], dims[1], dims[0], 4))
    op = WilsonClover(dims, pin.abelian_links(a, eps), m0, CSW_S, hop_s=HOP_S, csw_t=CSW_T)
    V = a[..., 0].size
    want = np.zeros((V, 12, 12), dtype=np.complex128)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            w = CSW_T if nu == 3 else CSW_S
            want += pin.closed_form_clover(a, eps, w, [(mu, nu)])
    got = op.A - (m0 + 1 + 3 * HOP_S) * np.eye(12)
    assert np.abs(got - want).max() < 1e-14


def test_structure_anisotropic():
    dims = (4, 4, 4, 4)
    U = inputs.gauge_field(dims, 0.5, 1400)
    op = WilsonClover(dims, U, -0.1, CSW_S, hop_s=HOP_S, csw_t=CSW_T)
    rng = np.random.default_rng(3)
    phi = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    psi = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    lhs = np.vdot(phi, op.apply_D(psi))
    rhs = np.vdot(op.gamma5(op.apply_D(op.gamma5(phi))), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    assert abs(np.vdot(op.apply_Ddag(phi), psi) - lhs) < 1e-12 * abs(lhs)
    Om = inputs.random_su3(op.lat.V, 77)
    opt = WilsonClover(dims, gauge_transform_links(op.lat, op.U, Om), -0.1, CSW_S, hop_s=HOP_S, csw_t=CSW_T)
    lhs = opt.apply_D(np.einsum("nab,nsb->nsa", Om, psi))
    rhs = np.einsum("nab,nsb->nsa", Om, op.apply_D(psi))
    assert np.abs(lhs - rhs).max() < 1e-13
    # the hop weight is not a no-op
    iso = WilsonClover(dims, U, -0.1, CSW_S)
    assert np.abs(iso.apply_D(psi) - op.apply_D(psi)).max() > 0.1


def test_force_central_differences_anisotropic():
    dims = (4, 4, 4, 4)
    U = inputs.random_links(dims, 0.3, 1000).reshape(-1, 4, 3, 3)
    rng = np.random.default_rng(8)
    eta = rng.standard_normal((256, 4, 3)) + 1j * rng.standard_normal((256, 4, 3))
    m0 = -0.1

    def solve(op, b):
        return bicgstab(op.apply_D, b, tol=1e-14, maxiter=5000)

    def loss(Uv):
        x = solve(WilsonClover(dims, Uv, m0, CSW_S, hop_s=HOP_S, csw_t=CSW_T), eta)
        return float(np.vdot(x, x).real)

    op = WilsonClover(dims, U, m0, CSW_S, hop_s=HOP_S, csw_t=CSW_T)
    x = solve(op, eta)
    lam = F.gamma5_sandwich(op, solve(op, F.gamma5_sandwich(op, 2.0 * x)))
    G = F.force(op, x, lam)
    h = 1e-4
    for site, mu in [(int(rng.integers(256)), m) for m in range(4)] + [(200, 1), (17, 3)]:
        X = F.su3_generator_direction(rng)
        an = F.directional_derivative(G, U, site, mu, X)
        fd = (loss(F.perturb_link(U, site, mu, X, h)) - loss(F.perturb_link(U, site, mu, X, -h))) / (2 * h)
        assert abs(an - fd) <= 1e-6 * abs(fd) + 1e-10, (site, mu, an, fd)
