"""GPU parity of the adjoint solve and the gauge-link force, and the
differentiable solve checked against the FP64 oracle and finite differences.

* force kernels vs the oracle force for given (psi, lambda) pairs, element by
  element, FP64 tolerance 1e-12 (max-norm relative), with and without the
  clover part, two right-hand sides summed, on three lattices (one with a
  ragged half volume, one with periodic time);
* D^dag solve vs the oracle's explicit adjoint;
* autograd gradients of L = ||D^-1 eta||^2 vs the oracle's dense gradients
  on 4^4;
* the same gradients vs central differences of L on 8^4 (20 random link
  directions, h = 1e-6) and 16^3x32 (5 directions).  The perturbed losses are
  formed from the correction delta = D(U')^-1 (eta - D(U') x), so that
  L(U') - L(U) = 2 Re<x, delta> + ||delta||^2 is resolved to the solver
  tolerance relative to the O(h) change rather than to ||eta||.
"""
import numpy as np
import pytest
import torch

import inputs
from oracle import force as F
from oracle.dirac import WilsonClover, dag

pytestmark = pytest.mark.gpu

w = pytest.importorskip("paper_1011_2775_amd")
from paper_1011_2775_amd import autograd as wad  # noqa: E402

CASES = [
    dict(dims=(4, 4, 4, 4), eps=0.3, seed=1001, m0=-0.2, csw=1.0, t_bc=-1),
    dict(dims=(6, 4, 8, 10), eps=0.5, seed=7, m0=-0.25, csw=1.0, t_bc=-1),
    dict(dims=(4, 6, 4, 6), eps=0.5, seed=8, m0=0.1, csw=1.3, t_bc=1),
]


def canon(v, dims):
    v = np.ascontiguousarray(v)
    return torch.from_numpy(v.reshape((-1,) + tuple(reversed(dims)) + (4, 3))).cuda()


def make_ctx(c, U):
    ctx = w.Context([(c["dims"], c["t_bc"])])
    ctx.set_gauge(torch.from_numpy(U).cuda())
    ctx.set_clover(c["m0"], c["csw"])
    return ctx


@pytest.mark.parametrize("case", range(len(CASES)))
def test_force_matches_oracle(case):
    c = CASES[case]
    print("case", c, flush=True)
    dims = c["dims"]
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, c["eps"], c["seed"])
    op = WilsonClover(dims, U, c["m0"], c["csw"], c["t_bc"])
    rng = np.random.default_rng(11 + case)
    x = rng.standard_normal((2, V, 4, 3)) + 1j * rng.standard_normal((2, V, 4, 3))
    lam = rng.standard_normal((2, V, 4, 3)) + 1j * rng.standard_normal((2, V, 4, 3))
    ctx = make_ctx(c, U)
    for include_clover in (True, False):
        got = ctx.force(canon(x, dims), canon(lam, dims), include_clover).cpu().numpy().reshape(V, 4, 3, 3)
        want = sum(F.force(op, x[r], lam[r], include_clover) for r in range(2))
        err = np.abs(got - want).max() / np.abs(want).max()
        assert err < 1e-12, (include_clover, err)
    ctx.close()


def test_force_needs_clover_from_gauge():
    c = CASES[0]
    U = inputs.gauge_field(c["dims"], c["eps"], c["seed"])
    op = WilsonClover(c["dims"], U, c["m0"], c["csw"])
    ctx = w.Context([(c["dims"], -1)])
    ctx.set_gauge(torch.from_numpy(U).cuda())
    ctx.set_clover(c["m0"], c["csw"], torch.from_numpy(op.A).cuda())
    v = canon(np.ones((256, 4, 3), dtype=np.complex128), c["dims"])
    with pytest.raises(w.WcmgError):
        ctx.force(v, v, include_clover=True)
    ctx.force(v, v, include_clover=False)
    ctx.close()


@pytest.mark.parametrize("solver", ["GCR", "BICGSTAB"])
def test_solve_dag_matches_oracle(solver):
    c = CASES[1]
    dims = c["dims"]
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, c["eps"], c["seed"])
    op = WilsonClover(dims, U, c["m0"], c["csw"], c["t_bc"])
    ctx = make_ctx(c, U)
    b = inputs.gaussian_source(dims, 77).reshape(V, 4, 3)
    x, st = ctx.solve_dag(canon(b, dims), getattr(w, solver), 1e-11)
    xv = x.cpu().numpy().reshape(V, 4, 3)
    res = np.linalg.norm(op.apply_Ddag(xv) - b) / np.linalg.norm(b)
    assert res < 2e-11, (res, st)
    ctx.close()


def test_autograd_matches_dense_oracle():
    c = CASES[0]
    dims = c["dims"]
    U = inputs.gauge_field(dims, c["eps"], c["seed"])
    eta = inputs.gaussian_source(dims, 4000)
    L_or, lam_or, G_or = F.loss_and_grads_dense(dims, U, c["m0"], c["csw"], eta.reshape(256, 4, 3))
    ctx = make_ctx(c, U)
    eta_t = canon(eta, dims).requires_grad_(True)
    U_t = torch.from_numpy(U).cuda().requires_grad_(True)
    x = wad.solve(ctx, eta_t, U_t, solver=w.GCR, tol=1e-13)
    L = (x.abs() ** 2).sum()
    L.backward()
    assert abs(L.item() - L_or) <= 1e-11 * L_or
    ge = eta_t.grad.cpu().numpy().reshape(256, 4, 3)
    gu = U_t.grad.cpu().numpy().reshape(256, 4, 3, 3)
    assert np.linalg.norm(ge - lam_or) / np.linalg.norm(lam_or) < 1e-10
    assert np.linalg.norm(gu - G_or) / np.linalg.norm(G_or) < 1e-10
    ctx.close()


def _fd_check(cfg_name, ndir, h=1e-6):
    cfg = inputs.config(cfg_name)
    dims = cfg["dims"]
    V = int(np.prod(dims))
    m0, csw = cfg["m0"][0], cfg["csw"]
    U = inputs.gauge_field(dims, cfg["eps"], cfg["gauge_seed"], ape_sweeps=cfg["ape"])
    eta = inputs.gaussian_source(dims, cfg["source_seeds"][0])
    params = w.default_params(block=cfg["blocks"], nvec=cfg["nvec"], seed=cfg["setup_seed"])
    ctx = w.Context(dims)

    def load(Uc, vecs=None):
        ctx.set_gauge(torch.from_numpy(np.ascontiguousarray(Uc)).cuda())
        ctx.set_clover(m0, csw)
        ctx.set_mg_params(params)
        if vecs is None:
            ctx.build_null_vectors()
        else:
            ctx.set_null_vectors(vecs)
        ctx.build_coarse()

    load(U)
    vecs = ctx.get_null_vectors()
    eta_t = canon(eta, dims).requires_grad_(True)
    U_t = torch.from_numpy(U).cuda().requires_grad_(True)
    x = wad.solve(ctx, eta_t, U_t, solver=w.MG_GCR, tol=1e-12)
    L = (x.abs() ** 2).sum()
    L.backward()
    G = U_t.grad.cpu().numpy().reshape(V, 4, 3, 3)
    x = x.detach()
    Uf = U.reshape(V, 4, 3, 3)
    worst = 0.0
    for j in range(ndir):
        rng = np.random.default_rng(4000 + j)
        site, mu = int(rng.integers(V)), int(rng.integers(4))
        X = F.su3_generator_direction(rng)
        dL = []
        for sgn in (1.0, -1.0):
            Up = F.perturb_link(Uf, site, mu, X, sgn * h)
            load(Up.reshape(U.shape), vecs)
            r = canon(eta, dims) - ctx.apply_D(x)
            d, _ = ctx.solve(r, w.MG_GCR, 1e-10)
            dL.append(2.0 * torch.vdot(x.flatten(), d.flatten()).real.item() + (d.abs() ** 2).sum().item())
        fd = (dL[0] - dL[1]) / (2 * h)
        an = F.directional_derivative(G, Uf, site, mu, X)
        err = abs(an - fd) / max(abs(fd), 1e-30)
        worst = max(worst, err)
        print("direction", j, site, mu, an, fd, err, flush=True)
        assert err < 1e-6, (j, site, mu, an, fd)
    ctx.close()
    return worst


def test_autograd_finite_differences_8x8x8x8():
    _fd_check("c4_8x8x8x8", 20)


def test_autograd_finite_differences_16x16x16x32():
    _fd_check("c2_16x16x16x32", 20)
