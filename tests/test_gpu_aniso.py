"""The anisotropic Wilson-clover operator (the Results section measures on
anisotropic lattices) on the GPU against the FP64 oracle: spatial hops
weighted hop_s, diagonal m0 + 1 + 3 hop_s, clover planes weighted csw_s
(spatial planes) and csw_t (planes with time).  Checked: every operator form
and its adjoint at three precisions (tolerances as for the isotropic
operator), the gauge-link force element by element (FP64, 1e-12), and the
MG-GCR solve to a true residual of 1e-10 measured by the oracle."""
import numpy as np
import pytest
import torch

import inputs
from oracle import force as F
from oracle.dirac import WilsonClover
from oracle.krylov import norm

pytestmark = pytest.mark.gpu

w = pytest.importorskip("paper_1011_2775_amd")

HOP_S, CSW_S, CSW_T = 0.35, 0.8, 1.4
CASES = [
    dict(dims=(4, 4, 4, 4), eps=0.3, seed=1001, m0=-0.05, t_bc=-1),
    dict(dims=(6, 4, 8, 10), eps=0.5, seed=7, m0=-0.1, t_bc=-1),
    dict(dims=(4, 6, 4, 6), eps=0.5, seed=8, m0=0.1, t_bc=1),
]
TOL = {w.F64: 1e-13, w.F32: 1e-5, w.F16: 5e-3}


def canon(v, dims):
    v = np.ascontiguousarray(v)
    return torch.from_numpy(v.reshape((-1,) + tuple(reversed(dims)) + (4, 3))).cuda()


@pytest.fixture(scope="module", params=range(len(CASES)))
def setup(request):
    c = CASES[request.param]
    U = inputs.gauge_field(c["dims"], c["eps"], c["seed"])
    op = WilsonClover(c["dims"], U, c["m0"], CSW_S, c["t_bc"], hop_s=HOP_S, csw_t=CSW_T)
    ctx = w.Context([(c["dims"], c["t_bc"])])
    ctx.set_gauge(torch.from_numpy(U).cuda())
    ctx.set_clover_aniso(c["m0"], HOP_S, CSW_S, CSW_T)
    print("case", c, flush=True)
    yield c, U, op, ctx
    ctx.close()


def oracle_apply(op, v, which, dag):
    lat = op.lat
    if which == w.OP_FULL:
        return op.apply_Ddag(v) if dag else op.apply_D(v)
    if which == w.OP_DP:
        return op.apply_Ainv(op.apply_Ddag(v)) if dag else op.apply_Dp(v)
    if which == w.OP_SCHUR_X:
        return op.apply_A(op.apply_Dr_dag(v), lat.even) if dag else op.apply_Dr(op.apply_A(v, lat.even))
    ve = v.copy()
    ve[lat.odd] = 0
    return op.apply_Dr_dag(ve) if dag else op.apply_Dr(ve)


@pytest.mark.parametrize("prec", [w.F64, w.F32, w.F16])
@pytest.mark.parametrize("which", [w.OP_FULL, w.OP_SCHUR, w.OP_DP, w.OP_SCHUR_X])
@pytest.mark.parametrize("dag", [False, True])
def test_apply_matches_oracle(setup, prec, which, dag):
    c, _, op, ctx = setup
    rng = np.random.default_rng(11)
    v = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    fn = ctx.apply_Ddag if dag else ctx.apply_D
    got = fn(canon(v, c["dims"]), which, prec).cpu().numpy().reshape(op.shape)
    want = oracle_apply(op, v, which, dag)
    if prec == w.F64:
        err = np.abs(got - want).max() / np.abs(want).max()
    else:
        err = np.linalg.norm(got - want) / np.linalg.norm(want)
    print("prec", prec, "op", which, "dag", dag, "err %.3e" % err)
    assert err < TOL[prec]


def test_force_matches_oracle(setup):
    c, _, op, ctx = setup
    V = op.lat.V
    rng = np.random.default_rng(21)
    x = rng.standard_normal((2, V, 4, 3)) + 1j * rng.standard_normal((2, V, 4, 3))
    lam = rng.standard_normal((2, V, 4, 3)) + 1j * rng.standard_normal((2, V, 4, 3))
    for include_clover in (True, False):
        got = ctx.force(canon(x, c["dims"]), canon(lam, c["dims"]), include_clover)
        got = got.cpu().numpy().reshape(V, 4, 3, 3)
        want = sum(F.force(op, x[r], lam[r], include_clover) for r in range(2))
        err = np.abs(got - want).max() / np.abs(want).max()
        assert err < 1e-12, (include_clover, err)


def test_isotropic_weights_reproduce_set_clover():
    """hop_s = 1, csw_s = csw_t reproduce the isotropic operator bit for bit."""
    dims = (4, 4, 4, 8)
    U = torch.from_numpy(inputs.gauge_field(dims, 0.4, 55)).cuda()
    a, b = w.Context(dims), w.Context(dims)
    try:
        a.set_gauge(U)
        b.set_gauge(U)
        a.set_clover(-0.1, 1.2)
        b.set_clover_aniso(-0.1, 1.0, 1.2, 1.2)
        v = torch.from_numpy(inputs.gaussian_source(dims, 3)[None]).cuda()
        for which in (w.OP_FULL, w.OP_SCHUR_X):
            assert torch.equal(a.apply_D(v, which), b.apply_D(v, which))
    finally:
        a.close()
        b.close()


def test_mg_solve_anisotropic():
    dims, m0 = (8, 8, 8, 16), -0.12
    U = inputs.gauge_field(dims, 0.5, 1310, ape_sweeps=2)
    op = WilsonClover(dims, U, m0, CSW_S, hop_s=HOP_S, csw_t=CSW_T)
    ctx = w.Context(dims)
    try:
        ctx.set_gauge(torch.from_numpy(U).cuda())
        ctx.set_clover_aniso(m0, HOP_S, CSW_S, CSW_T)
        ctx.set_mg_params(w.default_params(block=[(4, 4, 4, 4)], nvec=[12], seed=3400))
        ctx.build_null_vectors()
        ctx.build_coarse()
        b = inputs.z2_source(dims, 2311)
        x, st = ctx.solve(torch.from_numpy(b[None]).cuda(), w.MG_GCR, 1e-10)
        _, sp = ctx.solve(torch.from_numpy(b[None]).cuda(), w.GCR, 1e-10)
        print("MG-GCR / GCR outer iterations:", st[0]["iters"], sp[0]["iters"], flush=True)
        xr = x.cpu().numpy().reshape(op.shape)
        assert norm(b.reshape(op.shape) - op.apply_D(xr)) / norm(b) <= 1e-10
        assert st[0]["iters"] < sp[0]["iters"]
    finally:
        ctx.close()
