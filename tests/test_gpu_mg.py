"""GPU parity of the multigrid path against the FP64 oracle.

P, R and the coarse operator are compared given the same imported null
vectors (the setup itself is a heuristic and is only checked through its
invariants).  Solves are checked by the oracle's own FP64 residual
||b - D x|| / ||b|| <= 1e-10 and against a dense or oracle solve.
"""
import numpy as np
import pytest
import torch

import inputs
from oracle import multigrid as mg
from oracle.dirac import WilsonClover
from oracle.krylov import norm

pytestmark = pytest.mark.gpu

w = pytest.importorskip("paper_1011_2775_amd")


def canon(v, dims, nrhs=1):
    return torch.from_numpy(np.ascontiguousarray(v).reshape((nrhs,) + tuple(reversed(dims)) + (4, 3))).cuda()


def make(dims, eps, seed, m0, csw, ape=0, t_bc=-1):
    U = inputs.gauge_field(dims, eps, seed, ape_sweeps=ape)
    op = WilsonClover(dims, U, m0, csw, t_bc)
    ctx = w.Context([(dims, t_bc)])
    ctx.set_gauge(torch.from_numpy(U).cuda())
    ctx.set_clover(m0, csw)
    return op, ctx


@pytest.fixture(scope="module")
def c1():
    cfg = inputs.config("c1_4x4x4x4")
    op, ctx = make(cfg["dims"], cfg["eps"], cfg["gauge_seed"], cfg["m0"][0], cfg["csw"])
    vecs = mg.setup_null_vectors(op, cfg["nvec"][0], seed=cfg["setup_seed"])
    params = w.default_params(block=cfg["blocks"], nvec=cfg["nvec"], seed=cfg["setup_seed"],
                              smoother_prec=w.F64)
    ctx.set_mg_params(params)
    ctx.set_null_vectors(canon(vecs, cfg["dims"], len(vecs)))
    ctx.build_coarse()
    T = mg.Transfer(op, cfg["blocks"][0], vecs)
    Y = mg.coarse_operator(op, T)
    yield cfg, op, ctx, T, Y
    ctx.close()


def test_null_vector_roundtrip(c1):
    cfg, op, ctx, T, Y = c1
    got = ctx.get_null_vectors().cpu().numpy().reshape(T.nvec, op.lat.V, 12)
    vecs = mg.setup_null_vectors(op, cfg["nvec"][0], seed=cfg["setup_seed"]).reshape(T.nvec, op.lat.V, 12)
    assert np.array_equal(got, vecs)


def test_coarse_operator_matches_oracle(c1):
    cfg, op, ctx, T, Y = c1
    Yg = ctx.get_coarse()
    err = np.abs(Yg - Y).max() / np.abs(Y).max()
    print("coarse operator err %.3e" % err)
    assert err < 1e-13


@pytest.mark.parametrize("prec", [w.F64, w.F32, w.F16])
def test_restrict_prolong_match_oracle(c1, prec):
    cfg, op, ctx, T, Y = c1
    tol = {w.F64: 1e-13, w.F32: 1e-5, w.F16: 5e-3}[prec]
    rng = np.random.default_rng(20)
    r = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    got = ctx.restrict(canon(r, cfg["dims"]), prec=prec).cpu().numpy()[0]
    want = T.restrict(r)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < tol
    cv = rng.standard_normal((T.Vc, 2 * T.nvec)) + 1j * rng.standard_normal((T.Vc, 2 * T.nvec))
    got = ctx.prolong(torch.from_numpy(cv[None]).cuda(), prec=prec).cpu().numpy().reshape(op.shape)
    want = T.prolong(cv)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < tol


@pytest.mark.parametrize("prec", [w.F64, w.F32])
def test_coarse_stencil_matches_oracle(c1, prec):
    cfg, op, ctx, T, Y = c1
    cop = mg.CoarseOperator(T.cdims, Y)
    tol = {w.F64: 1e-13, w.F32: 1e-5}[prec]
    rng = np.random.default_rng(21)
    v = rng.standard_normal(cop.shape) + 1j * rng.standard_normal(cop.shape)
    vt = torch.from_numpy(v[None]).cuda()
    ve = v.copy()
    ve[cop.lat.odd] = 0
    for which, want in ((w.OP_FULL, cop.apply_D(v)), (w.OP_DP, cop.apply_Dp(v)), (w.OP_SCHUR, cop.apply_Dr(ve))):
        got = ctx.apply_coarse(vt, op=which, prec=prec).cpu().numpy()[0]
        err = np.linalg.norm(got - want) / np.linalg.norm(want)
        print("coarse op", which, "prec", prec, "err %.3e" % err)
        assert err < tol


def test_odd_coarse_extent_and_ragged_blocks():
    """8x8x4x12 with 2x2x2x4 blocks: coarse 4x4x2x3 has an odd extent (no
    red-black form on the coarse level) and 96 coarse sites."""
    dims = (8, 8, 4, 12)
    op, ctx = make(dims, 0.5, 31, -0.2, 1.0)
    rng = np.random.default_rng(32)
    vecs = rng.standard_normal((4,) + op.shape) + 1j * rng.standard_normal((4,) + op.shape)
    ctx.set_mg_params(w.default_params(block=[(2, 2, 2, 4)], nvec=[4]))
    ctx.set_null_vectors(canon(vecs, dims, 4))
    ctx.build_coarse()
    T = mg.Transfer(op, (2, 2, 2, 4), vecs)
    Y = mg.coarse_operator(op, T)
    assert np.abs(ctx.get_coarse() - Y).max() < 1e-13 * np.abs(Y).max()
    cop = mg.CoarseOperator(T.cdims, Y)
    v = rng.standard_normal(cop.shape) + 1j * rng.standard_normal(cop.shape)
    got = ctx.apply_coarse(torch.from_numpy(v[None]).cuda(), op=w.OP_FULL).cpu().numpy()[0]
    assert np.linalg.norm(got - cop.apply_D(v)) < 1e-13 * np.linalg.norm(got)
    with pytest.raises(w.WcmgError):
        ctx.apply_coarse(torch.from_numpy(v[None]).cuda(), op=w.OP_SCHUR)
    b = inputs.z2_source(dims, 33)
    x, st = ctx.solve(canon(b, dims), w.MG_GCR, 1e-10)
    xr = x.cpu().numpy().reshape(op.shape)
    assert norm(b.reshape(op.shape) - op.apply_D(xr)) / norm(b) <= 1e-10
    ctx.close()


@pytest.mark.parametrize("solver", [w.BICGSTAB, w.GCR, w.MG_GCR])
def test_solvers_c1(c1, solver):
    cfg, op, ctx, T, Y = c1
    b = inputs.z2_source(cfg["dims"], cfg["source_seeds"][0]).reshape(op.shape)
    x, st = ctx.solve(canon(b, cfg["dims"]), solver, cfg["tol"])
    xr = x.cpu().numpy().reshape(op.shape)
    res = norm(b - op.apply_D(xr)) / norm(b)
    print("solver", solver, st[0], "oracle residual %.3e" % res)
    assert st[0]["status"] == "OK"
    assert res <= 1e-10
    assert abs(res - st[0]["true_rel_res"]) < 1e-12
    xd = np.linalg.solve(op.dense(op.apply_D), b.reshape(-1)).reshape(op.shape)
    assert norm(xr - xd) / norm(xd) < 1e-8
    # deterministic
    x2, _ = ctx.solve(canon(b, cfg["dims"]), solver, cfg["tol"])
    assert torch.equal(x, x2)


def test_mg_iterations_match_oracle_cycle(c1):
    """Same vectors, FP64 everywhere: the GPU cycle takes the oracle's outer iteration count (+-1)."""
    cfg, op, ctx, T, Y = c1
    b = inputs.z2_source(cfg["dims"], cfg["source_seeds"][0]).reshape(op.shape)
    x, st = ctx.solve(canon(b, cfg["dims"]), w.MG_GCR, cfg["tol"])
    vecs = mg.setup_null_vectors(op, cfg["nvec"][0], seed=cfg["setup_seed"])
    H = mg.Hierarchy(op, mg.MGParams(blocks=cfg["blocks"], nvec=cfg["nvec"]), vecs=[vecs])
    from oracle.krylov import SolveInfo
    info = SolveInfo()
    H.solve(b, cfg["tol"], info)
    print("gpu outer iters", st[0]["iters"], "oracle", info.iters)
    assert abs(st[0]["iters"] - info.iters) <= 1


def test_manufactured_solution_and_warm_start(c1):
    cfg, op, ctx, T, Y = c1
    rng = np.random.default_rng(40)
    x0 = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    b = op.apply_D(x0)
    x, st = ctx.solve(canon(b, cfg["dims"]), w.MG_GCR, 1e-12)
    assert norm(x.cpu().numpy().reshape(op.shape) - x0) / norm(x0) < 1e-9
    # a converged guess returns immediately
    x2, st2 = ctx.solve(canon(b, cfg["dims"]), w.MG_GCR, 1e-10, x0=x)
    assert st2[0]["iters"] == 0


@pytest.mark.parametrize("prec,orth_tol", [("F64", 1e-12), ("F32", 5e-6), ("F16", 5e-6)])
def test_gpu_setup_and_solve_c1(prec, orth_tol):
    """Setup in FP64, FP32, or FP32 with half-precision fields: the vectors are
    orthonormal to the setup's precision, low modes of D_p, and the hierarchy
    built on them solves to 1e-10."""
    cfg = inputs.config("c1_4x4x4x4")
    op, ctx = make(cfg["dims"], cfg["eps"], cfg["gauge_seed"], cfg["m0"][0], cfg["csw"])
    ctx.set_mg_params(w.default_params(block=cfg["blocks"], nvec=cfg["nvec"], seed=cfg["setup_seed"],
                                       setup_prec=getattr(w, prec)))
    ctx.build_null_vectors()
    v = ctx.get_null_vectors().cpu().numpy().reshape(cfg["nvec"][0], -1)
    G = v.conj() @ v.T
    assert np.abs(G - np.eye(len(v))).max() < orth_tol
    rq = [norm(op.apply_Dp(x.reshape(op.shape))) ** 2 for x in v]
    rng = np.random.default_rng(41)
    rr = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    assert max(rq) < 0.2 * norm(op.apply_Dp(rr)) ** 2 / norm(rr) ** 2
    # the oracle setup from the same Philox seed lands on the same subspace
    vo = mg.setup_null_vectors(op, cfg["nvec"][0], seed=cfg["setup_seed"]).reshape(len(v), -1)
    ov = np.linalg.svd(vo.conj() @ v.T, compute_uv=False)
    print("setup subspace overlap (singular values)", ov.min(), ov.max())
    ctx.build_coarse()
    b = inputs.z2_source(cfg["dims"], cfg["source_seeds"][0])
    x, st = ctx.solve(canon(b, cfg["dims"]), w.MG_GCR, 1e-10)
    assert norm(b.reshape(op.shape) - op.apply_D(x.cpu().numpy().reshape(op.shape))) / norm(b) <= 1e-10
    ctx.close()


@pytest.mark.parametrize("solver", [w.BICGSTAB, w.GCR])
def test_krylov_heavy_mass_16x16x16x32(solver):
    """Well-conditioned system (m0 = 0.5): the multi-block reductions of the
    Krylov solvers on 786k-element vectors, checked by the oracle residual."""
    dims = (16, 16, 16, 32)
    op, ctx = make(dims, 0.5, 1002, 0.5, 1.0)
    b = inputs.z2_source(dims, 2201)
    x, st = ctx.solve(canon(b, dims), solver, 1e-10)
    res = norm(b.reshape(op.shape) - op.apply_D(x.cpu().numpy().reshape(op.shape))) / norm(b)
    print("solver", solver, st[0], "oracle residual %.3e" % res)
    assert st[0]["iters"] < 200
    assert res <= 1e-10
    ctx.close()


def test_mg_solve_16x16x16x32_full_size():
    cfg = inputs.config("c2_16x16x16x32")
    dims = cfg["dims"]
    m0 = -0.25
    op, ctx = make(dims, cfg["eps"], cfg["gauge_seed"], m0, cfg["csw"], ape=cfg["ape"])
    ctx.set_mg_params(w.default_params(block=cfg["blocks"], nvec=cfg["nvec"], seed=cfg["setup_seed"]))
    ctx.build_null_vectors()
    ctx.build_coarse()
    b = inputs.z2_source(dims, cfg["source_seeds"][0])
    x, st = ctx.solve(canon(b, dims), w.MG_GCR, 1e-10)
    xr = x.cpu().numpy().reshape(op.shape)
    res = norm(b.reshape(op.shape) - op.apply_D(xr)) / norm(b)
    print("C2 MG (FP32 cycle)", st[0], "oracle residual %.3e" % res)
    assert res <= 1e-10
    # an independent solve with an FP64 cycle lands on the same unique solution
    ctx.set_mg_params(w.default_params(block=cfg["blocks"], nvec=cfg["nvec"], seed=cfg["setup_seed"],
                                       smoother_prec=w.F64, setup_relax=20))
    ctx.build_null_vectors()
    ctx.build_coarse()
    x2, st2 = ctx.solve(canon(b, dims), w.MG_GCR, 1e-11)
    print("C2 MG (FP64 cycle)", st2[0])
    x2r = x2.cpu().numpy().reshape(op.shape)
    assert norm(xr - x2r) / norm(x2r) < 1e-7
    ctx.close()


def test_batched_coarse_stencil_on_matrix_cores():
    """Batches of FP32 coarse red-black applies run on the matrix cores with
    FP16 operands: they must agree with the FP64 single applies to FP16
    accuracy, for a full group of 16 and a partial second group."""
    cfg = inputs.config("c2_16x16x16x32")
    dims = cfg["dims"]
    U = inputs.gauge_field(dims, cfg["eps"], cfg["gauge_seed"], ape_sweeps=cfg["ape"])
    ctx = w.Context(dims)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    ctx.set_clover(-0.25, cfg["csw"])
    ctx.set_mg_params(w.default_params(block=cfg["blocks"], nvec=cfg["nvec"], seed=cfg["setup_seed"]))
    ctx.build_null_vectors()
    ctx.build_coarse()
    Vc = int(np.prod(ctx.coarse_dims()))
    n = 2 * cfg["nvec"][0]
    rng = np.random.default_rng(31)
    nrhs = 19
    v = rng.standard_normal((nrhs, Vc, n)) + 1j * rng.standard_normal((nrhs, Vc, n))
    # scale the right-hand sides differently: the per-block FP16 scaling must follow each
    v *= np.logspace(-6, 3, nrhs)[:, None, None]
    vt = torch.from_numpy(v).cuda()
    got = ctx.apply_coarse(vt, level=1, op=w.OP_SCHUR, prec=w.F32).cpu().numpy()
    for r in range(nrhs):
        want = ctx.apply_coarse(vt[r:r + 1].contiguous(), level=1, op=w.OP_SCHUR, prec=w.F64).cpu().numpy()[0]
        err = np.linalg.norm(got[r] - want) / np.linalg.norm(want)
        assert err < 5e-3, (r, err)
    ctx.close()


def test_fp16_field_smoother_16x16x16x32():
    """Half-precision links and clover in the smoother (FP32 vectors and
    arithmetic): the FP64 outer GCR still reaches 1e-10, within a few outer
    iterations of the FP32 smoother."""
    cfg = inputs.config("c2_16x16x16x32")
    dims = cfg["dims"]
    U = inputs.gauge_field(dims, cfg["eps"], cfg["gauge_seed"], ape_sweeps=cfg["ape"])
    ctx = w.Context(dims)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    ctx.set_clover(-0.25, cfg["csw"])
    base = dict(block=cfg["blocks"], nvec=cfg["nvec"], seed=cfg["setup_seed"])
    ctx.set_mg_params(w.default_params(**base))
    ctx.build_null_vectors()
    ctx.build_coarse()
    vecs = ctx.get_null_vectors()
    b = torch.from_numpy(inputs.z2_source(dims, cfg["source_seeds"][0])[None]).cuda()
    its = {}
    for sp in (w.F32, w.F16):
        ctx.set_mg_params(w.default_params(smoother_prec=sp, **base))
        ctx.set_null_vectors(vecs)
        ctx.build_coarse()
        x, st = ctx.solve(b, w.MG_GCR, 1e-10)
        assert st[0]["true_rel_res"] <= 1.0000001e-10
        its[sp] = st[0]["iters"]
    print("outer iterations F32 / F16 fields:", its, flush=True)
    assert its[w.F16] <= its[w.F32] + 3
    ctx.close()


def test_fp16_transfer_vectors_16x16x16x32():
    """Restriction and prolongation of the FP32 cycle with FP16 copies of the
    null vectors (transfer_fp16 = 1; the coarse operator is still built from
    the FP64 vectors): single and batched solves reach 1e-10 by the oracle's
    FP64 residual, within two outer iterations of FP32 copies."""
    cfg = inputs.config("c2_16x16x16x32")
    dims = cfg["dims"]
    op, ctx = make(dims, cfg["eps"], cfg["gauge_seed"], -0.25, cfg["csw"], ape=cfg["ape"])
    base = dict(block=cfg["blocks"], nvec=cfg["nvec"], seed=cfg["setup_seed"])
    ctx.set_mg_params(w.default_params(**base))
    ctx.build_null_vectors()
    ctx.build_coarse()
    vecs = ctx.get_null_vectors()
    s0 = cfg["source_seeds"][0]
    b = np.stack([inputs.z2_source(dims, s) for s in (s0, s0 + 1)])
    its = {}
    for tf in (0, 1):
        ctx.set_mg_params(w.default_params(transfer_fp16=tf, **base))
        ctx.set_null_vectors(vecs)
        ctx.build_coarse()
        x, st = ctx.solve(canon(b[0], dims), w.MG_GCR, 1e-10)
        res = norm(b[0].reshape(op.shape) - op.apply_D(x.cpu().numpy().reshape(op.shape))) / norm(b[0])
        assert st[0]["status"] == "OK" and res <= 1e-10, (tf, res)
        its[tf] = st[0]["iters"]
        xb, stb = ctx.solve(canon(b, dims, 2), w.MG_GCR, 1e-10)
        for r in range(2):
            rr = norm(b[r].reshape(op.shape) - op.apply_D(xb[r].cpu().numpy().reshape(op.shape))) / norm(b[r])
            assert stb[r]["status"] == "OK" and rr <= 1e-10, (tf, r, rr)
    print("outer iterations FP32 / FP16 transfer vectors:", its, flush=True)
    assert its[1] <= its[0] + 2
    ctx.close()
