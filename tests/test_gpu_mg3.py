"""Three-level multigrid on the GPU against the FP64 oracle.

With the raw null vectors of both levels imported on both sides, the
level-1 -> level-2 transfer, the level-2 operator R2 Dhat_p P2 and its
applications are compared element by element (FP64 1e-12, FP32 1e-5); the
three-level solve (coarsest GCR, and coarsest dense FP64 inverse) reaches a
true relative residual of 1e-10 checked with the oracle's D, in an outer
iteration count within 2 of the oracle's hierarchy.  The GPU setup on both
levels is checked through its invariants (the vectors are a heuristic:
parity unpinned) and through convergence on 16^3x32.
"""
import numpy as np
import pytest
import torch

import inputs
from oracle.dirac import WilsonClover
from oracle.multigrid import Hierarchy, MGParams

pytestmark = pytest.mark.gpu

w = pytest.importorskip("paper_1011_2775_amd")

DIMS = (8, 8, 8, 8)
BLOCKS = [(2, 2, 2, 2), (2, 2, 2, 2)]
NVEC = [8, 8]
M0, CSW = -0.2, 1.0


def canon(v, shape):
    return torch.from_numpy(np.ascontiguousarray(v).reshape(shape)).cuda()


def rel(got, want):
    return np.abs(got - want).max() / np.abs(want).max()


@pytest.fixture(scope="module")
def hier():
    U = inputs.gauge_field(DIMS, 0.3, 1004)
    op = WilsonClover(DIMS, U, M0, CSW)
    rng = np.random.default_rng(3)
    V = op.lat.V
    v0 = rng.standard_normal((NVEC[0], V, 4, 3)) + 1j * rng.standard_normal((NVEC[0], V, 4, 3))
    V1 = V // 16
    v1 = rng.standard_normal((NVEC[1], V1, 2 * NVEC[0])) + 1j * rng.standard_normal((NVEC[1], V1, 2 * NVEC[0]))
    H = {c: Hierarchy(op, MGParams(BLOCKS, NVEC, coarsest=c), vecs=[v0, v1]) for c in ("gcr", "lu")}
    ctx = w.Context(DIMS)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    ctx.set_clover(M0, CSW)

    def load(coarsest):
        ctx.set_mg_params(w.default_params(nlevels=2, block=BLOCKS, nvec=NVEC, coarsest=coarsest))
        ctx.set_null_vectors(canon(v0, (NVEC[0],) + tuple(reversed(DIMS)) + (4, 3)), level=0)
        ctx.build_coarse(0)
        ctx.set_null_vectors(canon(v1, v1.shape), level=1)
        ctx.build_coarse(1)

    load(0)
    print("hierarchy loaded", flush=True)
    yield op, H, ctx, load
    ctx.close()


def test_level2_operator_matches_oracle(hier):
    op, H, ctx, load = hier
    Y = ctx.get_coarse(level=1)
    Yo = H["gcr"].ops[2].Y
    assert Y.shape == Yo.shape
    assert rel(Y, Yo) < 1e-12


@pytest.mark.parametrize("prec,tol", [("F64", 1e-13), ("F32", 1e-5)])
def test_level2_transfer_matches_oracle(hier, prec, tol):
    op, H, ctx, load = hier
    T = H["gcr"].transfers[1]
    rng = np.random.default_rng(5)
    n1 = 2 * NVEC[0]
    r = rng.standard_normal((2, T.op.lat.V, n1)) + 1j * rng.standard_normal((2, T.op.lat.V, n1))
    c = ctx.restrict(canon(r, r.shape), level=1, prec=getattr(w, prec)).cpu().numpy()
    want = np.stack([T.restrict(r[k]) for k in range(2)])
    assert np.linalg.norm(c - want) / np.linalg.norm(want) < tol
    cc = rng.standard_normal(want.shape) + 1j * rng.standard_normal(want.shape)
    e = ctx.prolong(canon(cc, cc.shape), level=1, prec=getattr(w, prec)).cpu().numpy()
    want_e = np.stack([T.prolong(cc[k]) for k in range(2)])
    assert np.linalg.norm(e - want_e) / np.linalg.norm(want_e) < tol


@pytest.mark.parametrize("which", ["OP_FULL", "OP_DP", "OP_SCHUR"])
def test_level2_apply_matches_oracle(hier, which):
    op, H, ctx, load = hier
    C = H["gcr"].ops[2]
    rng = np.random.default_rng(9)
    v = rng.standard_normal(C.shape) + 1j * rng.standard_normal(C.shape)
    if which == "OP_SCHUR":
        v[C.lat.odd] = 0
    got = ctx.apply_coarse(canon(v, (1,) + C.shape), level=2, op=getattr(w, which)).cpu().numpy()[0]
    want = {"OP_FULL": C.apply_D, "OP_DP": C.apply_Dp, "OP_SCHUR": C.apply_Dr}[which](v)
    assert rel(got, want) < 1e-12


@pytest.mark.parametrize("coarsest", ["gcr", "lu", "deflated"])
def test_three_level_solve_matches_oracle(hier, coarsest):
    """The deflated FP64 coarsest GCR (no oracle counterpart: it solves the same
    coarsest system to the same tolerance) is compared with the oracle's GCR."""
    op, H, ctx, load = hier
    load({"gcr": 0, "lu": 1, "deflated": 2}[coarsest])
    if coarsest == "deflated":
        coarsest = "gcr"
    b = inputs.z2_source(DIMS, 2004)
    x, st = ctx.solve(canon(b, (1,) + tuple(reversed(DIMS)) + (4, 3)), w.MG_GCR, 1e-10)
    xv = x.cpu().numpy().reshape(op.shape)
    bv = b.reshape(op.shape)
    res = np.linalg.norm(bv - op.apply_D(xv)) / np.linalg.norm(bv)
    assert res <= 1.0000001e-10, res
    from oracle.krylov import SolveInfo
    info = SolveInfo()
    H[coarsest].solve(bv, tol=1e-10, info=info)
    print(coarsest, "gpu outer", st[0]["iters"], "inner", st[0]["inner_iters"], "oracle outer", info.iters,
          flush=True)
    assert abs(st[0]["iters"] - info.iters) <= 2
    load(0)


def test_three_level_gpu_setup_invariants(hier):
    op, H, ctx, load = hier
    ctx.set_mg_params(w.default_params(nlevels=2, block=BLOCKS, nvec=NVEC, seed=3004))
    ctx.build_null_vectors(0)
    ctx.build_coarse(0)
    ctx.build_null_vectors(1)
    ctx.build_coarse(1)
    v = ctx.get_null_vectors(level=1).cpu().numpy().reshape(NVEC[1], -1)
    G = v.conj() @ v.T
    # the default setup runs in FP32: orthonormal to FP32 accuracy
    assert np.abs(G - np.eye(NVEC[1])).max() < 5e-6
    b = inputs.z2_source(DIMS, 2005)
    x, st = ctx.solve(canon(b, (1,) + tuple(reversed(DIMS)) + (4, 3)), w.MG_GCR, 1e-10)
    xv = x.cpu().numpy().reshape(op.shape)
    res = np.linalg.norm(b.reshape(op.shape) - op.apply_D(xv)) / np.linalg.norm(b)
    assert res <= 1.0000001e-10
    load(0)


@pytest.mark.parametrize("coarsest", [0, 1, 2])
def test_three_level_16x16x16x32(coarsest):
    cfg = inputs.config("c5_16x16x16x32")
    dims = cfg["dims"]
    m0 = cfg["m0"][0]
    U = inputs.gauge_field(dims, cfg["eps"], cfg["gauge_seed"], ape_sweeps=cfg["ape"])
    ctx = w.Context(dims)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    ctx.set_clover(m0, cfg["csw"])
    ctx.set_mg_params(w.default_params(nlevels=2, block=cfg["blocks"], nvec=cfg["nvec"], seed=cfg["setup_seed"],
                                       coarsest=coarsest))
    for lvl in (0, 1):
        ctx.build_null_vectors(lvl)
        ctx.build_coarse(lvl)
        print("level", lvl, "built", flush=True)
    nrhs = cfg["nrhs"]
    b = np.stack([inputs.z2_source(dims, s) for s in cfg["source_seeds"][:nrhs]])
    x, st = ctx.solve(canon(b, (nrhs,) + tuple(reversed(dims)) + (4, 3)), w.MG_GCR, 1e-10)
    print("coarsest", coarsest, [(s["iters"], s["inner_iters"]) for s in st], flush=True)
    op = WilsonClover(dims, U, m0, cfg["csw"])
    xs = x.cpu().numpy().reshape((nrhs,) + op.shape)
    for r in range(nrhs):
        bv = b[r].reshape(op.shape)
        res = np.linalg.norm(bv - op.apply_D(xs[r])) / np.linalg.norm(bv)
        assert res <= 1.0000001e-10, (r, res)
    ctx.close()
