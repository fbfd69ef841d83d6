"""The multi-right-hand-side fine operator kernels against one right-hand
side at a time and against the FP64 oracle.

Several right-hand sides go through the interleaved-workgroup hop kernel by
default (one right-hand side per thread; the workgroups of a site block are
consecutive, so the links and clover records they share are read from HBM
once and then from L2) and through the register-group kernels when the tuner
picks them.  Checked: every operator form and its adjoint at F64/F32/F16 for
3, 12 and 20 right-hand sides on a lattice with a ragged last workgroup, with
antiperiodic and periodic time, equal to the one-at-a-time applies (FP64
1e-14, FP32 1e-6, FP16 2e-3, max-norm relative) and, at FP64, to the oracle
(1e-13); with the tuner on (which times every launch shape) the results stay
within the same bounds."""
import numpy as np
import pytest
import torch

import inputs
from oracle.dirac import WilsonClover

pytestmark = pytest.mark.gpu

w = pytest.importorskip("paper_1011_2775_amd")

TOL = {w.F64: 1e-14, w.F32: 1e-6, w.F16: 2e-3}
OPS = {"FULL": w.OP_FULL, "SCHUR": w.OP_SCHUR, "DP": w.OP_DP, "SCHUR_X": w.OP_SCHUR_X}


@pytest.fixture(scope="module", params=[-1, 1], ids=["antiperiodic", "periodic"])
def setup(request):
    dims = (6, 4, 8, 10)
    U = inputs.gauge_field(dims, 0.5, 1501)
    ctx = w.Context([(dims, request.param)])
    ctx.set_gauge(torch.from_numpy(U).cuda())
    ctx.set_clover(-0.2, 1.1)
    op = WilsonClover(dims, U, -0.2, 1.1, request.param)
    print("t_bc", request.param, flush=True)
    yield dims, ctx, op
    ctx.close()


def canon(v, dims):
    return torch.from_numpy(np.ascontiguousarray(v).reshape((-1,) + tuple(reversed(dims)) + (4, 3))).cuda()


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("nrhs", [3, 12, 20])
@pytest.mark.parametrize("opname", list(OPS))
@pytest.mark.parametrize("dag", [False, True])
def test_batched_equals_single(setup, nrhs, opname, dag):
    dims, ctx, op = setup
    V = op.lat.V
    rng = np.random.default_rng(nrhs)
    v = rng.standard_normal((nrhs, V, 4, 3)) + 1j * rng.standard_normal((nrhs, V, 4, 3))
    fn = ctx.apply_Ddag if dag else ctx.apply_D
    for prec in (w.F64, w.F32, w.F16):
        got = fn(canon(v, dims), OPS[opname], prec).cpu().numpy().reshape(nrhs, V, 4, 3)
        for r in (0, nrhs // 2, nrhs - 1):
            one = fn(canon(v[r], dims), OPS[opname], prec).cpu().numpy().reshape(V, 4, 3)
            assert rel(got[r], one) < TOL[prec], (prec, r)
        if prec == w.F64 and opname == "FULL":
            want = op.apply_Ddag(v[nrhs - 1]) if dag else op.apply_D(v[nrhs - 1])
            assert rel(got[nrhs - 1], want) < 1e-13


def test_tuned_shapes(setup):
    dims, ctx, op = setup
    V = op.lat.V
    rng = np.random.default_rng(5)
    v = rng.standard_normal((12, V, 4, 3)) + 1j * rng.standard_normal((12, V, 4, 3))
    ref = {p: ctx.apply_D(canon(v, dims), w.OP_SCHUR_X, p).cpu().numpy() for p in (w.F64, w.F32)}
    ctx.autotune(True)
    try:
        for p in (w.F64, w.F32):
            got = ctx.apply_D(canon(v, dims), w.OP_SCHUR_X, p).cpu().numpy()
            assert rel(got, ref[p]) < TOL[p]
        print("tuned:", [(r["prec"], r["diag"], r["group"], round(r["us"], 1)) for r in ctx.autotune_report()],
              flush=True)
    finally:
        ctx.autotune(False)
