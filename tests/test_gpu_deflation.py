"""Deflated FP64 GCR on the coarsest level (coarsest = 2).

K low modes of the coarsest operator, found by inverse iteration when the
level is built, stay at the head of the coarsest GCR basis, and every coarse
solve starts from the deflated guess.  The solve reaches the same tolerance
as plain GCR: the multigrid solves must reach 1e-10 (oracle D), on red-black
coarse lattices and on a coarse lattice with odd extents (full operator),
with adaptive and fixed-length cycles; deflation must not need more
coarsest steps than plain GCR.
"""
import numpy as np
import pytest
import torch

import inputs
from oracle.dirac import WilsonClover

pytestmark = pytest.mark.gpu

w = pytest.importorskip("paper_1011_2775_amd")


def canon(v, shape):
    return torch.from_numpy(np.ascontiguousarray(v).reshape(shape)).cuda()


def setup(dims, block, nvec, m0=-0.2, seed=23):
    U = inputs.gauge_field(dims, 0.3, 1000 + seed)
    ctx = w.Context(dims)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    ctx.set_clover(m0, 1.0)
    ctx.set_mg_params(w.default_params(block=[block], nvec=[nvec], seed=seed))
    ctx.build_null_vectors()
    vecs = ctx.get_null_vectors()
    return ctx, WilsonClover(dims, U, m0, 1.0), vecs


def solve(ctx, op, vecs, dims, block, nvec, **kw):
    ctx.set_mg_params(w.default_params(block=[block], nvec=[nvec], seed=23, **kw))
    ctx.set_null_vectors(vecs)
    ctx.build_coarse()
    b = inputs.z2_source(dims, 3300)
    x, st = ctx.solve(canon(b, (1,) + tuple(reversed(dims)) + (4, 3)), w.MG_GCR, 1e-10)
    xv = x.cpu().numpy().reshape(op.shape)
    res = np.linalg.norm(b.reshape(op.shape) - op.apply_D(xv)) / np.linalg.norm(b)
    print(kw, "outer", st[0]["iters"], "coarsest steps per solve", st[0]["inner_iters"][0], "res %.2e" % res,
          flush=True)
    return res, st[0]


def test_deflated_coarsest_red_black():
    dims, block, nvec = (8, 8, 8, 16), (2, 2, 2, 2), 12
    ctx, op, vecs = setup(dims, block, nvec)
    res0, st0 = solve(ctx, op, vecs, dims, block, nvec, max_iter=[200], restart=[30])
    res2, st2 = solve(ctx, op, vecs, dims, block, nvec, max_iter=[200], restart=[30], coarsest=2, nvec_defl=24)
    assert res0 <= 1.0000001e-10 and res2 <= 1.0000001e-10
    assert st2["inner_iters"][0] <= st0["inner_iters"][0]
    assert abs(st2["iters"] - st0["iters"]) <= 2
    # fixed-length cycles with the deflated coarsest solve
    res3, _ = solve(ctx, op, vecs, dims, block, nvec, max_iter=[12], restart=[12], coarsest=2, nvec_defl=24,
                    cycle_mode=1)
    assert res3 <= 1.0000001e-10
    ctx.close()


def test_deflated_coarsest_odd_extents():
    """Coarse lattice 3x3x3x4: no red-black form, the full coarse operator is deflated."""
    dims, block, nvec = (12, 12, 12, 16), (4, 4, 4, 4), 8
    ctx, op, vecs = setup(dims, block, nvec)
    res, st = solve(ctx, op, vecs, dims, block, nvec, max_iter=[200], restart=[30], coarsest=2, nvec_defl=16)
    assert res <= 1.0000001e-10
    ctx.close()
