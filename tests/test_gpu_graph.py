"""Fixed-length cycles and their HIP-graph replay.

cycle_mode 1 runs every inner GCR for exactly max_iter steps with no host
round trip; cycle_mode 2 captures that preconditioner once into a HIP graph
and replays it at every outer iteration.  The replays must reproduce the
eager fixed-length cycle bitwise: the outer GCR (run eagerly, with host reads
and synchronisations between replays) then produces bitwise the same
solution, on repeated solves and after other eager work on the context.
Both modes must still reach the 1e-10 true residual.  The comparison pins
the per-kernel coarse solve (coarse_launch 1) on both sides: a graph does
not hold the cooperative single-launch coarse solve, which sums in another
order; the fixed-length cycle with that solve must still converge.
"""
import numpy as np
import pytest
import torch

import inputs
from oracle.dirac import WilsonClover

pytestmark = pytest.mark.gpu

w = pytest.importorskip("paper_1011_2775_amd")


def canon(v, dims):
    return torch.from_numpy(np.ascontiguousarray(v).reshape((-1,) + tuple(reversed(dims)) + (4, 3))).cuda()


@pytest.mark.parametrize("nlevels", [1, 2])
def test_graph_replay_matches_eager(nlevels):
    dims = (8, 8, 8, 16)
    U = inputs.gauge_field(dims, 0.3, 1008)
    m0, csw = -0.2, 1.0
    ctx = w.Context(dims)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    ctx.set_clover(m0, csw)
    if nlevels == 1:
        kw = dict(block=[(4, 4, 4, 4)], nvec=[12], max_iter=[8])
    else:
        kw = dict(nlevels=2, block=[(2, 2, 2, 2), (2, 2, 2, 2)], nvec=[8, 8], max_iter=[6, 6], coarsest=1)
    ctx.set_mg_params(w.default_params(seed=3013, **kw))
    for lvl in range(nlevels):
        ctx.build_null_vectors(lvl)
        ctx.build_coarse(lvl)
    vecs = [ctx.get_null_vectors(level=l) for l in range(nlevels)]
    b = canon(inputs.z2_source(dims, 3100), dims)
    op = WilsonClover(dims, U, m0, csw)
    xs = {}
    for mode in (1, 2, 2):
        ctx.set_mg_params(w.default_params(seed=3013, cycle_mode=mode, coarse_launch=1, **kw))
        for l in range(nlevels):
            ctx.set_null_vectors(vecs[l], level=l)
            ctx.build_coarse(l)
        x, st = ctx.solve(b, w.MG_GCR, 1e-10)
        xv = x.cpu().numpy()
        res = np.linalg.norm(b.cpu().numpy().reshape(op.shape) - op.apply_D(xv.reshape(op.shape))) / \
            np.linalg.norm(b.cpu().numpy())
        assert res <= 1.0000001e-10, (mode, res)
        # eager work on the context between solves
        ctx.apply_D(b, w.OP_SCHUR, w.F32)
        # a second solve replays the same graph again
        x2, _ = ctx.solve(b, w.MG_GCR, 1e-10)
        assert torch.equal(x, x2), mode
        xs.setdefault(mode, []).append(xv)
        print("mode", mode, "outer iterations", st[0]["iters"], flush=True)
    assert np.array_equal(xs[1][0], xs[2][0])
    assert np.array_equal(xs[2][0], xs[2][1])

    # fixed-length cycles with the single-launch coarse solve
    ctx.set_mg_params(w.default_params(seed=3013, cycle_mode=1, coarse_launch=0, **kw))
    for l in range(nlevels):
        ctx.set_null_vectors(vecs[l], level=l)
        ctx.build_coarse(l)
    x, st = ctx.solve(b, w.MG_GCR, 1e-10)
    xv = x.cpu().numpy()
    res = np.linalg.norm(b.cpu().numpy().reshape(op.shape) - op.apply_D(xv.reshape(op.shape))) / \
        np.linalg.norm(b.cpu().numpy())
    assert res <= 1.0000001e-10
    ctx.close()


def test_adaptive_cycle_graph_with_persistent_coarse_solve():
    """cycle_mode 3: the adaptive two-level preconditioner whose coarse level
    is the single-launch persistent solve (tolerance tested on the device) is
    a pure kernel sequence; it is captured once and replayed at every outer
    iteration.  Replays equal the eager cycle bit for bit on repeated solves
    with eager work in between, and the coarse-step statistics are kept."""
    dims = (8, 8, 8, 16)
    U = inputs.gauge_field(dims, 0.3, 1008)
    m0, csw = -0.2, 1.0
    op = WilsonClover(dims, U, m0, csw)
    ctx = w.Context(dims)
    try:
        ctx.set_gauge(torch.from_numpy(U).cuda())
        ctx.set_clover(m0, csw)
        kw = dict(block=[(4, 4, 4, 4)], nvec=[12], seed=3013, restart=[30], max_iter=[100], tol=[0.2])
        ctx.set_mg_params(w.default_params(cycle_mode=0, **kw))
        ctx.build_null_vectors()
        ctx.build_coarse()
        vecs = ctx.get_null_vectors()
        b = canon(inputs.z2_source(dims, 2013), dims)
        x0, s0 = ctx.solve(b, w.MG_GCR, 1e-10)
        ctx.set_mg_params(w.default_params(cycle_mode=3, **kw))
        ctx.set_null_vectors(vecs)
        ctx.build_coarse()
        for rep in range(3):
            x3, s3 = ctx.solve(b, w.MG_GCR, 1e-10)
            print("replay", rep, s3[0]["iters"], s3[0]["inner_iters"][0], flush=True)
            assert torch.equal(x3, x0), rep
            assert s3[0]["iters"] == s0[0]["iters"]
            ctx.apply_D(b)  # eager work between solves
        assert s3[0]["inner_iters"][0] > 0
        xv = x3.cpu().numpy().reshape(op.shape)
        bv = inputs.z2_source(dims, 2013).reshape(op.shape)
        assert np.linalg.norm(bv - op.apply_D(xv)) / np.linalg.norm(bv) <= 1.0000001e-10
    finally:
        ctx.close()
