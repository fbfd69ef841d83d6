"""The allocation-free coarse solve (wcmg_coarse_solve_noalloc) against the
allocating one (wcmg_coarse_solve, launch 0): same kernel, same grid, so the
same iterations and the same solution, on two calls in a row -- the second
on a smaller coarse lattice, which finds the first call's contents in the
shared static array -- in FP64 and FP32; the solution also meets its
tolerance on the oracle's coarse operator; a solve whose work exceeds the
static array is refused before any launch."""
import numpy as np
import pytest
import torch

import inputs
from oracle.multigrid import CoarseOperator

pytestmark = pytest.mark.gpu

w = pytest.importorskip("paper_1011_2775_amd")


def build(dims, block, nvec, seed):
    U = inputs.gauge_field(dims, 0.3, 1000 + seed)
    ctx = w.Context(dims)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    ctx.set_clover(-0.2, 1.0)
    ctx.set_mg_params(w.default_params(block=[block], nvec=[nvec]))
    rng = np.random.default_rng(seed)
    V = int(np.prod(dims))
    v = rng.standard_normal((nvec, V, 4, 3)) + 1j * rng.standard_normal((nvec, V, 4, 3))
    ctx.set_null_vectors(torch.from_numpy(v.reshape((nvec,) + tuple(reversed(dims)) + (4, 3))).cuda(), level=0)
    ctx.build_coarse(0)
    cdims = tuple(d // b for d, b in zip(dims, block))
    return ctx, CoarseOperator(cdims, ctx.get_coarse(0))


@pytest.fixture(scope="module")
def pair():
    print("no-alloc: building 512-site and 32-site coarse levels", flush=True)
    big = build((8, 8, 8, 16), (2, 2, 2, 2), 12, 21)   # coarse 4^3x8, n = 24
    small = build((8, 8, 8, 16), (4, 4, 4, 4), 8, 22)  # coarse 2^3x4, n = 16
    yield big, small
    big[0].close()
    small[0].close()


@pytest.mark.parametrize("prec,tol", [("F64", 1e-10), ("F32", 1e-5)])
def test_two_calls_match_the_allocating_entry(pair, prec, tol):
    p = getattr(w, prec)
    for (ctx, cop), seed in zip(pair, (1, 2)):  # large first, then smaller
        rng = np.random.default_rng(seed)
        b = rng.standard_normal(cop.shape) + 1j * rng.standard_normal(cop.shape)
        bt = torch.from_numpy(b).cuda()
        print("no-alloc %s: %d coarse sites" % (prec, cop.lat.V), flush=True)
        xn, sn = ctx.coarse_solve_noalloc(bt, prec=p, tol=tol, max_iter=500, restart=30)
        xa, sa = ctx.coarse_solve(bt, prec=p, tol=tol, max_iter=500, restart=30, launch=0)
        assert sn["status"] == "OK" and sa["status"] == "OK"
        assert sn["iters"] == sa["iters"]
        xn, xa = xn.cpu().numpy(), xa.cpu().numpy()
        assert np.array_equal(xn, xa)  # the same kernel on the same inputs
        res = np.linalg.norm(b - cop.apply_D(xn)) / np.linalg.norm(b)
        assert res < 3 * tol
        assert abs(sn["true_rel_res"] - res) < 1e-3 * res + (1e-13 if prec == "F64" else 1e-6)


def test_refuses_a_solve_larger_than_the_static_array():
    ctx, cop = build((12, 12, 12, 16), (2, 2, 2, 2), 8, 23)  # coarse 6^3x8, n = 16
    try:
        bt = torch.zeros(cop.shape, dtype=torch.complex128, device="cuda")
        with pytest.raises(w.WcmgError, match="static scratch"):
            ctx.coarse_solve_noalloc(bt, prec=w.F64, tol=0.1, max_iter=500, restart=64)
        _, st = ctx.coarse_solve_noalloc(torch.ones(cop.shape, dtype=torch.complex128, device="cuda"),
                                         prec=w.F32, tol=0.1, max_iter=100, restart=10)
        assert st["status"] == "OK"
    finally:
        ctx.close()
