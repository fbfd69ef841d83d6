"""The coarse solve of the cycle in one cooperative launch (persistent GCR).

The whole red-black GCR of a coarse level (reduced source, GCR(m) with
classical Gram-Schmidt and a true residual at the end of every cycle,
reconstruction) runs in one launch with grid barriers.  Checked against
the oracle's coarse stencil, which the oracle builds itself (R D_p P,
direction resolved) from the same imported null vectors:

* tight tolerance: the solution equals the dense FP64 solve of the coarse
  system (small lattice) and the full coarse residual, recomputed by the
  oracle, is within the tolerance; FP32 to its own accuracy;
* the same solve issued one kernel at a time (launch 1) reaches the same
  tolerance in the same number of steps (within 2: the two sum in
  different orders), and the two solutions agree;
* the cycle's own setting (tol 0.1), ragged site counts (coarse sites not
  a multiple of the workgroup count), restart 1 and 64, a zero source;
* with at most one even site per workgroup (32 and 512 coarse sites)
  launch 0 runs the one-site kernel (basis in LDS, neighbour waits); it
  must give bitwise the solution and the step count of the strided kernel
  (launch 2), over several restart cycles, in FP64 and FP32;
* multigrid solves with coarse_launch 0 and 1 reach 1e-10 (oracle D) in
  outer iteration counts within 1 of each other, coarse_launch 2 gives
  bitwise the solution of 0, and the persistent kernel is the one that ran
  (its timer counts launches).
"""
import numpy as np
import pytest
import torch

import inputs
from oracle.dirac import WilsonClover
from oracle.multigrid import CoarseOperator, Transfer, coarse_operator

pytestmark = pytest.mark.gpu

w = pytest.importorskip("paper_1011_2775_amd")

# (fine dims, block, nvec): coarse sites 32 (16 per parity), 512, 1728 (864 per parity: ragged)
CASES = [((8, 8, 8, 16), (4, 4, 4, 4), 8), ((8, 8, 8, 16), (2, 2, 2, 2), 12), ((12, 12, 12, 16), (2, 2, 2, 2), 8)]


def canon(v, shape):
    return torch.from_numpy(np.ascontiguousarray(v).reshape(shape)).cuda()


def build(dims, block, nvec, m0=-0.2, csw=1.0, seed=11):
    U = inputs.gauge_field(dims, 0.3, 1000 + seed)
    ctx = w.Context(dims)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    ctx.set_clover(m0, csw)
    ctx.set_mg_params(w.default_params(block=[block], nvec=[nvec]))
    rng = np.random.default_rng(seed)
    V = int(np.prod(dims))
    v = rng.standard_normal((nvec, V, 4, 3)) + 1j * rng.standard_normal((nvec, V, 4, 3))
    ctx.set_null_vectors(canon(v, (nvec,) + tuple(reversed(dims)) + (4, 3)), level=0)
    ctx.build_coarse(0)
    op = WilsonClover(dims, U, m0, csw)
    T = Transfer(op, block, v)
    cop = CoarseOperator(T.cdims, coarse_operator(op, T))
    return ctx, cop, U


def rhs(cop, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(cop.shape) + 1j * rng.standard_normal(cop.shape)


def full_res(cop, x, b):
    return np.linalg.norm(b - cop.apply_D(x)) / np.linalg.norm(b)


@pytest.fixture(scope="module", params=range(len(CASES)), ids=["32sites", "512sites", "1728sites"])
def case(request):
    dims, block, nvec = CASES[request.param]
    print("case", dims, block, nvec, flush=True)
    ctx, cop, U = build(dims, block, nvec)
    yield ctx, cop
    ctx.close()


def test_tight_solve_fp64(case):
    ctx, cop = case
    b = rhs(cop, 1)
    bt = torch.from_numpy(b).cuda()
    xp, sp = ctx.coarse_solve(bt, prec=w.F64, tol=1e-12, max_iter=2000, restart=30, launch=0)
    xs, ss = ctx.coarse_solve(bt, prec=w.F64, tol=1e-12, max_iter=2000, restart=30, launch=1)
    xp, xs = xp.cpu().numpy(), xs.cpu().numpy()
    print("iters persistent %d, per-kernel %d" % (sp["iters"], ss["iters"]), flush=True)
    assert sp["status"] == "OK" and ss["status"] == "OK"
    assert full_res(cop, xp, b) < 1e-11
    assert full_res(cop, xs, b) < 1e-11
    assert abs(sp["true_rel_res"] - full_res(cop, xp, b)) < 1e-12
    assert abs(sp["iters"] - ss["iters"]) <= 2
    assert np.linalg.norm(xp - xs) / np.linalg.norm(xs) < 1e-9
    if cop.lat.V * cop.n <= 1024:
        x = np.linalg.solve(cop.dense(), b.reshape(-1)).reshape(cop.shape)
        assert np.linalg.norm(xp - x) / np.linalg.norm(x) < 1e-10


def test_fp32_solve(case):
    ctx, cop = case
    b = rhs(cop, 2)
    bt = torch.from_numpy(b).cuda()
    xp, sp = ctx.coarse_solve(bt, prec=w.F32, tol=1e-5, max_iter=2000, restart=30, launch=0)
    xs, ss = ctx.coarse_solve(bt, prec=w.F32, tol=1e-5, max_iter=2000, restart=30, launch=1)
    rp, rs = full_res(cop, xp.cpu().numpy(), b), full_res(cop, xs.cpu().numpy(), b)
    print("F32 iters %d / %d, residuals %.2e / %.2e" % (sp["iters"], ss["iters"], rp, rs), flush=True)
    assert rp < 2e-5 and rs < 2e-5
    assert abs(sp["iters"] - ss["iters"]) <= 2


@pytest.mark.parametrize("prec", ["F64", "F32"])
def test_cycle_setting(case, prec):
    """tol 0.1, the cycle's setting: same step count as the per-kernel solve."""
    ctx, cop = case
    b = rhs(cop, 3)
    bt = torch.from_numpy(b).cuda()
    xp, sp = ctx.coarse_solve(bt, prec=getattr(w, prec), tol=0.1, max_iter=100, restart=30, launch=0)
    xs, ss = ctx.coarse_solve(bt, prec=getattr(w, prec), tol=0.1, max_iter=100, restart=30, launch=1)
    assert sp["iters"] == ss["iters"] or abs(sp["iters"] - ss["iters"]) <= 1
    br = cop.reduced_source(b)
    bound = 0.1 * np.linalg.norm(br) / np.linalg.norm(b)
    assert full_res(cop, xp.cpu().numpy(), b) <= bound * 1.01


@pytest.mark.parametrize("restart", [1, 64])
def test_restart_extremes(case, restart):
    ctx, cop = case
    b = rhs(cop, 4)
    bt = torch.from_numpy(b).cuda()
    xp, sp = ctx.coarse_solve(bt, prec=w.F64, tol=1e-8, max_iter=5000, restart=restart, launch=0)
    xs, ss = ctx.coarse_solve(bt, prec=w.F64, tol=1e-8, max_iter=5000, restart=restart, launch=1)
    assert full_res(cop, xp.cpu().numpy(), b) < 1e-7
    assert abs(sp["iters"] - ss["iters"]) <= max(2, ss["iters"] // 50)


@pytest.mark.parametrize("prec,tol,restart", [("F64", 1e-9, 8), ("F64", 0.1, 30), ("F32", 1e-4, 6), ("F32", 0.2, 30)])
def test_one_site_kernel_matches_strided(case, prec, tol, restart):
    ctx, cop = case
    b = rhs(cop, 6)
    bt = torch.from_numpy(b).cuda()
    xo, so = ctx.coarse_solve(bt, prec=getattr(w, prec), tol=tol, max_iter=3000, restart=restart, launch=0)
    xg, sg = ctx.coarse_solve(bt, prec=getattr(w, prec), tol=tol, max_iter=3000, restart=restart, launch=2)
    print("%s tol %g restart %d: iters %d / %d" % (prec, tol, restart, so["iters"], sg["iters"]), flush=True)
    assert so["status"] == "OK" and sg["status"] == "OK"
    assert so["iters"] == sg["iters"]
    assert torch.equal(xo, xg)
    br = cop.reduced_source(b)
    assert full_res(cop, xo.cpu().numpy(), b) <= 1.01 * tol * np.linalg.norm(br) / np.linalg.norm(b) + \
        (1e-5 if prec == "F32" else 0.0)


@pytest.mark.parametrize("tol,restart", [(0.2, 30), (1e-3, 20)])
def test_fp16_hop_blocks(case, tol, restart):
    """launch 3 / 4: the hop blocks read in FP16 (FP32 vectors and arithmetic;
    the one-site kernel keeps the even site's blocks in LDS).  The two kernels
    give the same bits; the solution meets the tolerance on the oracle's FP64
    operator up to the FP16 rounding of the blocks (about 5e-4 relative); at
    the cycle's tolerance the step count is that of FP32 blocks within 2."""
    ctx, cop = case
    b = rhs(cop, 8)
    bt = torch.from_numpy(b).cuda()
    x3, s3 = ctx.coarse_solve(bt, prec=w.F32, tol=tol, max_iter=2000, restart=restart, launch=3)
    x4, s4 = ctx.coarse_solve(bt, prec=w.F32, tol=tol, max_iter=2000, restart=restart, launch=4)
    x0, s0 = ctx.coarse_solve(bt, prec=w.F32, tol=tol, max_iter=2000, restart=restart, launch=0)
    print("FP16 blocks tol %g: iters %d / %d, FP32 blocks %d" % (tol, s3["iters"], s4["iters"], s0["iters"]),
          flush=True)
    assert s3["status"] == "OK" and s4["status"] == "OK"
    assert s3["iters"] == s4["iters"] and torch.equal(x3, x4)
    br = cop.reduced_source(b)
    assert full_res(cop, x3.cpu().numpy(), b) <= 1.01 * tol * np.linalg.norm(br) / np.linalg.norm(b) + 2e-3
    if tol >= 0.1:
        assert abs(s3["iters"] - s0["iters"]) <= 2


def test_zero_source(case):
    ctx, cop = case
    bt = torch.zeros(cop.shape, dtype=torch.complex128, device="cuda")
    x, st = ctx.coarse_solve(bt, prec=w.F64, tol=0.1, max_iter=100, restart=30, launch=0)
    assert st["iters"] == 0
    assert torch.count_nonzero(x).item() == 0


@pytest.mark.parametrize("nlevels", [1, 2])
def test_multigrid_with_persistent_coarse_solve(nlevels):
    dims = (8, 8, 8, 16)
    U = inputs.gauge_field(dims, 0.3, 1021)
    m0, csw = -0.2, 1.0
    ctx = w.Context(dims)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    ctx.set_clover(m0, csw)
    if nlevels == 1:
        kw = dict(block=[(2, 2, 2, 2)], nvec=[12], max_iter=[100], restart=[30])
    else:
        kw = dict(nlevels=2, block=[(2, 2, 2, 2), (2, 2, 2, 2)], nvec=[12, 16], max_iter=[20, 100],
                  restart=[20, 30])
    ctx.set_mg_params(w.default_params(seed=5, **kw))
    for lvl in range(nlevels):
        ctx.build_null_vectors(lvl)
        ctx.build_coarse(lvl)
    vecs = [ctx.get_null_vectors(level=l) for l in range(nlevels)]
    b = canon(inputs.z2_source(dims, 3200), (1,) + tuple(reversed(dims)) + (4, 3))
    op = WilsonClover(dims, U, m0, csw)
    iters, sols = {}, {}
    for launch in (0, 1, 2):
        ctx.set_mg_params(w.default_params(seed=5, coarse_launch=launch, **kw))
        for l in range(nlevels):
            ctx.set_null_vectors(vecs[l], level=l)
            ctx.build_coarse(l)
        ctx.timer_enable(True)
        x, st = ctx.solve(b, w.MG_GCR, 1e-10)
        n_persist, _ = ctx.timer_read(28 + nlevels - 1)
        ctx.timer_enable(False)
        xv = x.cpu().numpy().reshape(op.shape)
        bv = b.cpu().numpy().reshape(op.shape)
        res = np.linalg.norm(bv - op.apply_D(xv)) / np.linalg.norm(bv)
        print("launch %d: outer %d, inner %s, res %.2e, persistent launches %d"
              % (launch, st[0]["iters"], st[0]["inner_iters"][:nlevels], res, n_persist), flush=True)
        assert res <= 1.0000001e-10
        assert (n_persist > 0) == (launch != 1)
        iters[launch] = st[0]
        sols[launch] = x
    assert abs(iters[0]["iters"] - iters[1]["iters"]) <= 1
    assert iters[0]["iters"] == iters[2]["iters"] and torch.equal(sols[0], sols[2])
    # FP16 hop blocks in the persistent coarsest solve: the same answer, outer
    # iteration count within 1 of FP32 blocks
    ctx.set_mg_params(w.default_params(seed=5, coarse_fp16=1, **kw))
    for l in range(nlevels):
        ctx.set_null_vectors(vecs[l], level=l)
        ctx.build_coarse(l)
    x16, s16 = ctx.solve(b, w.MG_GCR, 1e-10)
    xv = x16.cpu().numpy().reshape(op.shape)
    bv = b.cpu().numpy().reshape(op.shape)
    res = np.linalg.norm(bv - op.apply_D(xv)) / np.linalg.norm(bv)
    print("FP16 coarse blocks: outer %d, res %.2e" % (s16[0]["iters"], res), flush=True)
    assert res <= 1.0000001e-10 and abs(s16[0]["iters"] - iters[0]["iters"]) <= 1
    last = nlevels - 1
    assert abs(iters[0]["inner_iters"][last] - iters[1]["inner_iters"][last]) <= \
        0.1 * iters[1]["inner_iters"][last] + 1
    ctx.close()


@pytest.mark.parametrize("nvec,restart,prec", [(40, 30, "F32"), (40, 20, "F64"), (64, 64, "F64"), (64, 30, "F32")])
def test_one_site_kernel_wide_blocks(nvec, restart, prec):
    """n = 2 Nv of 80 and 128 on a 2^3x4 coarse lattice (16 even sites): the
    one-site kernel's block-wide step sums (n > 64), fewer hop columns staged
    in LDS, and, for n = 128 with restart 64 in FP64, a basis too large for
    LDS (the strided kernel runs for both launches).  Bitwise equal to the
    strided kernel; the full coarse residual (oracle) meets the tolerance."""
    dims, block = (8, 8, 8, 16), (4, 4, 4, 4)
    ctx, cop, U = build(dims, block, nvec, seed=13)
    b = rhs(cop, 7)
    bt = torch.from_numpy(b).cuda()
    tol = 1e-8 if prec == "F64" else 1e-4
    xo, so = ctx.coarse_solve(bt, prec=getattr(w, prec), tol=tol, max_iter=400, restart=restart, launch=0)
    xg, sg = ctx.coarse_solve(bt, prec=getattr(w, prec), tol=tol, max_iter=400, restart=restart, launch=2)
    print("n %d restart %d %s: iters %d / %d" % (2 * nvec, restart, prec, so["iters"], sg["iters"]), flush=True)
    assert so["status"] == "OK" and sg["status"] == "OK"
    assert so["iters"] == sg["iters"] and torch.equal(xo, xg)
    br = cop.reduced_source(b)
    slack = 1e-5 if prec == "F32" else 1e-12
    assert full_res(cop, xo.cpu().numpy(), b) <= 1.01 * tol * np.linalg.norm(br) / np.linalg.norm(b) + slack
    ctx.close()
