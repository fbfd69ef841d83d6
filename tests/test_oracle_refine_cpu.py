"""The oracle's adaptive null-vector refinement (Setup section, alphaSA /
hybrid; parity unpinned: a heuristic) checked by its invariants on the 4^4
workload: the refined vectors are orthonormal, satisfy D_p v = 0 on the odd
sites exactly (v_o = -D_oe D_ee^-1 v_e), sit lower in the spectrum of D_p than
the vectors they came from, and the hierarchy built on them still solves to
1e-10 in no more outer iterations than before."""
import numpy as np

import inputs
from oracle import multigrid as mg
from oracle.dirac import WilsonClover
from oracle.krylov import SolveInfo, norm


def test_refinement_invariants_c1():
    cfg = inputs.config("c1_4x4x4x4")
    dims = cfg["dims"]
    U = inputs.gauge_field(dims, cfg["eps"], cfg["gauge_seed"])
    op = WilsonClover(dims, U, cfg["m0"][0], cfg["csw"])
    # a deliberately cheap setup: one relaxation of 3 steps per vector
    params = mg.MGParams(cfg["blocks"], cfg["nvec"], seed=cfg["setup_seed"], n_relax=3, s_max=1)
    H0 = mg.Hierarchy(op, params)
    b = inputs.z2_source(dims, cfg["source_seeds"][0])
    i0 = SolveInfo()
    H0.solve(b, info=i0)
    H1 = mg.refine_null_vectors(H0, passes=1, iters=4)
    v = H1.raw[0].reshape(len(H1.raw[0]), -1)
    assert np.abs(v.conj() @ v.T - np.eye(len(v))).max() < 1e-12
    lat = op.lat
    for w in H1.raw[0]:
        dp = op.apply_Dp(w)
        assert norm(dp[lat.odd]) < 1e-12 * norm(w)
    rq = lambda vs: np.mean([norm(op.apply_Dp(x)) ** 2 / norm(x) ** 2 for x in vs])  # noqa: E731
    assert rq(H1.raw[0]) < rq(H0.raw[0])
    i1 = SolveInfo()
    x = H1.solve(b, info=i1)
    assert norm(b.reshape(op.shape) - op.apply_D(x)) / norm(b) <= 1e-10
    assert i1.iters <= i0.iters
