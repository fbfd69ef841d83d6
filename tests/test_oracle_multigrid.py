"""Pins of the oracle's multigrid pieces (CPU only).

P/R/Yhat are pinned given imported vectors: the block x chirality split is
checked against a library QR, the coarse operator against a brute-force
R D_p P and a U = 1 closed form, and the solver end to end against a dense
solve.  The setup itself is a heuristic and is parity unpinned; only its
invariants are checked.
"""
import os

import numpy as np
import pytest

import inputs
from oracle import multigrid as mg
from oracle.dirac import WilsonClover
from oracle.krylov import norm, SolveInfo
from oracle.lattice import GAMMA
from oracle.philox import philox4x32_10, gaussian_vector

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def unit_links(dims):
    V = inputs.volume(dims)
    return np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()


def rand_vecs(n, shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n,) + shape) + 1j * rng.standard_normal((n,) + shape)


@pytest.fixture(scope="module")
def c1():
    cfg = inputs.config("c1_4x4x4x4")
    U = inputs.gauge_field(cfg["dims"], cfg["eps"], cfg["gauge_seed"])
    op = WilsonClover(cfg["dims"], U, cfg["m0"][0], cfg["csw"])
    return cfg, op


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    for r in rows:
        v = [int(w, 16) for w in r]
        out = philox4x32_10(v[0:4], v[4:6])
        assert [int(o) for o in out] == v[6:10]


def test_gaussian_start_vectors_statistics():
    g = gaussian_vector(3001, 0, 0, 200000)
    assert abs(np.mean(g)) < 0.01
    assert abs(np.mean(np.abs(g) ** 2) - 2.0) < 0.02
    assert abs(np.mean(g.real * g.imag)) < 0.01


def test_block_orthonormalize_is_phase_fixed_qr(c1):
    cfg, op = c1
    vecs = rand_vecs(8, op.shape, 21)
    T = mg.Transfer(op, (2, 2, 2, 2), vecs)
    vecs = vecs.reshape(8, op.lat.V, 12)
    # per (block, chirality) the result equals numpy's QR with the diagonal of R
    # made real positive
    for b in (0, 7, 15):
        sites = np.nonzero(T.block_of == b)[0]
        for s in (0, 1):
            comps = np.nonzero(op.chirality == s)[0]
            M = vecs[:, sites][:, :, comps].reshape(8, -1).T
            Q, R = np.linalg.qr(M)
            ph = np.diagonal(R) / np.abs(np.diagonal(R))
            Q = Q * ph[None, :]
            got = T.V[:, sites][:, :, comps].reshape(8, -1).T
            assert np.abs(got - Q).max() < 1e-12


def test_transfer_algebra(c1):
    cfg, op = c1
    T = mg.Transfer(op, (2, 2, 2, 2), rand_vecs(8, op.shape, 22))
    P = T.dense_P()
    assert np.abs(P.conj().T @ P - np.eye(P.shape[1])).max() < 1e-13
    g5 = np.tile(np.repeat([1.0, 1.0, -1.0, -1.0], 3), op.lat.V)
    G5c = np.tile(np.repeat([1.0, -1.0], 8), T.Vc)
    assert np.abs(g5[:, None] * P - P * G5c[None, :]).max() < 1e-14     # gamma5 P = P Gamma5
    R = P.conj().T * g5[None, :]                                            # R = P^dag gamma5
    r = rand_vecs(1, op.shape, 23)[0]
    assert np.abs(R @ r.reshape(-1) - T.restrict(r).reshape(-1)).max() < 1e-13


def test_coarse_operator_equals_brute_force_RDpP(c1):
    cfg, op = c1
    T = mg.Transfer(op, (2, 2, 2, 2), rand_vecs(8, op.shape, 24))
    Y = mg.coarse_operator(op, T)
    Yd = mg.CoarseOperator(T.cdims, Y).dense()
    Dp = op.dense(op.apply_Dp)
    P = T.dense_P()
    g5 = np.tile(np.repeat([1.0, 1.0, -1.0, -1.0], 3), op.lat.V)
    Ybf = (P.conj().T * g5[None, :]) @ Dp @ P
    assert np.abs(Yd - Ybf).max() < 1e-13 * np.abs(Ybf).max()
    # coarse correction identity  P (R D_p P)^-1 R = P (P^dag D_p P)^-1 P^dag
    lhs = P @ np.linalg.solve(Ybf, P.conj().T * g5[None, :])
    rhs = P @ np.linalg.solve(P.conj().T @ Dp @ P, P.conj().T)
    assert np.abs(lhs - rhs).max() < 1e-11 * np.abs(rhs).max()


def test_coarse_operator_direction_resolved_odd_coarse_extent():
    """6^4 with 2^4 blocks gives a 3^4 coarse lattice where +mu and -mu
    neighbours differ, so every direction block is pinned separately."""
    dims = (6, 6, 6, 6)
    op = WilsonClover(dims, inputs.gauge_field(dims, 0.5, 25), -0.2, 1.0)
    T = mg.Transfer(op, (2, 2, 2, 2), rand_vecs(2, op.shape, 26))
    Y = mg.coarse_operator(op, T)
    Ybf = mg.coarse_operator_brute_force(op, T)
    cop = mg.CoarseOperator(T.cdims, Y)
    n = 4
    Ybf = Ybf.reshape(T.Vc, n, T.Vc, n)
    for c in range(T.Vc):
        assert np.abs(Ybf[c, :, c, :] - Y[c, 0]).max() < 1e-13
        for d in range(8):
            nb = cop.nbr(d)[c]
            assert np.abs(Ybf[c, :, nb, :] - Y[c, 1 + d]).max() < 1e-13
        # no other block of the row is populated
        others = np.setdiff1d(np.arange(T.Vc), [c] + [cop.nbr(d)[c] for d in range(8)])
        assert np.abs(Ybf[c, :, others, :]).max() == 0.0


@pytest.mark.parametrize("t_bc", [1, -1])
def test_coarse_operator_free_field_closed_form(t_bc):
    """U = 1 and block-constant vectors v_(alpha,a) = e_(alpha,a) + e_(alpha+2,a):
    Yhat = Gamma5 (4+m0)^-1 [X = 4+m0 - sum (b-1)/b,  Y_{+-mu} = -(1 -+ gamma_mu)/(2 b_mu)]."""
    dims = (4, 4, 4, 8)
    blocks = (2, 2, 2, 4)
    m0 = -0.1
    op = WilsonClover(dims, unit_links(dims), m0, 1.0, t_bc=t_bc)
    vecs = np.zeros((6,) + op.shape, dtype=np.complex128)
    for alpha in range(2):
        for a in range(3):
            vecs[alpha * 3 + a, :, alpha, a] = 1.0
            vecs[alpha * 3 + a, :, alpha + 2, a] = 1.0
    T = mg.Transfer(op, blocks, vecs)
    Y = mg.coarse_operator(op, T)
    cl = mg.CoarseOperator(T.cdims, Y).lat
    G5 = np.kron(np.diag([1.0, 1, -1, -1]), np.eye(3))
    X = (4 + m0 - sum((b - 1) / b for b in blocks)) * np.eye(12)
    assert np.abs(Y[:, 0] - G5 @ X / (4 + m0)).max() < 1e-14
    for mu in range(4):
        for back in (0, 1):
            sgn = 1 if back else -1
            blk = -np.kron(np.eye(4) + sgn * GAMMA[mu], np.eye(3)) / (2 * blocks[mu])
            want = np.broadcast_to(G5 @ blk / (4 + m0), (T.Vc, 12, 12)).copy()
            if mu == 3 and t_bc == -1:
                edge = cl.coords[:, 3] == (0 if back else T.cdims[3] - 1)
                want[edge] *= -1
            assert np.abs(Y[:, 1 + 2 * mu + back] - want).max() < 1e-14


def test_coarse_hermitian_without_clover():
    dims = (4, 4, 4, 4)
    op = WilsonClover(dims, inputs.gauge_field(dims, 0.4, 27), -0.2, 0.0)
    T = mg.Transfer(op, (2, 2, 2, 2), rand_vecs(4, op.shape, 28))
    Yd = mg.CoarseOperator(T.cdims, mg.coarse_operator(op, T)).dense()
    assert np.abs(Yd - Yd.conj().T).max() < 1e-13
    op2 = WilsonClover(dims, op.U, -0.2, 1.0)
    T2 = mg.Transfer(op2, (2, 2, 2, 2), rand_vecs(4, op.shape, 28))
    Yd2 = mg.CoarseOperator(T2.cdims, mg.coarse_operator(op2, T2)).dense()
    assert np.abs(Yd2 - Yd2.conj().T).max() > 1e-4


def test_coarse_red_black_matches_dense(c1):
    cfg, op = c1
    T = mg.Transfer(op, (2, 2, 2, 2), rand_vecs(8, op.shape, 29))
    cop = mg.CoarseOperator(T.cdims, mg.coarse_operator(op, T))
    b = rand_vecs(1, cop.shape, 30)[0]
    x_dense = np.linalg.solve(cop.dense(), b.reshape(-1)).reshape(cop.shape)
    br = cop.reduced_source(b)
    ev = cop.lat.parity == 0
    Dr = np.zeros((ev.sum() * cop.n,) * 2, dtype=np.complex128)
    # dense D_r column by column on the even sublattice
    idx = np.nonzero(ev)[0]
    for j, (c, i) in enumerate([(c, i) for c in idx for i in range(cop.n)]):
        e = np.zeros(cop.shape, dtype=np.complex128)
        e[c, i] = 1
        Dr[:, j] = cop.apply_Dr(e)[idx].reshape(-1)
    y = np.zeros(cop.shape, dtype=np.complex128)
    y[idx] = np.linalg.solve(Dr, br[idx].reshape(-1)).reshape(-1, cop.n)
    x = cop.reconstruct(y, b)
    assert norm(x - x_dense) / norm(x_dense) < 1e-11


def test_setup_invariants(c1):
    cfg, op = c1
    stats = []
    vecs = mg.setup_null_vectors(op, 6, seed=cfg["setup_seed"], stats=stats)
    flat = vecs.reshape(6, -1)
    G = flat.conj() @ flat.T
    assert np.abs(G - np.eye(6)).max() < 1e-12
    rq = [norm(op.apply_Dp(v)) ** 2 for v in vecs]
    rnd = rand_vecs(6, op.shape, 31)
    rq_rand = [norm(op.apply_Dp(v)) ** 2 / norm(v) ** 2 for v in rnd]
    assert max(rq) < 0.2 * min(rq_rand)
    assert all(1 <= s <= 10 for s, _ in stats)


def test_mg_gcr_c1_reaches_tolerance(c1):
    cfg, op = c1
    b = inputs.z2_source(cfg["dims"], cfg["source_seeds"][0]).reshape(op.shape)
    p = mg.MGParams(blocks=cfg["blocks"], nvec=cfg["nvec"], seed=cfg["setup_seed"])
    H = mg.Hierarchy(op, p)
    info = SolveInfo()
    x = H.solve(b, tol=cfg["tol"], info=info)
    assert info.converged
    res = norm(b - op.apply_D(x)) / norm(b)
    assert res <= 1e-10
    x_dense = np.linalg.solve(op.dense(op.apply_D), b.reshape(-1)).reshape(op.shape)
    assert norm(x - x_dense) / norm(x_dense) < 1e-8


def test_mg_three_levels_and_lu_coarsest():
    dims = (8, 8, 8, 8)
    op = WilsonClover(dims, inputs.gauge_field(dims, 0.5, 32, ape_sweeps=1), -0.25, 1.0)
    b = inputs.z2_source(dims, 33).reshape(op.shape)
    p = mg.MGParams(blocks=[(2, 2, 2, 2), (2, 2, 2, 2)], nvec=[6, 6], seed=34,
                    n_relax=4, s_max=3)
    H = mg.Hierarchy(op, p)
    info = SolveInfo()
    x = H.solve(b, tol=1e-10, info=info)
    assert info.converged and norm(b - op.apply_D(x)) / norm(b) <= 1e-10
    assert H.inner_calls[2] > 0
    p.coarsest = "lu"
    info = SolveInfo()
    x2 = H.solve(b, tol=1e-10, info=info)
    assert info.converged and norm(x2 - x) / norm(x) < 1e-8


def test_four_levels_galerkin_at_every_coarse_level():
    """Three coarse levels (8^4 -> 4^4 -> 2x2x4x4 -> 2^4, blocks of extent 1 in
    some directions): every coarse operator the hierarchy builds from a
    coarse level equals the brute-force R Dhat_p P of that level, and the
    four-level solve reaches the tolerance."""
    dims = (8, 8, 8, 8)
    op = WilsonClover(dims, inputs.gauge_field(dims, 0.4, 35), -0.1, 1.0)
    blocks = [(2, 2, 2, 2), (2, 2, 1, 1), (1, 1, 2, 2)]
    nvec = [4, 4, 4]
    V1, V2 = op.lat.V // 16, op.lat.V // 64
    vecs = [rand_vecs(4, op.shape, 36), rand_vecs(4, (V1, 8), 37), rand_vecs(4, (V2, 8), 38)]
    H = mg.Hierarchy(op, mg.MGParams(blocks, nvec), vecs=vecs)
    assert [o.lat.dims for o in H.ops[1:]] == [(4, 4, 4, 4), (2, 2, 4, 4), (2, 2, 2, 2)]
    for l in (1, 2):
        Ybf = mg.coarse_operator_brute_force(H.ops[l], H.transfers[l])
        Yd = H.ops[l + 1].dense()
        assert np.abs(Yd - Ybf).max() < 1e-12 * np.abs(Ybf).max(), l
    b = inputs.z2_source(dims, 39).reshape(op.shape)
    info = SolveInfo()
    x = H.solve(b, tol=1e-8, info=info)
    assert info.converged and norm(b - op.apply_D(x)) / norm(b) <= 1e-8
    assert H.inner_calls[3] > 0
