"""The formulation of the library's GCR steps, checked on the CPU.

Each step of the outer (and setup) GCR in csrc/solvers.cpp is one multi-dot
and one fused pass, and the directions are kept raw:

* one pass of dot products gives <q_j, q> for the basis, <q, q> and <r, q>;
  with the basis orthogonal, ||q_orth||^2 = ||q||^2 - sum_j |<q_j, q>|^2 /
  ||q_j||^2 (Pythagoras) and <q_orth, r> = <q, r> (r is orthogonal to every
  q_j), so alpha is known before q is orthogonalised;
* the preconditioned vectors z_k are stored as they come; with the
  orthogonalisation coefficients c_jk = <q_j, q_k> / ||q_j||^2 the effective
  directions are z~_k = z_k - sum_{j<k} c_jk z~_j, and the cycle's update
  x += sum_k alpha_k z~_k equals x += sum_k y_k z_k with (I + C) y = alpha
  (back substitution).

This test runs that formulation in plain NumPy (written from the description
above) next to the oracle's classical GCR with the same fixed preconditioner
and requires the same residual history and solution; and, with every stored
vector rounded to single precision as in the FP32 setup GCR, a residual
history that tracks the FP64 one to single-precision accuracy.
"""
import numpy as np
import pytest

from oracle.krylov import SolveInfo, gcr, norm


def problem(n, seed):
    rng = np.random.default_rng(seed)
    A = np.eye(n) + 0.6 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    # a fixed, imperfect preconditioner: the inverse of a perturbed A
    E = 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    M = np.linalg.inv(A + E)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, M, b


def raw_direction_gcr(A, M, b, steps, store=np.complex128):
    rnd = (lambda v: v.astype(store).astype(np.complex128))
    r = b.copy()
    Q, qn2, Z, alphas = [], [], [], []
    C = np.zeros((steps, steps), dtype=np.complex128)
    hist = [norm(r)]
    for k in range(steps):
        z = rnd(M @ r)
        q = rnd(A @ z)
        beta = [np.vdot(Qj, q) for Qj in Q]
        qq = np.vdot(q, q).real
        for j, bj in enumerate(beta):
            if qn2[j] > 0:
                qq -= abs(bj) ** 2 / qn2[j]
        qr = np.vdot(q, r)
        c = [bj / qn2[j] if qn2[j] > 0 else 0.0 for j, bj in enumerate(beta)]
        q_o = q.copy()
        for j, cj in enumerate(c):
            q_o = q_o - cj * Q[j]
        q_o = rnd(q_o)
        alpha = qr / qq if qq > 0 else 0.0
        r = rnd(r - alpha * q_o)
        Q.append(q_o)
        qn2.append(qq)
        Z.append(z)
        C[:k, k] = c
        alphas.append(alpha)
        hist.append(norm(r))
    y = np.zeros(steps, dtype=np.complex128)
    for i in range(steps - 1, -1, -1):
        y[i] = alphas[i] - np.dot(C[i, i + 1:], y[i + 1:])
    x = sum(yi * zi for yi, zi in zip(y, Z))
    return x, np.array(hist), Z, C, np.array(alphas)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_matches_classical_gcr(seed):
    n, steps = 60, 12
    A, M, b = problem(n, seed)
    x, hist, Z, C, alphas = raw_direction_gcr(A, M, b, steps)
    info = SolveInfo()
    xo = gcr(lambda v: A @ v, b, tol=1e-300, restart=steps, maxiter=steps, precond=lambda v: M @ v, info=info)
    ho = np.array(info.history[:steps + 1])
    assert len(ho) == steps + 1
    np.testing.assert_allclose(hist, ho, rtol=1e-9, atol=1e-12 * ho[0])
    assert norm(x - xo) <= 1e-9 * norm(xo)
    # the recurrence residual is the true one
    assert abs(norm(b - A @ x) - hist[-1]) <= 1e-10 * hist[0]


def test_raw_directions_span_the_orthogonalised_ones():
    """z~_k built explicitly by the recurrence equal Z (I + C)^-1 column by column."""
    n, steps = 40, 8
    A, M, b = problem(n, 7)
    _, _, Z, C, _ = raw_direction_gcr(A, M, b, steps)
    Zm = np.array(Z).T
    Zt = []
    for k in range(steps):
        zt = Z[k].copy()
        for j in range(k):
            zt = zt - C[j, k] * Zt[j]
        Zt.append(zt)
    np.testing.assert_allclose(np.array(Zt).T, Zm @ np.linalg.inv(np.eye(steps) + C), rtol=1e-10, atol=1e-12)
    # and their images under A are mutually orthogonal
    G = np.array([A @ z for z in Zt])
    off = G.conj() @ G.T
    off = off - np.diag(np.diag(off))
    assert np.abs(off).max() <= 1e-9 * np.abs(G).max() ** 2 * n


def test_single_precision_storage_tracks_double():
    """Vectors stored in single precision (the FP32 setup GCR): the residual
    history stays within single-precision accuracy of the FP64 one while the
    residual is well above the rounding level, and the Pythagorean ||q||^2
    does not break down."""
    n, steps = 80, 16
    A, M, b = problem(n, 11)
    _, h64, *_ = raw_direction_gcr(A, M, b, steps)
    _, h32, *_ = raw_direction_gcr(A, M, b, steps, store=np.complex64)
    assert np.all(np.isfinite(h32))
    ok = h64 > 1e-4 * h64[0]
    assert ok.sum() >= 4
    np.testing.assert_allclose(h32[ok], h64[ok], rtol=2e-3)
