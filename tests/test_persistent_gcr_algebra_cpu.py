"""The recurrences of the persistent coarse GCR, checked on the CPU.

The single-launch coarse solve (csrc/coarse_persist.hip) runs GCR on the
red-black reduced operator D_r = 1 - Ye Yo (Ye: odd -> even hop, Yo: even ->
odd hop, both with the diagonal inverse folded in) with two reformulations
that save global reductions and hops:

* Pythagoras: with q_0..q_{k-1} mutually orthogonal, the orthogonalised
  q_k = q - sum_j c_j q_j (c_j = <q_j, q> / ||q_j||^2) has
  ||q_k||^2 = ||q||^2 - sum_j |<q_j, q>|^2 / ||q_j||^2, and <q_k, r> = <q, r>
  because the residual is orthogonal to every earlier q_j; so alpha comes
  from sums taken before the orthogonalisation.
* linearity: the odd-site hop of the next direction z_{k+1} = r_{k+1} is
  t_{k+1} = Yo r_{k+1} = t_k - alpha T_k with T_k = Yo q_k
  = Yo q - sum_j c_j T_j, so no hop of r is needed inside a cycle.

This test runs those recurrences in plain NumPy (written here from the
description above, not from the kernel) on random red-black systems and
requires the residual history to match the oracle's classical GCR step by
step, the recurrence-built t to equal Yo r (to rounding of the cycle's start
scale: the recurrence drifts as r shrinks, which is why the kernel recomputes
the true residual at the end of every cycle), and ||q_k||^2 and <q_k, r> from
the identities to equal the directly computed values.
"""
import numpy as np
import pytest

from oracle.krylov import SolveInfo, gcr, norm


def system(ne, no, scale, seed):
    rng = np.random.default_rng(seed)
    Ye = scale * (rng.standard_normal((ne, no)) + 1j * rng.standard_normal((ne, no))) / np.sqrt(no)
    Yo = scale * (rng.standard_normal((no, ne)) + 1j * rng.standard_normal((no, ne))) / np.sqrt(ne)
    b = rng.standard_normal(ne) + 1j * rng.standard_normal(ne)
    return Ye, Yo, b


def persistent_form(Ye, Yo, b, steps):
    """GCR(steps) on D_r = 1 - Ye Yo from zero with the two reformulations;
    returns the residual norms and the per-step identity errors."""
    r = b.copy()
    y = np.zeros_like(b)
    t = Yo @ r  # cycle start: t = Yo z_0, z_0 = r
    z = r.copy()
    Q, Z, T, qn = [], [], [], []
    hist = [norm(r)]
    err_t = err_qq = err_qr = 0.0
    for k in range(steps):
        q = r - Ye @ t  # D_r z_k (z_k = r)
        dots = [np.vdot(qj, q) for qj in Q]
        qq = np.vdot(q, q).real - sum(abs(d) ** 2 / n for d, n in zip(dots, qn))
        qr = np.vdot(q, r)
        alpha = qr / qq
        c = [d / n for d, n in zip(dots, qn)]
        qk = q - sum((cj * qj for cj, qj in zip(c, Q)), np.zeros_like(q))
        zk = z - sum((cj * zj for cj, zj in zip(c, Z)), np.zeros_like(z))
        Tk = Yo @ q - sum((cj * Tj for cj, Tj in zip(c, T)), np.zeros_like(t))
        # the identities against direct evaluation
        err_qq = max(err_qq, abs(qq - np.vdot(qk, qk).real) / np.vdot(qk, qk).real)
        err_qr = max(err_qr, abs(qr - np.vdot(qk, r)) / abs(np.vdot(qk, r)))
        y = y + alpha * zk
        r = r - alpha * qk
        t = t - alpha * Tk
        z = r.copy()
        Q.append(qk)
        Z.append(zk)
        T.append(Tk)
        qn.append(qq)
        hist.append(norm(r))
        err_t = max(err_t, norm(t - Yo @ r) / norm(Yo @ b))  # drift against the cycle's start scale
        # the true residual of y matches the recurred one
        assert norm(b - (y - Ye @ (Yo @ y)) - r) <= 1e-11 * norm(b)
    return np.array(hist), err_t, err_qq, err_qr


@pytest.mark.parametrize("ne,no,scale,seed", [(40, 40, 0.5, 1), (96, 96, 0.8, 2), (64, 48, 0.9, 3)])
def test_recurrences_match_classical_gcr(ne, no, scale, seed):
    Ye, Yo, b = system(ne, no, scale, seed)
    steps = 12
    hist, err_t, err_qq, err_qr = persistent_form(Ye, Yo, b, steps)
    info = SolveInfo()
    Dr = lambda v: v - Ye @ (Yo @ v)  # noqa: E731
    gcr(Dr, b, tol=1e-300, restart=steps, maxiter=steps, info=info)
    ref = np.array(info.history[: steps + 1])
    assert len(ref) == steps + 1
    assert np.max(np.abs(hist - ref) / ref) < 1e-10
    assert np.all(np.diff(hist) <= 1e-12 * hist[0]) and hist[-1] < 0.9 * hist[0]  # minimal residual: progress
    assert err_t < 1e-13 and err_qq < 1e-10 and err_qr < 1e-10


def test_pythagoras_fails_without_orthogonal_residual():
    """A planted mistake: taking <q_k, r> from a residual that is not
    orthogonal to the earlier q_j (here: the cycle's start residual) breaks
    the step-by-step agreement, so the check above would catch it."""
    Ye, Yo, b = system(40, 40, 0.5, 1)
    r0 = b.copy()
    r = b.copy()
    t = Yo @ r
    Q, qn = [], []
    hist = [norm(r)]
    for k in range(6):
        q = r - Ye @ t
        dots = [np.vdot(qj, q) for qj in Q]
        qq = np.vdot(q, q).real - sum(abs(d) ** 2 / n for d, n in zip(dots, qn))
        alpha = np.vdot(q, r0) / qq  # wrong residual
        c = [d / n for d, n in zip(dots, qn)]
        qk = q - sum((cj * qj for cj, qj in zip(c, Q)), np.zeros_like(q))
        r = r - alpha * qk
        t = Yo @ r
        Q.append(qk)
        qn.append(qq)
        hist.append(norm(r))
    info = SolveInfo()
    gcr(lambda v: v - Ye @ (Yo @ v), b, tol=1e-300, restart=6, maxiter=6, info=info)
    ref = np.array(info.history[:7])
    assert np.max(np.abs(np.array(hist) - ref) / ref) > 1e-6


def persistent_form_f32(Ye, Yo, b, steps):
    """The same recurrences with every stored vector (q_k, z_k, T_k, y, r, t)
    rounded to complex64 after each update and the hops taken in complex64,
    as the FP32 kernel stores them; the sums behind alpha and the Gram-Schmidt
    coefficients are formed in FP64 from the stored values.  Returns the
    residual norms of the recurrence, the smallest Pythagorean ||q_k||^2
    relative to the direct ||q||^2, and the final true residual."""
    r32 = lambda v: v.astype(np.complex64)  # noqa: E731
    Ye32, Yo32 = r32(Ye), r32(Yo)
    r = r32(b)
    y = np.zeros_like(r)
    t = r32(Yo32 @ r)
    Q, Z, T, qn = [], [], [], []
    hist = [norm(r.astype(np.complex128))]
    worst_ratio = np.inf
    for k in range(steps):
        q = r32(r - Ye32 @ t)
        q64 = q.astype(np.complex128)
        dots = [np.vdot(qj.astype(np.complex128), q64) for qj in Q]
        qq_direct = np.vdot(q64, q64).real
        qq = qq_direct - sum(abs(d) ** 2 / n for d, n in zip(dots, qn))
        worst_ratio = min(worst_ratio, qq / qq_direct)
        assert qq > 0.0  # no false breakdown from cancellation
        alpha = np.vdot(q64, r.astype(np.complex128)) / qq
        c = [d / n for d, n in zip(dots, qn)]
        qk = r32(q64 - sum((cj * qj.astype(np.complex128) for cj, qj in zip(c, Q)), np.zeros_like(q64)))
        zk = r32(r.astype(np.complex128) - sum((cj * zj.astype(np.complex128) for cj, zj in zip(c, Z)),
                                               np.zeros_like(q64)))
        Tk = r32((Yo32 @ q).astype(np.complex128) - sum((cj * Tj.astype(np.complex128) for cj, Tj in zip(c, T)),
                                                        np.zeros(t.shape, np.complex128)))
        y = r32(y.astype(np.complex128) + alpha * zk.astype(np.complex128))
        r = r32(r.astype(np.complex128) - alpha * qk.astype(np.complex128))
        t = r32(t.astype(np.complex128) - alpha * Tk.astype(np.complex128))
        Q.append(qk)
        Z.append(zk)
        T.append(Tk)
        qn.append(qq)
        hist.append(norm(r.astype(np.complex128)))
    y64 = y.astype(np.complex128)
    true_res = norm(b - (y64 - Ye @ (Yo @ y64)))
    return np.array(hist), worst_ratio, true_res


@pytest.mark.parametrize("ne,no,scale,seed", [(96, 96, 0.8, 2), (64, 48, 0.9, 3), (200, 200, 0.95, 4)])
def test_recurrences_in_fp32_storage_track_classical_gcr(ne, no, scale, seed):
    """FP32 storage: the Pythagorean ||q_k||^2 stays positive and the residual
    history tracks FP64 classical GCR down to the cycle's coarse tolerance
    (0.05-0.3 of ||b_r||); the recurred residual agrees with the true one to
    FP32 rounding of the cycle's start scale."""
    Ye, Yo, b = system(ne, no, scale, seed)
    steps = 16
    hist, worst_ratio, true_res = persistent_form_f32(Ye, Yo, b, steps)
    info = SolveInfo()
    gcr(lambda v: v - Ye @ (Yo @ v), b, tol=1e-300, restart=steps, maxiter=steps, info=info)
    ref = np.array(info.history[: steps + 1])
    above = ref >= 0.05 * ref[0]  # the part of the history a coarse solve at tol >= 0.05 uses
    assert above.sum() >= 3
    assert np.max(np.abs(hist[above] - ref[above]) / ref[above]) < 1e-4
    assert worst_ratio > 1e-6
    assert abs(true_res - hist[-1]) < 1e-5 * hist[0]
