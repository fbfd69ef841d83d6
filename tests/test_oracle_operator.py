"""Pins of the oracle's Wilson-clover operator (CPU only).

Each test checks the oracle against something fixed independently of its
own code: the Clifford algebra, the free-field momentum-space symbol, an
FFT solve at U = 1, the abelian closed form of the clover leaves, gamma5
hermiticity, gauge covariance, and the red-black identities of Eqs.(2)-(4).
"""
import numpy as np
import pytest

import inputs
from oracle.dirac import WilsonClover, gauge_transform_links, field_strength
from oracle.krylov import gcr, bicgstab, norm, SolveInfo
from oracle.lattice import GAMMA, GAMMA5, Lattice, sigma_munu


def unit_links(dims):
    V = inputs.volume(dims)
    return np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()


def rand_spinor(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def symbol(p, m0):
    """Free-field D(p) = m0 + sum(1 - cos p) + i sum gamma_mu sin p_mu (4x4)."""
    return (m0 + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * sum(
        GAMMA[mu] * np.sin(p[mu]) for mu in range(4))


# --------------------------------------------------------------------------
def test_gamma_basis():
    for m in range(4):
        assert np.allclose(GAMMA[m], GAMMA[m].conj().T)
        for n in range(4):
            ac = GAMMA[m] @ GAMMA[n] + GAMMA[n] @ GAMMA[m]
            assert np.allclose(ac, 2 * (m == n) * np.eye(4))
    assert np.allclose(GAMMA5, np.diag([1, 1, -1, -1]))
    for m in range(4):
        for n in range(4):
            s = sigma_munu(m, n)
            assert np.allclose(s, s.conj().T)
            assert np.allclose(s @ GAMMA5, GAMMA5 @ s)   # block diagonal in chirality


@pytest.mark.parametrize("t_bc", [-1, 1])
def test_free_field_plane_waves(t_bc):
    dims = (4, 4, 4, 6)
    m0 = -0.2
    op = WilsonClover(dims, unit_links(dims), m0, csw=1.0, t_bc=t_bc)
    lat = op.lat
    rng = np.random.default_rng(1)
    shift = 0.5 if t_bc == -1 else 0.0
    for _ in range(6):
        n = [rng.integers(0, L) for L in dims]
        p = np.array([2 * np.pi * n[0] / dims[0], 2 * np.pi * n[1] / dims[1],
                      2 * np.pi * n[2] / dims[2], 2 * np.pi * (n[3] + shift) / dims[3]])
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * lat.coords @ p)
        psi = phase[:, None, None] * u[None]
        got = op.apply_D(psi)
        want = phase[:, None, None] * (symbol(p, m0) @ u)[None]
        assert np.abs(got - want).max() < 1e-13


def test_free_field_dense_spectrum():
    dims = (4, 2, 2, 4)
    m0 = -0.2
    op = WilsonClover(dims, unit_links(dims), m0, csw=1.0)
    ev = np.linalg.eigvals(op.dense(op.apply_D))
    want = []
    for n0 in range(dims[0]):
        for n1 in range(dims[1]):
            for n2 in range(dims[2]):
                for n3 in range(dims[3]):
                    p = 2 * np.pi * np.array([n0 / dims[0], n1 / dims[1], n2 / dims[2],
                                              (n3 + 0.5) / dims[3]])
                    a = m0 + np.sum(1 - np.cos(p))
                    s = np.sqrt(np.sum(np.sin(p) ** 2))
                    want += [a + 1j * s] * 6 + [a - 1j * s] * 6
    want = np.array(want)
    ev = list(ev)
    for w in want:
        k = int(np.argmin(np.abs(np.array(ev) - w)))
        assert abs(ev[k] - w) < 1e-10
        ev.pop(k)


def test_free_field_fft_solve():
    """x = FFT^-1[D(p)^-1 FFT(b)] with antiperiodic time, vs the oracle solvers."""
    dims = (4, 4, 4, 8)
    m0 = -0.2
    op = WilsonClover(dims, unit_links(dims), m0, csw=1.0)
    Lx, Ly, Lz, Lt = dims
    b = inputs.z2_source(dims, 7)                       # [t][z][y][x][s][c]
    t = np.arange(Lt)[:, None, None, None, None, None]
    bt = np.fft.fftn(b * np.exp(-1j * np.pi * t / Lt), axes=(0, 1, 2, 3))
    kx = 2 * np.pi * np.fft.fftfreq(Lx) * 1.0
    xt = np.zeros_like(bt)
    for it in range(Lt):
        for iz in range(Lz):
            for iy in range(Ly):
                for ix in range(Lx):
                    p = np.array([2 * np.pi * ix / Lx, 2 * np.pi * iy / Ly,
                                  2 * np.pi * iz / Lz, 2 * np.pi * (it + 0.5) / Lt])
                    xt[it, iz, iy, ix] = np.linalg.solve(symbol(p, m0), bt[it, iz, iy, ix])
    del kx
    x_exact = np.fft.ifftn(xt, axes=(0, 1, 2, 3)) * np.exp(1j * np.pi * t / Lt)
    x_exact = x_exact.reshape(op.shape)
    bf = b.reshape(op.shape)
    assert norm(op.apply_D(x_exact) - bf) / norm(bf) < 1e-13
    x = op.reconstruct(gcr(op.apply_Dr, op.reduced_source(bf), tol=1e-12,
                           target_norm=norm(bf), restart=16, maxiter=2000), bf)
    assert norm(x - x_exact) / norm(x_exact) < 1e-10


def test_clover_vanishes_at_unit_links():
    dims = (4, 4, 4, 4)
    op = WilsonClover(dims, unit_links(dims), 0.1, csw=1.7)
    assert np.abs(op.A - 4.1 * np.eye(12)).max() < 1e-15


def test_clover_abelian_closed_form():
    """U_mu(x) = exp(i eps a_mu(x) T), T = diag(1,-1,0): each leaf is exp(i eps Phi T)
    so Fhat_mu_nu = (i/4) sum_leaves sin(eps Phi_leaf T) exactly."""
    dims = (4, 4, 4, 4)
    lat = Lattice(dims)
    rng = np.random.default_rng(3)
    eps = 0.7
    a = rng.standard_normal((lat.V, 4))
    Tdiag = np.array([1.0, -1.0, 0.0])
    U = np.zeros((lat.V, 4, 3, 3), dtype=np.complex128)
    for mu in range(4):
        U[:, mu] = np.exp(1j * eps * a[:, mu, None] * Tdiag[None, :])[:, :, None] * np.eye(3)
    sites = np.arange(lat.V)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            F = field_strength(lat, U, mu, nu, sites)
            f, g = lat.fwd, lat.bwd
            x = sites
            am, an = a[:, mu], a[:, nu]
            phis = [am[x] + an[f[mu][x]] - am[f[nu][x]] - an[x],
                    an[x] - am[f[nu][g[mu][x]]] - an[g[mu][x]] + am[g[mu][x]],
                    -am[g[mu][x]] - an[g[nu][g[mu][x]]] + am[g[nu][g[mu][x]]] + an[g[nu][x]],
                    -an[g[nu][x]] + am[g[nu][x]] + an[f[mu][g[nu][x]]] - am[x]]
            want = sum(0.25j * np.sin(eps * ph[:, None] * Tdiag[None, :]) for ph in phis)
            got = np.diagonal(F, axis1=1, axis2=2)
            assert np.abs(got - want).max() < 1e-14
            assert np.abs(F - np.einsum("ni,ij->nij", got, np.eye(3))).max() < 1e-15


def test_clover_structure():
    """Hermitian, commutes with gamma5, norm <= 3 csw, covariant field strength."""
    dims = (4, 4, 4, 4)
    U = inputs.gauge_field(dims, 0.9, 11)
    csw = 1.3
    op = WilsonClover(dims, U, 0.0, csw)
    C = op.A - 4.0 * np.eye(12)
    assert np.abs(C - np.conj(np.swapaxes(C, 1, 2))).max() < 1e-14
    G5 = np.kron(GAMMA5, np.eye(3))
    assert np.abs(C @ G5 - G5 @ C).max() < 1e-14
    assert np.linalg.norm(C, ord=2, axis=(1, 2)).max() <= 3 * csw + 1e-12
    assert np.abs(C).max() > 1e-3


def test_gamma5_hermiticity():
    dims = (4, 4, 4, 4)
    U = inputs.gauge_field(dims, 0.5, 12)
    for csw in (0.0, 1.0):
        op = WilsonClover(dims, U, -0.25, csw)
        phi, psi = rand_spinor(op.shape, 1), rand_spinor(op.shape, 2)
        lhs = np.vdot(phi, op.apply_D(psi))
        rhs = np.vdot(op.gamma5(op.apply_D(op.gamma5(phi))), psi)
        assert abs(lhs - rhs) / abs(lhs) < 1e-14
        # D^dag written term by term agrees with gamma5 D gamma5
        assert norm(op.apply_Ddag(phi) - op.gamma5(op.apply_D(op.gamma5(phi)))) < 1e-12 * norm(phi)
        # D_p = D M^-1 is gamma5-hermitian only without the clover term
        lhs = np.vdot(phi, op.gamma5(op.apply_Dp(psi)))
        rhs = np.vdot(op.gamma5(op.apply_Dp(phi)), psi)
        if csw == 0.0:
            assert abs(lhs - rhs) / abs(lhs) < 1e-14
        else:
            assert abs(lhs - rhs) / abs(lhs) > 1e-6


def test_gauge_covariance():
    dims = (4, 4, 4, 4)
    U = inputs.gauge_field(dims, 0.6, 13).reshape(-1, 4, 3, 3)
    op = WilsonClover(dims, U, -0.3, 1.0)
    Om = inputs.random_su3(op.lat.V, 14)
    opg = WilsonClover(dims, gauge_transform_links(op.lat, U, Om), -0.3, 1.0)
    psi = rand_spinor(op.shape, 3)
    Opsi = np.einsum("nab,nsb->nsa", Om, psi)
    assert norm(opg.apply_D(Opsi) - np.einsum("nab,nsb->nsa", Om, op.apply_D(psi))) < 1e-12 * norm(psi)
    b = inputs.z2_source(dims, 5).reshape(op.shape)
    x = gcr(op.apply_D, b, tol=1e-12, restart=20, maxiter=3000)
    xg = gcr(opg.apply_D, np.einsum("nab,nsb->nsa", Om, b), tol=1e-12, restart=20, maxiter=3000)
    assert norm(xg - np.einsum("nab,nsb->nsa", Om, x)) / norm(x) < 1e-9


def test_red_black_identities():
    """Eq.(2): D_p has unit diagonal blocks; Eqs.(3)-(4): the Schur solve plus
    reconstruction is the full solve and leaves an exactly zero odd residual."""
    dims = (4, 2, 2, 4)
    U = inputs.gauge_field(dims, 0.5, 15)
    op = WilsonClover(dims, U, -0.2, 1.0)
    lat = op.lat
    Dp = op.dense(op.apply_Dp)
    ev = np.repeat(lat.parity == 0, 12)
    od = ~ev
    assert np.abs(Dp[np.ix_(ev, ev)] - np.eye(ev.sum())).max() < 1e-14
    assert np.abs(Dp[np.ix_(od, od)] - np.eye(od.sum())).max() < 1e-14
    # spectrum: D_p v = lam v  =>  D_r v_e = lam (2 - lam) v_e
    Dr = op.dense(op.apply_Dr)[np.ix_(ev, ev)]
    lam = np.linalg.eigvals(Dp)
    mapped = list(lam * (2 - lam))
    for mu in np.repeat(np.linalg.eigvals(Dr), 2):
        k = int(np.argmin(np.abs(np.array(mapped) - mu)))
        assert abs(mapped[k] - mu) < 1e-9
        mapped.pop(k)
    # Schur solve + reconstruction == dense solve
    D = op.dense(op.apply_D)
    b = inputs.z2_source(dims, 4).reshape(op.shape)
    x_dense = np.linalg.solve(D, b.reshape(-1)).reshape(op.shape)
    br = op.reduced_source(b)
    ye = np.linalg.solve(Dr, br.reshape(-1)[np.repeat(lat.parity == 0, 12)])
    y = np.zeros(op.shape, dtype=np.complex128)
    y[lat.even] = ye.reshape(-1, 4, 3)
    x = op.reconstruct(y, b)
    assert norm(x - x_dense) / norm(x_dense) < 1e-12
    r = b - op.apply_D(x)
    assert norm(r[lat.odd]) < 1e-13 * norm(b)


def test_Dr_adjoint():
    dims = (4, 4, 2, 4)
    op = WilsonClover(dims, inputs.gauge_field(dims, 0.5, 16), -0.2, 1.0)
    a, c = rand_spinor(op.shape, 7), rand_spinor(op.shape, 8)
    a[op.lat.odd] = 0
    c[op.lat.odd] = 0
    assert abs(np.vdot(a, op.apply_Dr(c)) - np.vdot(op.apply_Dr_dag(a), c)) < 1e-12 * norm(a) * norm(c)


def test_manufactured_solution_bicgstab_and_gcr():
    """b = D x0 (the paper's error-measurement construction): both solvers recover x0."""
    dims = (4, 4, 4, 4)
    op = WilsonClover(dims, inputs.gauge_field(dims, 0.3, 1001), -0.2, 1.0)
    x0 = rand_spinor(op.shape, 9)
    b = op.apply_D(x0)
    br = op.reduced_source(b)
    info = SolveInfo()
    y = bicgstab(op.apply_Dr, br, tol=1e-12, target_norm=norm(b), info=info)
    x = op.reconstruct(y, b)
    assert info.converged
    assert norm(b - op.apply_D(x)) / norm(b) < 1e-11
    assert norm(x - x0) / norm(x0) < 1e-9
    y2 = gcr(op.apply_Dr, br, tol=1e-12, target_norm=norm(b), restart=16, maxiter=2000)
    assert norm(op.reconstruct(y2, b) - x0) / norm(x0) < 1e-9


def test_sampled_sites_match_full():
    dims = (4, 4, 4, 4)
    U = inputs.gauge_field(dims, 0.5, 17)
    op = WilsonClover(dims, U, -0.2, 1.0)
    psi = rand_spinor(op.shape, 10)
    sites = np.array([0, 5, 77, 200, 255])
    full = op.apply_H(psi)
    part = op.apply_H(psi, sites)
    assert np.abs(full[sites] - part[sites]).max() < 1e-15
    from oracle.dirac import site_matrix
    assert np.abs(site_matrix(op.lat, op.U, -0.2, 1.0, sites) - op.A[sites]).max() < 1e-15


def test_input_links_are_su3():
    U = inputs.gauge_field((4, 4, 4, 4), 0.5, 18, ape_sweeps=2).reshape(-1, 3, 3)
    I = np.conj(np.swapaxes(U, 1, 2)) @ U
    assert np.abs(I - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13
