"""Seeded synthetic inputs shared by the oracle-side tests and the HIP path.

This module only draws random numbers and builds gauge fields and sources;
it holds none of the Dirac-operator or multigrid arithmetic.  The paper's
production lattices (anisotropic clover ensembles, Results section) are not
available, so every workload is replaced by a seeded synthetic stand-in of
the same shape:

* links ``U = exp(i*eps*H)``, ``H = sum_a h_a lambda_a / 2`` with
  ``h_a ~ N(0,1)`` iid (Gell-Mann basis), exponentiated through ``eigh`` so
  that every link is exactly SU(3) to rounding;
* optional APE-style smoothing ``U' = Proj_SU3[(1-alpha) U + alpha/6 * sum of
  the 6 staples]`` (Jacobi update of all four directions per sweep), where
  ``Proj_SU3`` is the polar projection ``X (X^dag X)^{-1/2}`` followed by a
  division by the principal cube root of the determinant;
* Z2 sources (real +-1 per site, spin and colour) and complex Gaussian
  sources.

Canonical layouts (interleaved complex128):
  gauge  ``[Lt][Lz][Ly][Lx][4 mu][3][3]``  (mu = x, y, z, t)
  spinor ``[Lt][Lz][Ly][Lx][4 spin][3 colour]``
The flat site index is ``((t*Lz + z)*Ly + y)*Lx + x``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume", "gell_mann", "random_links", "project_su3", "ape_smear",
    "gauge_field", "z2_source", "gaussian_source", "random_su3",
    "CONFIGS", "config",
]


def volume(dims):
    v = 1
    for d in dims:
        v *= int(d)
    return v


def _shape(dims):
    lx, ly, lz, lt = (int(d) for d in dims)
    return (lt, lz, ly, lx)


def gell_mann():
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j
    l[1][1, 0] = 1j
    l[2][0, 0] = 1
    l[2][1, 1] = -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j
    l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j
    l[6][2, 1] = 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


def _expi_hermitian(H, eps):
    """exp(i*eps*H) for a stack of Hermitian 3x3 matrices, via eigh."""
    w, Q = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return (Q * ph[..., None, :]) @ np.conj(np.swapaxes(Q, -1, -2))


def random_links(dims, eps, seed):
    """Links exp(i*eps*H), H random traceless Hermitian Gaussian.

    Draw order: canonical site order, then mu, then the 8 coefficients.
    Returns complex128 of shape [Lt][Lz][Ly][Lx][4][3][3].
    """
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    h = rng.standard_normal((V, 4, 8))
    H = np.einsum("vma,aij->vmij", h, gell_mann() * 0.5)
    U = _expi_hermitian(H, eps)
    return U.reshape(_shape(dims) + (4, 3, 3))


def project_su3(X):
    """Polar projection onto U(3), then divide out det^{1/3} (principal root)."""
    XhX = np.conj(np.swapaxes(X, -1, -2)) @ X
    w, Q = np.linalg.eigh(XhX)
    inv_sqrt = (Q * (1.0 / np.sqrt(w))[..., None, :]) @ np.conj(np.swapaxes(Q, -1, -2))
    W = X @ inv_sqrt
    det = np.linalg.det(W)
    root = np.exp(1j * np.angle(det) / 3.0)
    return W / root[..., None, None]


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def ape_smear(U, alpha=0.5, sweeps=5):
    """APE-style smoothing on periodic boundaries (Jacobi update, all mu)."""
    U = np.array(U, dtype=np.complex128, copy=True)
    axis = {0: 3, 1: 2, 2: 1, 3: 0}  # lattice direction -> array axis
    for _ in range(sweeps):
        new = np.empty_like(U)
        for mu in range(4):
            am = axis[mu]
            Umu = U[..., mu, :, :]
            staple = np.zeros_like(Umu)
            Umu_xpm = np.roll(Umu, -1, axis=am)
            for nu in range(4):
                if nu == mu:
                    continue
                an = axis[nu]
                Unu = U[..., nu, :, :]
                # upper: U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
                Unu_xpm = np.roll(Unu, -1, axis=am)
                Umu_xpn = np.roll(Umu, -1, axis=an)
                staple += Unu @ Umu_xpn @ _dag(Unu_xpm)
                # lower: U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu)
                Unu_xmn = np.roll(Unu, 1, axis=an)
                Umu_xmn = np.roll(Umu, 1, axis=an)
                Unu_xmn_pm = np.roll(Unu_xmn, -1, axis=am)
                staple += _dag(Unu_xmn) @ Umu_xmn @ Unu_xmn_pm
            del Umu_xpm
            new[..., mu, :, :] = project_su3((1.0 - alpha) * Umu + (alpha / 6.0) * staple)
        U = new
    return U


def gauge_field(dims, eps, seed, ape_sweeps=0, ape_alpha=0.5):
    U = random_links(dims, eps, seed)
    if ape_sweeps:
        U = ape_smear(U, ape_alpha, ape_sweeps)
    return U


def z2_source(dims, seed):
    """Real +-1 (probability 1/2 each) per site, spin and colour, as complex128."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = rng.integers(0, 2, size=_shape(dims) + (4, 3)) * 2 - 1
    return s.astype(np.complex128)


def gaussian_source(dims, seed):
    """Complex Gaussian source, re and im ~ N(0,1) iid."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal(_shape(dims) + (4, 3, 2))
    return g[..., 0] + 1j * g[..., 1]


def random_su3(n, seed):
    """n Haar-distributed SU(3) matrices (QR of complex Gaussians, phase-fixed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Z = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    return Q / np.exp(1j * np.angle(det) / 3.0)[:, None, None]


# Synthetic workloads.  Gauge seed 1000+i, source seed 2000+100*i+rhs,
# setup seed 3000+i for workload i (1-based).
CONFIGS = {
    "c1_4x4x4x4": dict(index=1, dims=(4, 4, 4, 4), eps=0.3, ape=0, csw=1.0,
                       m0=[-0.2], blocks=[(2, 2, 2, 2)], nvec=[8], nrhs=1,
                       tol=1e-10),
    "c2_16x16x16x32": dict(index=2, dims=(16, 16, 16, 32), eps=0.5, ape=5,
                           csw=1.0, m0=[-0.15, -0.25, -0.30],
                           blocks=[(4, 4, 4, 4)], nvec=[24], nrhs=1, tol=1e-10),
    "c3_24x24x24x64": dict(index=3, dims=(24, 24, 24, 64), eps=0.5, ape=5,
                           csw=1.0, m0=[-0.25], blocks=[(4, 4, 4, 4)],
                           nvec=[24], nrhs=12, tol=1e-10),
    "c4_8x8x8x8": dict(index=4, dims=(8, 8, 8, 8), eps=0.5, ape=5, csw=1.0,
                       m0=[-0.25], blocks=[(4, 4, 4, 4)], nvec=[24], nrhs=1,
                       tol=1e-10),
    "c5_16x16x16x32": dict(index=5, dims=(16, 16, 16, 32), eps=0.5, ape=5,
                           csw=1.0, m0=[-0.28],
                           blocks=[(4, 4, 4, 4), (2, 2, 2, 2)], nvec=[24, 32],
                           nrhs=4, tol=1e-10),
}


def config(name):
    c = dict(CONFIGS[name])
    i = c["index"]
    c["gauge_seed"] = 1000 + i
    c["source_seeds"] = [2000 + 100 * i + r for r in range(c["nrhs"])]
    c["setup_seed"] = 3000 + i
    return c
