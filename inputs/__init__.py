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

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

# Per-site work (3x3 eigendecompositions, products) runs over chunks of the
# leading axis in a thread pool: NumPy's linear-algebra loops release the
# GIL, and every matrix is computed on its own, so the chunking leaves every
# bit of the result unchanged.
_THREADS = max(1, min(16, os.cpu_count() or 1))


def _chunked(fn, *arrays):
    """fn(*chunks) over chunks of axis 0 of the arrays, results concatenated."""
    n = arrays[0].shape[0]
    k = min(_THREADS, max(1, n // 4096))
    if k <= 1:
        return fn(*arrays)
    edges = np.linspace(0, n, k + 1).astype(int)
    with ThreadPoolExecutor(k) as ex:
        parts = list(ex.map(lambda i: fn(*(a[edges[i]:edges[i + 1]] for a in arrays)), range(k)))
    return np.concatenate(parts, axis=0)

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
    def one(Hc):
        w, Q = np.linalg.eigh(Hc)
        ph = np.exp(1j * eps * w)
        return (Q * ph[..., None, :]) @ np.conj(np.swapaxes(Q, -1, -2))
    return _chunked(one, H)


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
    return _chunked(_project_su3, X)


def _project_su3(X):
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
                staple += _chunked(lambda a, b, c: a @ b @ _dag(c), Unu, Umu_xpn, Unu_xpm)
                # lower: U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu)
                Unu_xmn = np.roll(Unu, 1, axis=an)
                Umu_xmn = np.roll(Umu, 1, axis=an)
                Unu_xmn_pm = np.roll(Unu_xmn, -1, axis=am)
                staple += _chunked(lambda a, b, c: _dag(a) @ b @ c, Unu_xmn, Umu_xmn, Unu_xmn_pm)
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


# ----------------------------------------------------------------------------
# The same recipe with elementwise torch operations (any device).  Lattices of
# a few million links take minutes through NumPy's per-matrix loops; this
# version runs the identical draws through whole-array arithmetic on a GPU in
# seconds.  It agrees with gauge_field to rounding (a CPU test checks it), but
# not bit for bit: every consumer of a field takes it from one of the two.
# ----------------------------------------------------------------------------
def _t_mm(A, B):
    """Stacked 3x3 products by broadcasting (no batched-GEMM library call)."""
    return (A[..., :, :, None] * B[..., None, :, :]).sum(-2)


def _t_dag(A):
    return A.conj().transpose(-1, -2)


def _t_det(A):
    return (A[..., 0, 0] * (A[..., 1, 1] * A[..., 2, 2] - A[..., 1, 2] * A[..., 2, 1])
            - A[..., 0, 1] * (A[..., 1, 0] * A[..., 2, 2] - A[..., 1, 2] * A[..., 2, 0])
            + A[..., 0, 2] * (A[..., 1, 0] * A[..., 2, 1] - A[..., 1, 1] * A[..., 2, 0]))


def _t_inv(A):
    """3x3 inverse from the adjugate."""
    import torch
    c = torch.empty_like(A)
    for i in range(3):
        for j in range(3):
            r = [k for k in range(3) if k != j]
            s = [k for k in range(3) if k != i]
            minor = A[..., r[0], s[0]] * A[..., r[1], s[1]] - A[..., r[0], s[1]] * A[..., r[1], s[0]]
            c[..., i, j] = minor if (i + j) % 2 == 0 else -minor
    return c / _t_det(A)[..., None, None]


def _t_project_su3(X, iters=30):
    """Polar factor by the Newton iteration W <- (W + W^-dag)/2 (converged when
    the update stops changing W), then divide out det^{1/3} (principal root)."""
    import torch
    W = X
    for _ in range(iters):
        Wn = 0.5 * (W + _t_dag(_t_inv(W)))
        done = bool((Wn - W).abs().max() <= 4e-16)
        W = Wn
        if done:
            break
    root = torch.exp(1j * torch.angle(_t_det(W)) / 3.0)
    return W / root[..., None, None]


def _t_expi(H, eps, terms=30):
    """exp(i eps H) by its Taylor series (|eps H| is O(1) here), then projected
    onto SU(3) so that unitarity holds to rounding."""
    import torch
    A = 1j * eps * H
    term = torch.eye(3, dtype=H.dtype, device=H.device).expand_as(H).clone()
    out = term.clone()
    for k in range(1, terms):
        term = _t_mm(term, A) / k
        out = out + term
    return _t_project_su3(out)


def gauge_field_torch(dims, eps, seed, ape_sweeps=0, ape_alpha=0.5, device="cpu"):
    """gauge_field's recipe (the same PCG64 draws) as a complex128 torch tensor
    [Lt][Lz][Ly][Lx][4][3][3] on `device`."""
    import torch
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    h = torch.from_numpy(rng.standard_normal((V, 4, 8))).to(device)
    gm = torch.from_numpy(gell_mann() * 0.5).to(device)
    H = (h.to(torch.complex128)[..., :, None, None] * gm).sum(-3)
    U = _t_expi(H, eps).reshape(_shape(dims) + (4, 3, 3))
    axis = {0: 3, 1: 2, 2: 1, 3: 0}
    for _ in range(ape_sweeps):
        new = torch.empty_like(U)
        for mu in range(4):
            am = axis[mu]
            Umu = U[..., mu, :, :]
            staple = torch.zeros_like(Umu)
            for nu in range(4):
                if nu == mu:
                    continue
                an = axis[nu]
                Unu = U[..., nu, :, :]
                staple += _t_mm(_t_mm(Unu, torch.roll(Umu, -1, dims=an)), _t_dag(torch.roll(Unu, -1, dims=am)))
                Unu_xmn = torch.roll(Unu, 1, dims=an)
                staple += _t_mm(_t_mm(_t_dag(Unu_xmn), torch.roll(Umu, 1, dims=an)), torch.roll(Unu_xmn, -1, dims=am))
            new[..., mu, :, :] = _t_project_su3((1.0 - ape_alpha) * Umu + (ape_alpha / 6.0) * staple)
        U = new
    return U
