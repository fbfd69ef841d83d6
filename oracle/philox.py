"""Philox4x32-10 counter-based generator (oracle; test infrastructure only).

Definition from Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3" (SC'11): a 4x32-bit counter and a 2x32-bit key; each of the
10 rounds maps (c0,c1,c2,c3) to
    (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57, and the key is bumped by the Weyl
constants (0x9E3779B9, 0xBB67AE85) before every round after the first.

The multigrid setup draws its random start vectors from this generator so
that any implementation of the same published definition reproduces them:
entry n (= site*ncomp + component) of vector k on level l uses counter
(n mod 2^32, n div 2^32, k, l) and key (seed mod 2^32, seed div 2^32); the
first two output words u0, u1 give uniforms (w + 1/2) / 2^32 and a complex
Gaussian by Box-Muller:  sqrt(-2 ln u0) * exp(2 pi i u1).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """ctr: [..., 4] uint32-valued, key: [..., 2]; returns [..., 4] uint32."""
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = (ctr[..., i] & MASK for i in range(4))
    k0, k1 = key[..., 0] & MASK, key[..., 1] & MASK
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> S32, p0 & MASK
        hi1, lo1 = p1 >> S32, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def gaussian_vector(seed, vec, level, n):
    """n complex Gaussians for start vector `vec` on level `level`."""
    idx = np.arange(n, dtype=np.uint64)
    ctr = np.stack([idx & MASK, idx >> S32,
                    np.full(n, vec, dtype=np.uint64),
                    np.full(n, level, dtype=np.uint64)], axis=-1)
    seed = int(seed)
    key = np.broadcast_to(np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF],
                                   dtype=np.uint64), (n, 2))
    w = philox4x32_10(ctr, key).astype(np.float64)
    u0 = (w[:, 0] + 0.5) / 4294967296.0
    u1 = (w[:, 1] + 0.5) / 4294967296.0
    return np.sqrt(-2.0 * np.log(u0)) * np.exp(2j * np.pi * u1)
