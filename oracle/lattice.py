"""Lattice geometry and Dirac matrices (oracle; test infrastructure only).

Conventions (the paper does not fix them; these are the readings used):
* directions mu = 0,1,2,3 are x, y, z, t; flat site index
  ((t*Lz + z)*Ly + y)*Lx + x;
* parity (x+y+z+t) mod 2, even sites have parity 0 (red-black paragraph);
* chiral gamma basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] for
  k = 1,2,3 and gamma_4 = [[0, 1], [1, 0]], so gamma5 = gamma1 gamma2 gamma3
  gamma4 = diag(1, 1, -1, -1); spins {0,1} have chirality +1, {2,3} -1;
* spinor component index = spin*3 + colour;
* fermion boundary: periodic in space, antiperiodic in time by default.
"""
import numpy as np

SIGMA = np.array([[[0, 1], [1, 0]],
                  [[0, -1j], [1j, 0]],
                  [[1, 0], [0, -1]]], dtype=np.complex128)


def gamma_matrices():
    """Return (gamma[0..3], gamma5) in the chiral basis."""
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    Z = np.zeros((2, 2))
    I2 = np.eye(2)
    for k in range(3):
        g[k] = np.block([[Z, -1j * SIGMA[k]], [1j * SIGMA[k], Z]])
    g[3] = np.block([[Z, I2], [I2, Z]])
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    return g, g5


GAMMA, GAMMA5 = gamma_matrices()


def sigma_munu(mu, nu):
    """sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu]."""
    return 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])


class Lattice:
    """Periodic 4D lattice with neighbour tables and boundary phases."""

    def __init__(self, dims, t_bc=-1):
        self.dims = tuple(int(d) for d in dims)
        Lx, Ly, Lz, Lt = self.dims
        self.V = Lx * Ly * Lz * Lt
        self.t_bc = t_bc
        idx = np.arange(self.V)
        x = idx % Lx
        y = (idx // Lx) % Ly
        z = (idx // (Lx * Ly)) % Lz
        t = idx // (Lx * Ly * Lz)
        self.coords = np.stack([x, y, z, t], axis=1)
        self.parity = (x + y + z + t) % 2
        self.even = np.nonzero(self.parity == 0)[0]
        self.odd = np.nonzero(self.parity == 1)[0]
        self.fwd = np.empty((4, self.V), dtype=np.int64)
        self.bwd = np.empty((4, self.V), dtype=np.int64)
        self.fwd_phase = np.ones((4, self.V))
        self.bwd_phase = np.ones((4, self.V))
        for mu in range(4):
            e = np.zeros(4, dtype=np.int64)
            e[mu] = 1
            self.fwd[mu] = self.index((self.coords + e) % self.dims)
            self.bwd[mu] = self.index((self.coords - e) % self.dims)
        # antiperiodic time: a hop that wraps around t picks up t_bc
        self.fwd_phase[3][t == Lt - 1] = t_bc
        self.bwd_phase[3][t == 0] = t_bc

    def index(self, c):
        Lx, Ly, Lz, _ = self.dims
        c = np.asarray(c)
        return ((c[..., 3] * Lz + c[..., 2]) * Ly + c[..., 1]) * Lx + c[..., 0]

    def mask(self, parity):
        return (self.parity == parity).astype(np.float64)
