"""Plain FP64 CPU oracle for the Wilson-clover multigrid hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
executes this package; it exists so that the tests, the smoke check and the
CPU leg of the benchmark can compare the HIP path against a slow, obviously
correct implementation written directly from the paper (Osborn et al.,
"Multigrid solver for clover fermions", Lattice 2010):

* ``lattice``   geometry, checkerboarding, neighbour tables, gamma matrices;
* ``dirac``     Eq.(1) operator with the clover term, the red-black split of
                Eq.(2), D_p, the reduced operator D_r and source b_r of
                Eqs.(3)-(4), and the reconstruction of x_e, x_o;
* ``krylov``    flexible GCR, BiCGStab and MR in plain NumPy;
* ``multigrid`` the inverse-iteration setup (section 3), the block x
                chirality split of P, R = P^dag gamma5, the coarse operator
                R D_p P, coarse red-black solve and the recursive GCR cycle
                ("Implementation" paragraph);
* ``philox``    Philox4x32-10 counter-based generator (Salmon et al., SC'11)
                for the random start vectors of the setup;
* ``force``     the adjoint solve and gauge-link gradient of ||D^-1 eta||^2.

Every floating-point result is FP64.  The null vectors produced by the setup
are a heuristic (random start + inverse iteration) and are parity unpinned:
only their invariants (orthonormality, Rayleigh-quotient settling) are
checked; P, R and the coarse operator are pinned given imported vectors.
"""
