"""Plain FP64 CPU oracle for the tanTRG one-site tangent-space sweep.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the C-ABI library and its
Python binding) imports, links or calls anything in this package; only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark do.

The oracle is written directly from the paper (arXiv:2212.11973):

* ``lattice``  - cylinder / open-square lattices and the quasi-1D snake order
                 (main text, Hubbard-model paragraph and Fig. 1a).
* ``ed``       - sector-blocked exact diagonalisation of Eq. (3) in the Fock
                 basis, the U=0 closed form, and the "same-ODE" reference
                 values for a linear start rho0 = 1 - beta0*H.
* ``mpo``      - finite-state-machine MPO of Eq. (3) and the super-MPS form
                 of rho0 = 1 - beta0*H (Choi map, SM Sec. II.A).
* ``tdvp``     - one-site TDVP sweep (SM Sec. II.F steps 1-7, Eq. S-local
                 split as in SM Sec. II.E), Lanczos exponential (SM Sec. II.H),
                 environments and effective Hamiltonians (SM Fig. optimalB),
                 bilayer observables (SM Sec. II.A).
* ``charges``  - U(1)xU(1) bond-sector bookkeeping used to pad rho0 to a
                 target bond dimension, and a SplitMix64 counter generator for
                 the padding noise.

Everything is float64 NumPy; library primitives (matmul/tensordot, QR, eigh)
serve as single steps.  No blocking, fusion or reordering beyond the paper's
own contraction order.
"""
