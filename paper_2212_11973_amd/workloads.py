"""Seeded synthetic workloads (inputs only; no arithmetic of the method).

Every workload is a model Hamiltonian of the paper's kind (Eq. 3 on the
lattices of its main text), so no dataset is involved; the only random
inputs are the dense tensors of the effective-Hamiltonian microbenchmark,
drawn i.i.d. N(0, 1) in float64 from ``numpy.random.default_rng(20221223 + D)``
in the order L, W, A, R.
"""
import numpy as np

CHAIN, CYLINDER, OPEN_SQUARE = 0, 1, 2

# name -> model and run parameters
MODELS = {
    # Hubbard chain L=4, OBC, t=1, U=4, mu=0; untruncated bonds [1,16,256,16,1];
    # rho0 = 1 - 0.01 H, 399 sweeps of d_beta = 0.01 to beta = 4, Krylov 8.
    "chain4": dict(W=1, L=4, geometry=CHAIN, t=1.0, U=4.0, mu=0.0, D=256,
                   beta0=0.01, dbeta=0.01, nsteps=399, krylov=8),
    # 4x16 cylinder, U=8, mu=1.5, U(1)xU(1) bond D=2000, linear stage d_beta=0.05.
    "cl4x16": dict(W=4, L=16, geometry=CYLINDER, t=1.0, U=8.0, mu=1.5, D=2000,
                   beta0=0.05 * 2.0 ** -12, dbeta=0.05, krylov=8),
    # 6x12 cylinder, U=8, bond D=1500; mu scan 4 -> 1 in 8 steps.
    "cl6x12": dict(W=6, L=12, geometry=CYLINDER, t=1.0, U=8.0, mu=4.0, D=1500,
                   beta0=0.05 * 2.0 ** -12, dbeta=0.05, krylov=8),
    # 10x10 open square and 8x16 cylinder at half filling, D=4000.
    "os10x10": dict(W=10, L=10, geometry=OPEN_SQUARE, t=1.0, U=8.0, mu=4.0,
                    D=4000, beta0=0.05 * 2.0 ** -12, dbeta=0.05, krylov=8),
    "cl8x16": dict(W=8, L=16, geometry=CYLINDER, t=1.0, U=8.0, mu=4.0,
                   D=4000, beta0=0.05 * 2.0 ** -12, dbeta=0.05, krylov=8),
}

MU_SCAN = [4.0 - 3.0 * k / 7.0 for k in range(8)]


def heff_inputs(D, DH=18, seed_base=20221223):
    """Dense L[D,DH,D], W[DH,4,4,DH], A[D,4,4,D], R[D,DH,D] (float64)."""
    rng = np.random.default_rng(seed_base + D)
    L = rng.standard_normal((D, DH, D))
    W = rng.standard_normal((DH, 4, 4, DH))
    A = rng.standard_normal((D, 4, 4, D))
    R = rng.standard_normal((D, DH, D))
    return L, W, A, R


def heff2_inputs(Dl, Dr, DH, seed):
    """Two-site operands L[Dl,DH,Dl], W1, W2 [DH,4,4,DH], C[Dl,4,4,4,4,Dr], R[Dr,DH,Dr]."""
    rng = np.random.default_rng(seed)
    L = rng.standard_normal((Dl, DH, Dl))
    W1 = rng.standard_normal((DH, 4, 4, DH))
    W2 = rng.standard_normal((DH, 4, 4, DH))
    C = rng.standard_normal((Dl, 4, 4, 4, 4, Dr))
    R = rng.standard_normal((Dr, DH, Dr))
    return L, W1, W2, C, R


def heff_inputs_rect(Dl, Dr, DH, seed):
    """Rectangular variant L[Dl,DH,Dl], W, A[Dl,4,4,Dr], R[Dr,DH,Dr]."""
    rng = np.random.default_rng(seed)
    L = rng.standard_normal((Dl, DH, Dl))
    W = rng.standard_normal((DH, 4, 4, DH))
    A = rng.standard_normal((Dl, 4, 4, Dr))
    R = rng.standard_normal((Dr, DH, Dr))
    return L, W, A, R
