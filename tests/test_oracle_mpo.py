"""Pins of the oracle MPO: contracted to a dense matrix it must equal the
Fock-space Hamiltonian of Eq. (3) (independent construction), rho0 must be
1 - beta0 H, and every W entry must conserve U(1)xU(1) charge."""

import numpy as np
import pytest

from oracle import charges, ed, lattice, mpo


CASES = [(1, 4, 0, 1.0, 4.0, 0.0), (2, 2, 2, 1.0, 8.0, 1.3), (3, 2, 1, 0.7, 0.0, -0.5),
         (2, 3, 2, 1.0, 8.0, 4.0), (1, 5, 0, 1.3, 2.0, 0.4)]


@pytest.mark.parametrize("W,L,geo,t,U,mu", CASES)
def test_mpo_equals_fock_hamiltonian(W, L, geo, t, U, mu):
    Hd = ed.Hubbard(W, L, geo, t, U, mu).dense_hamiltonian()
    m = mpo.HubbardMPO(W, L, geo, t, U, mu)
    assert np.abs(mpo.mpo_to_dense(m.mpo_for_env()) - Hd).max() < 1e-13
    b0 = 0.013
    r0 = mpo.mpo_to_dense(m.rho0_tensors(b0))
    assert np.abs(r0 - (np.eye(Hd.shape[0]) - b0 * Hd)).max() < 1e-13


@pytest.mark.parametrize("W,L,geo,t,U,mu", CASES)
def test_mpo_charge_conservation(W, L, geo, t, U, mu):
    m = mpo.HubbardMPO(W, L, geo, t, U, mu)
    for k, Wk in enumerate(m.W):
        qa, qb = m.bond_charges(k), m.bond_charges(k + 1)
        for a, so, si, b in zip(*np.nonzero(Wk)):
            qo, qi = mpo.local_charge(so), mpo.local_charge(si)
            assert (qa[a][0] + qo[0] - qi[0], qa[a][1] + qo[1] - qi[1]) == qb[b]


@pytest.mark.parametrize("W", [3, 4, 6, 8])
def test_mpo_bulk_bond_is_4w_plus_2(W):
    """The construction's own count (the paper prints no D_H): on a snake
    cylinder of width W, W sites behind a bulk bond have a partner ahead, each
    with one open strand per operator type (4), plus the start and done
    states."""
    m = mpo.HubbardMPO(W, 6, lattice.CYLINDER, 1.0, 8.0, 0.0)
    dims = [len(s) for s in m.states]
    assert max(dims) == 4 * W + 2
    assert dims[m.N // 2] == 4 * W + 2


@pytest.mark.parametrize("W,L,geo", [(4, 4, 1), (3, 4, 2), (4, 16, 1)])
def test_rho0_fits_maximal_sectors(W, L, geo):
    m = mpo.HubbardMPO(W, L, geo, 1.0, 8.0, 1.5)
    N = m.N
    for k in range(1, N):
        cnt = {}
        for q in m.bond_charges(k):
            cnt[q] = cnt.get(q, 0) + 1
        for q, c in cnt.items():
            assert c <= charges._dmax(N, k, q)


def test_sector_allocation_properties():
    m = mpo.HubbardMPO(4, 4, 1, 1.0, 8.0, 1.5)
    N = m.N
    q0 = [m.bond_charges(k) for k in range(N)] + [[(0, 0)]]
    for D in (40, 64, 200):
        lay = charges.bond_layouts(q0, N, D, True)
        for k in range(N + 1):
            d = {}
            for q in lay[k].charges:
                d[q] = d.get(q, 0) + 1
            # sorted sectors, every sector within its maximal size
            assert lay[k].charges == sorted(lay[k].charges)
            for q, v in d.items():
                assert v <= (charges._dmax(N, k, q) if 0 < k < N else 1)
            if 0 < k < N:
                assert lay[k].dim <= D + len(q0[k])
        # maximal sizes are exact near the ends
        assert lay[1].dim == 16
    # total maximal size at bond k is 16^min(k, N-k)
    for k in range(1, 5):
        tot = sum(charges._dmax(8, k, (a, b)) for a in range(-k, k + 1) for b in range(-k, k + 1))
        assert tot == 16 ** min(k, 8 - k)


def test_splitmix64_reference_values():
    # first outputs of SplitMix64 seeded with 0 (published reference sequence)
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    got = [charges.splitmix64((n * charges.GAMMA) & charges.MASK) for n in (1, 2, 3)]
    assert got == want
    u = charges.noise_uniform(0, 0, np.array([0, 1, 2]))
    assert np.allclose(u, [2.0 * (w >> 11) * 2.0 ** -53 - 1.0 for w in want])
