"""Host-side tests of the C-ABI library (no GPU): every declared symbol is
exported, argument validation fails cleanly, descriptor bounds hold for every
workload, and the bond sectors equal the oracle's allocation rule."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

from paper_2212_11973_amd import tantrg as T  # noqa: E402
from paper_2212_11973_amd import workloads as WL  # noqa: E402


def _declared():
    src = open(os.path.join(ROOT, "include", "tantrg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = T.lib()
    names = _declared()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(T.SYMBOLS) == names


def _m(**kw):
    d = dict(W=1, L=4, geometry=T.TT_CHAIN, t=1.0, U=4.0, mu=0.0)
    d.update(kw)
    return T.model(d["W"], d["L"], d["geometry"], d["t"], d["U"], d["mu"], kw.get("tp", 0.0))


@pytest.mark.parametrize("field,value", [("precision", 7), ("krylov_dim", 0), ("krylov_dim", 33),
                                         ("taylor_order", 5), ("symmetry", 3), ("D", 0),
                                         ("env_on_host", 1), ("krylov_tol", -1.0)])
def test_invalid_options_rejected_without_gpu(field, value):
    o = T.options(**{field: value})
    with pytest.raises(T.TTError) as e:
        T.mpo_init_highT(_m(), o)
    assert e.value.code == T.TT_EINVAL


def test_pairing_field_needs_the_non_symmetric_mode():
    m = T.model(1, 4, T.TT_CHAIN, 1.0, 4.0, 0.0, hp=0.1)
    with pytest.raises(T.TTError) as e:
        T.mpo_init_highT(m, T.options(symmetry=1))
    assert e.value.code == T.TT_EINVAL
    with pytest.raises(T.TTError) as e:
        T.mpo_init_highT(T.model(1, 4, T.TT_CHAIN, 1.0, 4.0, 0.0, hp=float("inf")), T.options(symmetry=0))
    assert e.value.code == T.TT_EINVAL
    # non-symmetric bonds hold the larger pairing MPO: max(min(D, 16^k), D_H) states
    from oracle import mpo
    mm = mpo.HubbardMPO(2, 3, lattice_open_square(), 1.0, 8.0, 1.0, hp=0.2)
    o = T.options(D=20, symmetry=0)
    m = T.model(2, 3, T.TT_OPEN_SQUARE, 1.0, 8.0, 1.0, hp=0.2)
    for k in range(7):
        n = len(mm.bond_charges(k)) if k < 6 else 1
        want = max(min(20, 16 ** min(k, 6 - k)), n)
        assert dict(T.tt_model_bond_sectors(m, o, k)) == {(0, 0): want}, k
    v, _, rep = T.tt_check_plans(m, o)
    assert v == 0, rep


def lattice_open_square():
    from oracle import lattice
    return lattice.OPEN_SQUARE


@pytest.mark.parametrize("kw", [dict(tp=float("nan")), dict(W=2, geometry=T.TT_CHAIN), dict(L=1), dict(geometry=5)])
def test_invalid_model_rejected_without_gpu(kw):
    with pytest.raises(T.TTError) as e:
        T.mpo_init_highT(_m(**kw), T.options())
    assert e.value.code == T.TT_EINVAL


def test_load_rejects_foreign_file(tmp_path):
    p = tmp_path / "x.bin"
    p.write_bytes(b"not a state at all")
    with pytest.raises(T.TTError) as e:
        T.tt_state_load(str(p))
    assert e.value.code == T.TT_EIO
    with pytest.raises(T.TTError) as e:
        T.tt_state_load(str(tmp_path / "missing.bin"))
    assert e.value.code == T.TT_EIO


def test_heff_apply_rejects_bad_arguments():
    with pytest.raises(T.TTError) as e:
        T.tt_heff_apply(0, 4, 2, 1, 1, 1, 1, 1)
    assert e.value.code == T.TT_EINVAL
    with pytest.raises(T.TTError) as e:
        T.tt_heff_apply(4, 4, 2, 0, 1, 1, 1, 1)
    assert e.value.code == T.TT_EINVAL


CASES = [(1, 4, 0, 256, 1), (1, 4, 0, 256, 0), (2, 3, 2, 40, 1), (4, 4, 1, 64, 1), (1, 6, 0, 12, 0),
         (3, 4, 2, 100, 1), (4, 16, 1, 200, 1)]


@pytest.mark.parametrize("W,L,geo,D,sym", CASES)
def test_descriptor_bounds(W, L, geo, D, sym):
    v, work, rep = T.tt_check_plans(T.model(W, L, geo, 1.0, 8.0, 1.5), T.options(D=D, symmetry=sym))
    assert v == 0, rep
    assert work > 0


@pytest.mark.parametrize("name,cap,D", [("cl4x16", 64, 0), ("cl4x16", 0, 0), ("cl6x12", 64, 0),
                                        ("os10x10", 0, 4000), ("os10x10", 64, 8000)])
def test_descriptor_bounds_full_workloads(name, cap, D):
    """The workloads' own shapes (sector cap 64 and uncapped, up to D = 8000):
    every descriptor stays inside its buffer (the same check runs before the
    first launch of every state)."""
    c = WL.MODELS[name]
    m = T.model(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"])
    v, work, rep = T.tt_check_plans(m, T.options(D=D or c["D"], symmetry=1, sector_cap=cap))
    assert v == 0, rep


def test_mid_size_chain_plans_in_bounds():
    """The 8-site chain at D = 1000 of the GPU parity tests: 64-column QR
    blocks in four row chunks (cap 64) and the global-memory QR (no cap)."""
    for cap in (64, 0):
        v, _, rep = T.tt_check_plans(T.model(1, 8, 0, 1.0, 8.0, 1.5), T.options(D=1000, symmetry=1, sector_cap=cap))
        assert v == 0, rep


@pytest.mark.parametrize("W,L,geo,D,cap,tp", [(4, 4, 1, 64, 0, 0.0), (2, 3, 2, 40, 0, 0.0), (4, 16, 1, 300, 0, 0.0),
                                              (1, 6, 0, 30, 0, 0.0), (4, 4, 1, 64, 6, 0.0), (4, 16, 1, 300, 12, 0.0),
                                              (4, 16, 1, 2000, 64, 0.0), (3, 4, 2, 100, 5, 0.0),
                                              (4, 4, 1, 64, 0, -0.25), (3, 4, 2, 100, 5, 0.3)])
def test_sectors_match_oracle_allocation(W, L, geo, D, cap, tp):
    from oracle import charges, mpo
    mm = mpo.HubbardMPO(W, L, geo, 1.0, 8.0, 1.0, tp=tp)
    N = mm.N
    q0 = [mm.bond_charges(k) for k in range(N)] + [[(0, 0)]]
    lay = charges.bond_layouts(q0, N, D, True, cap)
    m = T.model(W, L, geo, 1.0, 8.0, 1.0, tp)
    o = T.options(D=D, symmetry=1, sector_cap=cap)
    bonds = range(N + 1) if N <= 16 else sorted({0, 1, 2, 3, 4, 6, 9, 13, N // 2, N - 5, N - 2, N - 1, N})
    for k in bonds:
        want = {}
        for q in lay[k].charges:
            want[q] = want.get(q, 0) + 1
        got = dict(T.tt_model_bond_sectors(m, o, k))
        assert got == want, k


@pytest.mark.parametrize("W,L,geo,D,cap,order,b0", [(1, 6, 0, 30, 0, 2, 0.01), (2, 3, 2, 60, 0, 2, 2.0 ** -10),
                                                    (3, 3, 1, 120, 64, 2, 0.01), (1, 8, 0, 40, 8, 3, 2.0 ** -10),
                                                    (4, 8, 1, 600, 64, 2, 2.0 ** -10)])
def test_settn_sectors_match_oracle(W, L, geo, D, cap, order, b0):
    # the SETTN start's reduced bond states (counts per charge) and the sectors
    # allocated around them equal the oracle's
    from oracle import charges, mpo
    mm = mpo.HubbardMPO(W, L, geo, 1.0, 8.0, 1.0)
    N = mm.N
    _, q0 = mpo.settn_rho0(mm, b0, order)
    lay = charges.bond_layouts(list(q0) + [[(0, 0)]], N, D, True, cap)
    m = T.model(W, L, geo, 1.0, 8.0, 1.0)
    o = T.options(D=D, symmetry=1, sector_cap=cap, beta0=b0, taylor_order=order)
    bonds = range(N + 1) if N <= 16 else sorted({0, 1, 2, 3, 4, N // 2, N - 3, N - 1, N})
    for k in bonds:
        want = {}
        for q in lay[k].charges:
            want[q] = want.get(q, 0) + 1
        assert dict(T.tt_model_bond_sectors(m, o, k)) == want, k
    v, _, rep = T.tt_check_plans(m, o)
    assert v == 0, rep


def test_settn_rejects_bad_orders():
    m = T.model(1, 4, 0, 1.0, 4.0, 0.0)
    for order in (0, 5):
        with pytest.raises(T.TTError):
            T.tt_model_bond_sectors(m, T.options(D=16, taylor_order=order), 1)


def test_binding_fails_loudly_without_the_library(monkeypatch):
    # no fallback: with the shared library absent every call raises
    monkeypatch.setattr(T, "_lib", None)
    monkeypatch.setattr(T, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libtantrg.so"))
    with pytest.raises(RuntimeError):
        T.lib()
    with pytest.raises(RuntimeError):
        T.mpo_init_highT(_m(), T.options())



@pytest.mark.parametrize("W,L,geo,D,cap,hp", [(2, 3, 2, 40, 0, 0.1), (4, 4, 1, 64, 0, 0.2), (1, 6, 0, 30, 8, 0.0),
                                              (4, 16, 1, 500, 64, 0.05), (3, 4, 2, 100, 5, 0.3)])
def test_sz_sectors_match_oracle(W, L, geo, D, cap, hp):
    # symmetry = 2: blocks by q_up - q_dn alone (sectors (sz, 0)), as the
    # oracle allocates them for the pairing field
    from oracle import charges, mpo
    mm = mpo.HubbardMPO(W, L, geo, 1.0, 8.0, 1.0, hp=hp)
    N = mm.N
    q0 = [mm.bond_charges(k) for k in range(N)] + [[(0, 0)]]
    lay = charges.bond_layouts(q0, N, D, True, cap, mode="sz")
    m = T.model(W, L, geo, 1.0, 8.0, 1.0, hp=hp)
    o = T.options(D=D, symmetry=2, sector_cap=cap)
    bonds = range(N + 1) if N <= 16 else sorted({0, 1, 2, 3, 4, N // 2, N - 3, N - 1, N})
    for k in bonds:
        want = {}
        for q in lay[k].charges:
            want[q] = want.get(q, 0) + 1
        assert dict(T.tt_model_bond_sectors(m, o, k)) == want, k
    v, _, rep = T.tt_check_plans(m, o)
    assert v == 0, rep
