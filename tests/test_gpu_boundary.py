"""The plumbing side of the C ABI on the GPU: device memory from torch's
caching allocator and work on a torch stream (tt_set_allocator,
tt_set_stream), an allocation failure injected through the allocator hook
(TT_ENOMEM, then a clean recovery), and the per-call statistics (phase
timers, launch counts, minimum apply bytes).  The sweep results are checked
against exact diagonalisation (SM Sec. II.E: exact at untruncated bonds)."""
import pytest

from oracle import ed
from paper_2212_11973_amd import tantrg as T
from paper_2212_11973_amd import workloads as WL

pytestmark = pytest.mark.gpu


def _chain4(**kw):
    c = WL.MODELS["chain4"]
    m = T.model(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"])
    return c, m, T.options(D=c["D"], symmetry=1, beta0=c["beta0"], krylov_dim=c["krylov"], **kw)


def _ed_check(c, o):
    E, _, _ = ed.Hubbard(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"]).spectrum()
    lnZ, Ebl = ed.same_ode_bilayer(E, c["beta0"], o["beta"])
    assert abs(o["lnZ"] - lnZ) <= 1e-10 * abs(lnZ)
    assert abs(o["E"] - Ebl) <= 1e-10 * max(abs(Ebl), 1e-2)


def test_torch_allocator_and_stream():
    import torch
    c, m, o = _chain4()
    ref = T.State.init(m, o)
    for _ in range(10):
        ref.sweep(c["dbeta"])
    want = ref.observables()
    ref.free()
    side = torch.cuda.Stream()                 # default priority
    before = torch.cuda.memory_allocated(0)
    try:
        with torch.cuda.stream(side):
            T.use_torch_memory_and_stream(0)
            st = T.State.init(m, o)
            assert torch.cuda.memory_allocated(0) > before     # the state lives in torch's pool
            for _ in range(10):
                st.sweep(c["dbeta"])
            got = st.observables()
            st.free()
        assert torch.cuda.memory_allocated(0) == before        # and all of it went back
    finally:
        T.use_library_memory_and_stream()
    assert got == want                                         # same kernels, same order: bit for bit
    _ed_check(c, got)


@pytest.mark.parametrize("fail_at", [1, 7, 40, 150])
def test_allocation_failure_is_reported_and_recovered(fail_at):
    import torch
    c, m, o = _chain4()
    count = [0]
    live = {}

    def alloc(n):
        count[0] += 1
        if count[0] == fail_at:
            return 0
        t = torch.empty(int(n), dtype=torch.uint8, device="cuda:0")
        live[t.data_ptr()] = t
        return t.data_ptr()

    def free(p):
        live.pop(p)

    print("allocation failure at", fail_at, flush=True)
    try:
        T.tt_set_allocator(alloc, free)
        with pytest.raises(T.TTError) as e:
            T.State.init(m, o)
        assert e.value.code == T.TT_ENOMEM
        assert not live                                        # nothing of the failed state is kept
    finally:
        T.use_library_memory_and_stream()
    st = T.State.init(m, o)                                    # the library still works
    for _ in range(5):
        st.sweep(c["dbeta"])
    _ed_check(c, st.observables())
    st.free()


def test_sweep_stats_phases_launches_and_bytes():
    c, m, o = _chain4()
    st = T.State.init(m, o)
    plain = st.sweep(c["dbeta"], stats=True)
    assert plain.t_heff == 0.0 and plain.t_lanczos == 0.0    # phase timing off by default
    assert plain.n_launches > 0 and plain.bytes_min > 0
    T.tt_phase_timing(True)
    try:
        timed = st.sweep(c["dbeta"], stats=True)
    finally:
        T.tt_phase_timing(False)
    for k in ("t_heff", "t_bond", "t_lanczos", "t_qr", "t_env", "t_absorb"):
        assert getattr(timed, k) > 0.0, k
    total = timed.t_heff + timed.t_bond + timed.t_lanczos + timed.t_qr + timed.t_env + timed.t_absorb
    assert total <= 1e3 * timed.seconds * 1.05                # phases are disjoint parts of the call
    assert timed.n_launches == plain.n_launches               # the same sweep
    assert timed.bytes_min == plain.bytes_min
    assert timed.n_applies == plain.n_applies
    # with captured sweeps the replay reports the launches it holds
    T.tt_sweep_graphs(True)
    try:
        st.sweep(c["dbeta"])                                   # capture
        replay = st.sweep(c["dbeta"], stats=True)
    finally:
        T.tt_sweep_graphs(False)
    assert replay.n_launches == plain.n_launches
    st.free()
