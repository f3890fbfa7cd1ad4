"""ctypes binding of libtantrg.so (argument marshalling only).

Every name mirrors an entry point of ``include/tantrg.h``.  The library is
loaded on first use from this package's directory; if it is missing the
binding raises (there is no other implementation).
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# TANTRG_LIB names another build of the same library (e.g. one with host
# sanitizers); by default the one built in this package's directory
LIB_PATH = os.environ.get("TANTRG_LIB") or os.path.join(_HERE, "libtantrg.so")

TT_OK, TT_EINVAL, TT_ENOMEM, TT_EDEVICE, TT_ENUMERIC, TT_EIO = 0, -1, -2, -3, -4, -5
TT_CHAIN, TT_CYLINDER, TT_OPEN_SQUARE = 0, 1, 2
TT_FP64, TT_FP32, TT_BF16X3, TT_BF16X6 = 0, 1, 2, 3

SYMBOLS = [
    "tt_options_default", "mpo_init_highT", "tdvp_sweep", "tdvp_sweep_batch",
    "thermo_observables", "tt_state_free", "tt_last_error", "tt_state_info",
    "tt_state_bond_sectors", "tt_state_export_site", "tt_state_import_site",
    "tt_state_save", "tt_state_load", "tt_heff_apply", "tt_set_stream",
    "tt_set_allocator", "tt_heff_last_timing", "tt_check_plans", "tt_model_bond_sectors",
    "tt_profile_enable", "tt_profile_read", "thermo_local_observables", "tt_thermo_derived",
    "thermo_spin_correlation", "tt_sweep_graphs", "tt_svd_lds_limit", "thermo_green_function", "thermo_pairing_order",
    "tt_heff2_apply", "tt_heff_apply_noalloc", "tt_phase_timing", "tt_tune_apply", "tdvp_sweep2",
]


class tt_model(C.Structure):
    _fields_ = [("W", C.c_int), ("L", C.c_int), ("geometry", C.c_int),
                ("t", C.c_double), ("tp", C.c_double), ("U", C.c_double), ("mu", C.c_double),
                ("hp", C.c_double)]


class tt_options(C.Structure):
    _fields_ = [("D", C.c_int), ("symmetry", C.c_int), ("beta0", C.c_double),
                ("taylor_order", C.c_int), ("krylov_dim", C.c_int), ("krylov_tol", C.c_double),
                ("precision", C.c_int), ("pad_eps", C.c_double), ("seed", C.c_uint64),
                ("env_on_host", C.c_int), ("sector_cap", C.c_int)]


class tt_observables(C.Structure):
    _fields_ = [("beta", C.c_double), ("beta_phys", C.c_double), ("lnZ", C.c_double),
                ("f", C.c_double), ("E", C.c_double), ("e", C.c_double),
                ("lnZ_single", C.c_double), ("lambda_", C.c_double), ("n_sites", C.c_int),
                ("herm_defect", C.c_double)]


class tt_sweep_stats(C.Structure):
    _fields_ = [("seconds", C.c_double), ("flops_alg", C.c_double), ("flops_heff", C.c_double),
                ("n_applies", C.c_int), ("n_exps", C.c_int), ("max_krylov_err", C.c_double),
                ("bytes_min", C.c_double), ("t_heff", C.c_double), ("t_bond", C.c_double),
                ("t_lanczos", C.c_double), ("t_qr", C.c_double), ("t_env", C.c_double),
                ("t_absorb", C.c_double), ("n_launches", C.c_longlong), ("discarded", C.c_double)]


class TTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("tantrg error %d: %s" % (code, msg))
        self.code = code


_lib = None


def _init_torch_runtime():
    """Initialise torch's HIP runtime before the library's own.  torch ships
    its own copy of the HIP runtime, whose soname equals the system one's;
    loaded first, it is the only runtime in the process (the library's
    dependency resolves to it by soname), so device pointers and streams pass
    freely between torch and the library.  Loaded after the system runtime
    (as under a profiler that preloads it), torch maps a second HIP and HSA
    runtime into the process, because its libraries name the runtime without
    the version suffix."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def lib(init_torch=True):
    """The loaded library (raises if it was not built).  init_torch=False
    keeps torch out of the process: the library then runs on the system HIP
    runtime alone, with its own hipMalloc and the null stream (the form a
    profiler that preloads the system runtime needs)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libtantrg.so is not built: run __graft_entry__.build()")
        if init_torch:
            _init_torch_runtime()
        L = C.CDLL(LIB_PATH)
        vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
        L.tt_last_error.restype = C.c_char_p
        L.tt_options_default.argtypes = [C.POINTER(tt_options)]
        L.mpo_init_highT.argtypes = [C.POINTER(tt_model), C.POINTER(tt_options), C.POINTER(vp)]
        L.tdvp_sweep.argtypes = [vp, C.c_double, C.POINTER(tt_sweep_stats)]
        L.tdvp_sweep_batch.argtypes = [C.POINTER(vp), C.c_int, C.c_double, C.POINTER(tt_sweep_stats)]
        L.tdvp_sweep2.argtypes = [vp, C.c_double, C.c_int, C.c_double, C.POINTER(tt_sweep_stats)]
        L.thermo_observables.argtypes = [vp, C.POINTER(tt_observables)]
        L.thermo_local_observables.argtypes = [vp, dp]
        L.tt_thermo_derived.argtypes = [C.c_int, dp, dp, dp, dp, dp]
        L.thermo_spin_correlation.argtypes = [vp, C.c_int, dp, ip]
        L.tt_sweep_graphs.argtypes = [C.c_int]
        L.tt_svd_lds_limit.argtypes = [C.c_longlong]
        L.tt_phase_timing.argtypes = [C.c_int]
        L.tt_tune_apply.argtypes = [vp, C.c_int, ip]
        L.thermo_green_function.argtypes = [vp, C.c_double, C.c_double, dp]
        L.thermo_pairing_order.argtypes = [vp, dp, ip]
        L.tt_heff2_apply.argtypes = [C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, C.c_int, vp]
        L.tt_state_free.argtypes = [vp]
        L.tt_state_free.restype = None
        L.tt_state_info.argtypes = [vp, ip, ip]
        L.tt_state_bond_sectors.argtypes = [vp, C.c_int, ip, ip, ip, ip]
        L.tt_state_export_site.argtypes = [vp, C.c_int, dp]
        L.tt_state_import_site.argtypes = [vp, C.c_int, dp]
        L.tt_state_save.argtypes = [vp, C.c_char_p]
        L.tt_state_load.argtypes = [C.c_char_p, C.POINTER(vp)]
        L.tt_heff_apply.argtypes = [C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp, C.c_int, vp]
        L.tt_heff_apply_noalloc.argtypes = [C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp, C.c_int, vp]
        L.tt_set_stream.argtypes = [vp]
        L.tt_set_allocator.argtypes = [vp, vp, vp]
        L.tt_heff_last_timing.argtypes = [dp]
        L.tt_model_bond_sectors.argtypes = [C.POINTER(tt_model), C.POINTER(tt_options), C.c_int, ip, ip, ip, ip]
        L.tt_profile_enable.argtypes = [C.c_int]
        L.tt_profile_read.argtypes = [dp]
        L.tt_check_plans.argtypes = [C.POINTER(tt_model), C.POINTER(tt_options),
                                     C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]
        _lib = L
    return _lib


def _check(code):
    if code != TT_OK:
        raise TTError(code, lib().tt_last_error().decode())


def options_default():
    o = tt_options()
    _check(lib().tt_options_default(C.byref(o)))
    return o


def model(W, L, geometry, t=1.0, U=8.0, mu=0.0, tp=0.0, hp=0.0):
    return tt_model(W, L, geometry, t, tp, U, mu, hp)


def options(**kw):
    o = options_default()
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def mpo_init_highT(m, o):
    h = C.c_void_p()
    _check(lib().mpo_init_highT(C.byref(m), C.byref(o), C.byref(h)))
    return h


def tdvp_sweep(state, dbeta, stats=False):
    if stats:
        s = tt_sweep_stats()
        _check(lib().tdvp_sweep(state, dbeta, C.byref(s)))
        return s
    _check(lib().tdvp_sweep(state, dbeta, None))
    return None


def tdvp_sweep2(state, dbeta, D_max, cutoff=0.0, stats=False):
    """One 2-TDVP step (bond growth by SVD splits); returns tt_sweep_stats if stats."""
    s = tt_sweep_stats()
    _check(lib().tdvp_sweep2(state, dbeta, int(D_max), float(cutoff), C.byref(s) if stats else None))
    return s if stats else None


def tdvp_sweep_batch(states, dbeta, stats=False):
    arr = (C.c_void_p * len(states))(*[s.value for s in states])
    if stats:
        s = tt_sweep_stats()
        _check(lib().tdvp_sweep_batch(arr, len(states), dbeta, C.byref(s)))
        return s
    _check(lib().tdvp_sweep_batch(arr, len(states), dbeta, None))
    return None


def thermo_observables(state):
    o = tt_observables()
    _check(lib().thermo_observables(state, C.byref(o)))
    return {k: getattr(o, k) for k, _ in o._fields_}


def thermo_local_observables(state):
    """dict(n=density, docc=double occupancy) per site at beta_phys = 2 beta."""
    out = (C.c_double * 2)()
    _check(lib().thermo_local_observables(state, out))
    return dict(n=out[0], docc=out[1])


def tt_svd_lds_limit(max_doubles):
    """Largest SVD block (doubles of X and its column norms) one workgroup takes
    in LDS for the 2-TDVP split; larger blocks spread each Jacobi round over the
    GPU.  0: the device's LDS."""
    _check(lib().tt_svd_lds_limit(int(max_doubles)))


def tt_sweep_graphs(on):
    """Replay captured sweeps (hipGraph) for repeated steps of equal dbeta."""
    _check(lib().tt_sweep_graphs(1 if on else 0))


def tt_tune_apply(state, mode, forms=None):
    """Apply forms per site, f + 4 b: f the site apply (0: L.A, W, .R; 1: MPO
    folded into L; 2: the fused LW.A.R kernel, FP64 states), b the left bond's
    apply (0: L.S then .R; 1: fused, FP64 states).  mode 0 / 1: f = 0 / 1 and
    b = 0 everywhere; 2: time every form and keep the fastest; 3: the given
    list; 4: f = 2, b = 1 everywhere.  Returns the forms."""
    n, _ = tt_state_info(state)
    arr = (C.c_int * n)(*(forms or []))
    _check(lib().tt_tune_apply(state, int(mode), arr))
    return list(arr)


def tt_phase_timing(on):
    """Per-phase device timing (t_heff ... t_absorb) of sweeps that return stats."""
    _check(lib().tt_phase_timing(1 if on else 0))


def thermo_spin_correlation(state, d2):
    """(F(d), number of pairs) for pairs at squared lattice distance d2."""
    F, n = C.c_double(), C.c_int()
    _check(lib().thermo_spin_correlation(state, d2, C.byref(F), C.byref(n)))
    return F.value, n.value


def thermo_green_function(state, kx, ky):
    """G(k, beta_phys/2) at k = (kx, ky) (x along the length, y across the width)."""
    G = C.c_double()
    _check(lib().thermo_green_function(state, float(kx), float(ky), C.byref(G)))
    return G.value


def thermo_pairing_order(state):
    """(Delta_p = <Delta_tot> / N_p, N_p) for a state with symmetry = 0."""
    d, n = C.c_double(), C.c_int()
    _check(lib().thermo_pairing_order(state, C.byref(d), C.byref(n)))
    return d.value, n.value


def tt_thermo_derived(beta_phys, e, f):
    """(C_e, s) per site for a series of bilayer observables (beta_phys
    strictly increasing, at least three points)."""
    n = len(beta_phys)
    if len(e) != n or len(f) != n:
        raise ValueError("beta_phys, e and f must have the same length")
    arr = lambda x: (C.c_double * n)(*[float(v) for v in x])
    c, s = (C.c_double * n)(), (C.c_double * n)()
    _check(lib().tt_thermo_derived(n, arr(beta_phys), arr(e), arr(f), c, s))
    return list(c), list(s)


def tt_state_free(state):
    lib().tt_state_free(state)


def tt_state_info(state):
    n = C.c_int()
    _check(lib().tt_state_info(state, C.byref(n), None))
    dims = (C.c_int * (n.value + 1))()
    _check(lib().tt_state_info(state, C.byref(n), dims))
    return n.value, list(dims)


def tt_state_bond_sectors(state, k):
    ns = C.c_int()
    _check(lib().tt_state_bond_sectors(state, k, C.byref(ns), None, None, None))
    qu, qd, dm = (C.c_int * ns.value)(), (C.c_int * ns.value)(), (C.c_int * ns.value)()
    _check(lib().tt_state_bond_sectors(state, k, C.byref(ns), qu, qd, dm))
    return [((qu[i], qd[i]), dm[i]) for i in range(ns.value)]


def tt_state_export_site(state, k):
    _, dims = tt_state_info(state)
    out = np.zeros((dims[k], 4, 4, dims[k + 1]))
    _check(lib().tt_state_export_site(state, k, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def tt_state_import_site(state, k, arr):
    a = np.ascontiguousarray(arr, dtype=np.float64)
    _check(lib().tt_state_import_site(state, k, a.ctypes.data_as(C.POINTER(C.c_double))))


def tt_state_save(state, path):
    _check(lib().tt_state_save(state, path.encode()))


def tt_state_load(path):
    h = C.c_void_p()
    _check(lib().tt_state_load(path.encode(), C.byref(h)))
    return h


def tt_heff_apply(Dl, Dr, DH, L_ptr, W_ptr, A_ptr, R_ptr, out_ptr, precision=TT_FP64, stream=None):
    """Device pointers (ints, e.g. torch ``data_ptr()``) of FP64 row-major arrays."""
    _check(lib().tt_heff_apply(Dl, Dr, DH, C.c_void_p(L_ptr), C.c_void_p(W_ptr), C.c_void_p(A_ptr),
                               C.c_void_p(R_ptr), C.c_void_p(out_ptr), precision,
                               C.c_void_p(stream) if stream else None))


def tt_heff_apply_noalloc(Dl, Dr, DH, L_ptr, W_ptr, A_ptr, R_ptr, out_ptr, precision=TT_FP64, stream=None):
    """tt_heff_apply without device allocation (the library's static scratch)."""
    _check(lib().tt_heff_apply_noalloc(Dl, Dr, DH, C.c_void_p(L_ptr), C.c_void_p(W_ptr), C.c_void_p(A_ptr),
                                       C.c_void_p(R_ptr), C.c_void_p(out_ptr), precision,
                                       C.c_void_p(stream) if stream else None))


def tt_heff2_apply(Dl, Dr, DH, L_ptr, W1_ptr, W2_ptr, C_ptr, R_ptr, out_ptr, precision=TT_FP64, stream=None):
    """Two-site generator on device pointers of FP64 row-major arrays."""
    _check(lib().tt_heff2_apply(Dl, Dr, DH, C.c_void_p(L_ptr), C.c_void_p(W1_ptr), C.c_void_p(W2_ptr),
                                C.c_void_p(C_ptr), C.c_void_p(R_ptr), C.c_void_p(out_ptr), precision,
                                C.c_void_p(stream) if stream else None))


def tt_heff_last_timing():
    ms = (C.c_double * 4)()
    _check(lib().tt_heff_last_timing(ms))
    return list(ms)


def tt_check_plans(m, o):
    """(violations, work_doubles, report) of the host-side bounds check."""
    v, w = C.c_longlong(), C.c_longlong()
    _check(lib().tt_check_plans(C.byref(m), C.byref(o), C.byref(v), C.byref(w)))
    rep = lib().tt_last_error().decode() if v.value else ""
    return v.value, w.value, rep


def tt_model_bond_sectors(m, o, k):
    ns = C.c_int()
    _check(lib().tt_model_bond_sectors(C.byref(m), C.byref(o), k, C.byref(ns), None, None, None))
    qu, qd, dm = (C.c_int * ns.value)(), (C.c_int * ns.value)(), (C.c_int * ns.value)()
    _check(lib().tt_model_bond_sectors(C.byref(m), C.byref(o), k, C.byref(ns), qu, qd, dm))
    return [((qu[i], qd[i]), dm[i]) for i in range(ns.value)]


def tt_profile_enable(on):
    _check(lib().tt_profile_enable(1 if on else 0))


PROFILE_KINDS = ("gemm_LA", "gemm_R", "gemm_envL", "gemm_envR1", "gemm_envR3", "gemm_bond", "gemm_absorb",
                 "gemm_Wdense", "wstage", "qr",
                 "k_gemm_64x64", "k_gemm_128x32", "k_gemm_256x16", "k_gemm_32x128", "k_gemm_32x32",
                 "k_gemm_reduce", "k_wgemm", "k_fused")


def tt_profile_read():
    """{kind: dict(ms, flops, bytes, launches)} since the last read; 'gemm' sums the
    grouped-GEMM kinds (gemm_*), the k_gemm_* kinds time single kernel dispatches."""
    buf = (C.c_double * 72)()
    _check(lib().tt_profile_read(buf))
    out = {}
    for i, k in enumerate(PROFILE_KINDS):
        out[k] = dict(ms=buf[4 * i], flops=buf[4 * i + 1], bytes=buf[4 * i + 2], launches=int(buf[4 * i + 3]))
    g = dict(ms=0.0, flops=0.0, bytes=0.0, launches=0)
    for k in PROFILE_KINDS:
        if k.startswith("gemm_"):
            for f in g:
                g[f] += out[k][f]
    out["gemm"] = g
    return out


def tt_set_stream(stream):
    _check(lib().tt_set_stream(C.c_void_p(stream) if stream else None))


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_allocator = None   # the registered callbacks (kept alive while registered)


def tt_set_allocator(alloc, free):
    """Register Python callables alloc(nbytes) -> device address (0 on
    failure) and free(address) as the library's device allocator; None, None
    restores hipMalloc/hipFree."""
    global _allocator
    if alloc is None and free is None:
        _check(lib().tt_set_allocator(None, None, None))
        _allocator = None
        return
    a = ALLOC_FN(lambda n, ctx: alloc(n) or None)
    f = FREE_FN(lambda p, ctx: free(p))
    _check(lib().tt_set_allocator(C.cast(a, C.c_void_p), C.cast(f, C.c_void_p), None))
    _allocator = (a, f)


def use_torch_memory_and_stream(device=0):
    """Route the library's device memory through torch's caching allocator and
    its work onto torch's current stream of `device` (torch stays the owner
    of both; the library only borrows them)."""
    import torch
    dev = torch.device("cuda", device)
    stream = torch.cuda.current_stream(dev)

    def alloc(n):
        try:
            return torch.cuda.caching_allocator_alloc(int(n), dev, stream)
        except RuntimeError:
            return 0

    tt_set_allocator(alloc, torch.cuda.caching_allocator_delete)
    tt_set_stream(stream.cuda_stream)


def use_library_memory_and_stream():
    """Back to hipMalloc/hipFree and the null stream."""
    tt_set_allocator(None, None)
    tt_set_stream(None)


class State:
    """Owning wrapper of a tt_state handle."""

    def __init__(self, handle):
        self.h = handle

    @classmethod
    def init(cls, m, o):
        return cls(mpo_init_highT(m, o))

    def sweep(self, dbeta, stats=False):
        return tdvp_sweep(self.h, dbeta, stats)

    def sweep2(self, dbeta, D_max, cutoff=0.0, stats=False):
        return tdvp_sweep2(self.h, dbeta, D_max, cutoff, stats)

    def observables(self):
        return thermo_observables(self.h)

    def tune_apply(self, mode=2, forms=None):
        return tt_tune_apply(self.h, mode, forms)

    def local_observables(self):
        return thermo_local_observables(self.h)

    def spin_correlation(self, d2):
        return thermo_spin_correlation(self.h, d2)

    def green_function(self, kx, ky):
        return thermo_green_function(self.h, kx, ky)

    def pairing_order(self):
        return thermo_pairing_order(self.h)

    def info(self):
        return tt_state_info(self.h)

    def sectors(self, k):
        return tt_state_bond_sectors(self.h, k)

    def export_site(self, k):
        return tt_state_export_site(self.h, k)

    def free(self):
        if self.h is not None and self.h.value:
            tt_state_free(self.h)
        self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
