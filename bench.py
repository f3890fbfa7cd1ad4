#!/usr/bin/env python3
"""Benchmark of the tanTRG hot path on one MI355X.

Metric: seconds per symmetric 1-TDVP beta step (one tdvp_sweep) on the 4x16
cylinder Hubbard model (t=1, U=8, mu=1.5, U(1)xU(1) block-sparse, D=2000), and
the dense effective-Hamiltonian apply throughput (TFLOP/s) at D=2000, D_H=18.
Every input is synthetic: the state is rho0 = 1 - beta0 H padded with seeded
noise; the dense apply uses i.i.d. N(0,1) tensors.

Prints one JSON line.  --gpus N with N > 1 exits: the build runs on one GPU.
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}   # dense MFMA TFLOP/s (MI355X)
PEAK_FP64_VALU = 78.6                                   # 256 CU x 2.4 GHz x 128 flop/clk
PEAK_HBM_GBS = 8000.0
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
# single kernels that can be the dominant one, with the name rocprofv3 reports
SHAPES = ("64x64", "128x32", "256x16", "32x128", "32x32")


def kernel_name(kind, prec):
    if kind.startswith("k_gemm_") and kind != "k_gemm_reduce":
        return "tt::k_gemm<%d, %d>" % (SHAPES.index(kind[len("k_gemm_"):]), prec)
    # the names rocprofv3 reports: the wave GEMM is instantiated per multiply
    # type (FP64 multiplies in the FP64 and FP32 modes), the W stage per
    # intermediate type (the 32-bit index form in the headline plans)
    return {"k_gemm_reduce": "tt::k_gemm_reduce", "k_wgemm": "tt::k_wgemm<%d>" % (prec if prec >= 2 else 0),
            "wstage": "tt::k_wstage<%s, int>" % ("double" if prec == 0 else "float"),
            "k_fused": "tt::k_fused_apply",
            "qr": "tt::k_qr_chunk + k_qr_stack + k_qr_combine + k_qrw_*"}[kind]


def cpu_baseline(c, D, sector_cap, budget_s=25.0):
    """The block-sparse FP64 oracle on the same workload, timed on the host
    over a bounded sample: from the same start (rho0 padded with seed 1), the
    left-to-right site steps k = 0, 1, ... (site exponential, QR, left
    environment, bond exponential, absorb) until budget_s has elapsed with at
    least two steps between full bonds done.  A sweep's 2N - 1 site steps are
    priced by the measured step whose pair of bond dimensions matches (the
    right-to-left step at site k costs what the left-to-right one at k - 1
    does: the same contractions mirrored)."""
    from oracle import blocked, mpo as ompo
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    m = ompo.HubbardMPO(c["W"], c["L"], c["geometry"], t=c["t"], U=c["U"], mu=c["mu"])
    t0 = time.perf_counter()
    st = blocked.initial_state(m, c["beta0"], D, pad_eps=1e-3, seed=1, sector_cap=sector_cap)
    t_start = time.perf_counter() - t0
    dims = [b.dim for b in st.bonds]
    N = st.N
    tau = 0.5 * c["dbeta"]
    cost = {}            # sorted (D_k, D_k+1) -> seconds of one step
    t_sample, k = 0.0, 0
    full = max(dims)
    while k < N - 1:
        t0 = time.perf_counter()
        st.site_step_lr(k, tau, K=c["krylov"])
        dt = time.perf_counter() - t0
        t_sample += dt
        key = tuple(sorted((dims[k], dims[k + 1])))
        cost.setdefault(key, []).append(dt)
        k += 1
        print("cpu baseline: oracle site step %d %.2f s" % (k - 1, dt), file=sys.stderr, flush=True)
        if t_sample >= budget_s and len(cost.get((full, full), [])) >= 2:
            break
    def price(k):
        key = tuple(sorted((dims[k], dims[k + 1])))
        if key not in cost:
            return None
        return sum(cost[key]) / len(cost[key])
    prices = [price(k) for k in range(N - 1)]
    if any(p is None for p in prices):
        return None
    est = 2.0 * sum(prices) + price(N - 2)   # both directions, plus the merged turn priced as an edge step
    return dict(value=est, unit="s/step", cores=threads, kind="oracle",
                sample="block-sparse FP64 oracle (oracle/blocked.py) on the same workload and start: %d left-to-right "
                       "site steps timed (%.1f s; start built in %.1f s, not timed), the 2N-1 = %d site steps of a sweep "
                       "priced by the measured step of the same bond dimensions" % (k, t_sample, t_start, 2 * N - 1))


def green_map(args, T, WL):
    """beta G(k, beta/2) (main text, Fermi-surface paragraph) on the 10x10 open
    square at U = 8, mu = 2 and temperature T: linear start at beta0 = 2^-20,
    doubling grid up to beta = 1/4 (or to 1/(2T) if that is lower), linear
    steps (0.05 in beta by default) to 1/(2T), then G on kx, ky in {0, pi/5, ..., pi}."""
    c = WL.MODELS["os10x10"]
    D = args.D or c["D"]
    b0 = 2.0 ** -20
    m = T.model(c["W"], c["L"], c["geometry"], c["t"], c["U"], 2.0)
    t0 = time.perf_counter()
    st = T.State.init(m, T.options(D=D, symmetry=1, beta0=b0, pad_eps=args.green_map_pad, seed=1,
                                   krylov_dim=c["krylov"], sector_cap=args.green_map_cap))
    t_init = time.perf_counter() - t0
    b, nsw = b0, 0
    b_end = 0.5 / args.green_map_T
    t0 = time.perf_counter()
    while 2.0 * b <= min(args.green_map_exp_end, b_end) * (1 + 1e-12):
        st.sweep(b)
        b *= 2.0
        nsw += 1
        print("green map: beta %.3g" % b, file=sys.stderr, flush=True)
    while b < b_end - 1e-12:
        db = min(args.green_map_dbeta, b_end - b)
        st.sweep(db)
        b += db
        nsw += 1
        print("green map: beta %.3g" % b, file=sys.stderr, flush=True)
    t_sweeps = time.perf_counter() - t0
    o = st.observables()
    ks = [math.pi * i / 5 for i in range(6)]
    grid = []
    t0 = time.perf_counter()
    for kx in ks:
        for ky in ks:
            G = st.green_function(kx, ky)
            grid.append([kx, ky, o["beta_phys"] * G])
        print("green map: kx %.3f done" % kx, file=sys.stderr, flush=True)
    t_g = time.perf_counter() - t0
    loc = st.local_observables()
    st.free()
    print(json.dumps({"metric": "beta G(k, beta/2) map", "workload": "Hubbard 10x10 open square, U=8, mu=2, "
                      "U(1)xU(1) D=%d" % D, "beta_phys": o["beta_phys"], "n": loc["n"], "docc": loc["docc"],
                      "e": o["e"],
                      "grid": grid, "sweeps": nsw, "dbeta": args.green_map_dbeta, "pad_eps": args.green_map_pad, "sector_cap": args.green_map_cap, "exp_end": args.green_map_exp_end, "seconds_init": t_init, "seconds_sweeps": t_sweeps,
                      "seconds_per_k": t_g / len(grid)}))


def pairing_scan(args, T):
    """d-wave pairing response (main text, pairing paragraph; Fig. 5 workload):
    chi_SC = <Delta_tot> / (N_p hp) on the 4x24 cylinder, U = 8, hp = 0.01,
    T = 1 (beta_phys = 1), Sz blocks; linear start at 2^-20, doubling grid to
    beta = 1/4, one linear step to 1/2."""
    D = args.D or 2000
    hp = 0.01
    out = []
    for mu in (4.0, 3.0, 2.0):
        t0 = time.perf_counter()
        st = T.State.init(T.model(4, 24, T.TT_CYLINDER, 1.0, 8.0, mu, hp=hp),
                          T.options(D=D, symmetry=2, beta0=2.0 ** -20, pad_eps=1e-3, seed=1))
        b = 2.0 ** -20
        while 2.0 * b <= 0.25:
            st.sweep(b)
            b *= 2.0
        st.sweep(0.25)
        o = st.observables()
        loc = st.local_observables()
        d, nb = st.pairing_order()
        out.append(dict(mu=mu, beta_phys=o["beta_phys"], n=loc["n"], delta_p=d, chi_sc=d / hp, e=o["e"],
                        seconds=time.perf_counter() - t0))
        print("pairing scan: mu %g done" % mu, file=sys.stderr, flush=True)
        st.free()
    print(json.dumps({"metric": "chi_SC = Delta_p / hp", "workload": "Hubbard 4x24 cylinder, U=8, hp=0.01, Sz blocks "
                      "D=%d, T=1" % D, "points": out}))


def sweep_only(args):
    """The headline sweep without torch in the process.  A profiler that
    preloads the system HIP runtime would otherwise see torch map a second
    HIP and HSA runtime; here the library is the only HIP user.  With
    --calib-copy-mib, one device-to-device copy of that size runs after the
    warmup sweeps (the runtime's own copy kernel): the reference for HBM byte
    counters."""
    import ctypes
    from paper_2212_11973_amd import tantrg as T
    from paper_2212_11973_amd import workloads as WL
    T.lib(init_torch=False)
    c = WL.MODELS[args.workload]
    D = args.D or c["D"]
    m = T.model(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"])
    o = T.options(D=D, symmetry=1, beta0=c["beta0"], pad_eps=1e-3, seed=1, krylov_dim=c["krylov"],
                  precision=PREC[args.precision], sector_cap=args.sector_cap)
    print("init %s D=%d %s (no torch)" % (args.workload, D, args.precision), file=sys.stderr, flush=True)
    st = T.State.init(m, o)
    forms = st.tune_apply(args.apply_form)
    for i in range(args.warmup):
        st.sweep(c["dbeta"], stats=True)
        print("warmup %d done" % i, file=sys.stderr, flush=True)
    if args.calib_copy_mib > 0:
        # one device-to-device copy of known size (the runtime's own copy
        # kernel): the reference for HBM byte counters, and the marker after
        # which every dispatch belongs to the timed sweeps
        hip = ctypes.CDLL("libamdhip64.so.7")
        nbytes = args.calib_copy_mib << 20
        a, b = ctypes.c_void_p(), ctypes.c_void_p()
        for x in (a, b):
            if hip.hipMalloc(ctypes.byref(x), ctypes.c_size_t(nbytes)) != 0:
                raise RuntimeError("hipMalloc failed")
        if hip.hipMemset(a, 0, ctypes.c_size_t(nbytes)) != 0 or hip.hipDeviceSynchronize() != 0:
            raise RuntimeError("hipMemset failed")
        if hip.hipMemcpy(b, a, ctypes.c_size_t(nbytes), 3) != 0 or hip.hipDeviceSynchronize() != 0:
            raise RuntimeError("hipMemcpy failed")   # 3 = hipMemcpyDeviceToDevice
        hip.hipFree(a)
        hip.hipFree(b)
        print("calibration copy of %d MiB done" % args.calib_copy_mib, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        stats.append(st.sweep(c["dbeta"], stats=True))   # returns after the stream is synchronised
        print("step %d done" % i, file=sys.stderr, flush=True)
    s_step = (time.perf_counter() - t0) / args.steps
    # under a counter run every dispatch after the calibration copy belongs to
    # the timed sweeps: no observables then
    obs = st.observables() if args.calib_copy_mib <= 0 else {"f": None, "e": None}
    st.free()
    print(json.dumps({"metric": "s/step (sweep only, no torch)", "value": s_step, "unit": "s/step",
                      "steps": args.steps, "warmup": args.warmup, "precision": args.precision,
                      "sector_cap": args.sector_cap, "apply_form": args.apply_form,
                      "site_forms_0_1_2": [sum(f & 3 == i for f in forms) for i in (0, 1, 2)],
                      "fused_bonds": sum(f >> 2 for f in forms),
                      "workload": "%s D=%d" % (args.workload, D),
                      "flops_alg_per_step": statistics.mean(x.flops_alg for x in stats),
                      "applies_per_step": statistics.mean(x.n_applies for x in stats),
                      "f": obs["f"], "e": obs["e"]}), flush=True)


def summarize_counters(args):
    """Per-kernel counter means over the timed sweeps of `bench.py
    --sweep-only --calib-copy-mib M` runs under rocprofv3 --pmc (one rocpd
    database per pass): every dispatch after the calibration copy, grouped by
    kernel name.  FETCH_SIZE and WRITE_SIZE (KiB) are scaled by known bytes /
    counter reading of the calibration copy (M MiB read and M MiB written),
    and their sum per launch is the measured HBM traffic.  Writes
    profiles/counters_<workload>_<precision>.txt."""
    from collections import defaultdict
    known_kib = args.calib_copy_mib * 1024.0
    per = defaultdict(lambda: defaultdict(list))   # kernel -> counter -> values
    factors = {}
    for db in args.summarize_counters:
        rows = read_counter_rows(db)
        counters = sorted({r[2] for r in rows})
        # the calibration copy: the copy kernel with the largest reading of the first counter
        copies = [r for r in rows if "copyBuffer" in r[1]]
        if not copies:
            raise SystemExit("%s: no calibration copy kernel among %s" % (db, sorted({r[1] for r in rows})[:20]))
        calib = max(copies, key=lambda r: r[3])
        for cn in counters:
            cv = [r[3] for r in rows if r[0] == calib[0] and r[2] == cn]
            if cn in ("FETCH_SIZE", "WRITE_SIZE") and cv and cv[0] > 0:
                factors[cn] = known_kib / cv[0]
        for (did, kname, cn, v, dur) in rows:
            if did <= calib[0]:
                continue
            short = kname.split("(")[0].replace("void ", "")
            per[short][cn].append(v)
            per[short]["_duration_ns[" + cn + "]"].append(dur)
    out = ["# rocprofv3 counter summary: the timed sweeps of bench.py --sweep-only (dispatches after the calibration "
           "copy), means per dispatch",
           "# commands: " + args.counter_commands,
           "workload=%s" % args.workload, "precision=%s" % args.precision,
           "sources_digest=%s" % kernel_sources_digest(),
           "calibration_copy_MiB=%d" % args.calib_copy_mib]
    for cn, f in sorted(factors.items()):
        out.append("calibration_factor[%s]=%.6f" % (cn, f))
    for k in sorted(per, key=lambda k: -len(per[k].get("FETCH_SIZE", per[k].get(next(iter(per[k])), [])))):
        cs = per[k]
        n = max(len(v) for c, v in cs.items() if not c.startswith("_"))
        out.append("dispatches[%s]=%d" % (k, n))
        for cn, v in sorted(cs.items()):
            if cn.startswith("_"):
                continue
            out.append("mean[%s][%s]=%.6g" % (k, cn, sum(v) / len(v)))
        if "FETCH_SIZE" in cs and "WRITE_SIZE" in cs and len(factors) == 2:
            fb = sum(cs["FETCH_SIZE"]) / len(cs["FETCH_SIZE"]) * factors["FETCH_SIZE"] * 1024
            wb = sum(cs["WRITE_SIZE"]) / len(cs["WRITE_SIZE"]) * factors["WRITE_SIZE"] * 1024
            out.append("traffic_bytes_per_launch[%s]=%.6g" % (k, fb + wb))
        for t in ("F64", "F32", "BF16"):
            v = cs.get("SQ_INSTS_VALU_MFMA_MOPS_" + t)
            if v:   # each MOPS unit is 512 floating-point operations
                out.append("mfma_%s_flop_per_launch[%s]=%.6g" % (t.lower(), k, sum(v) / len(v) * 512))
    path = os.path.join(ROOT, "profiles", "counters_%s_%s.txt" % (args.workload, args.precision))
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    print(path)


def read_counter_rows(path):
    """(dispatch id, kernel name, counter name, value, duration ns) of every
    counter record of one rocprofv3 --pmc run, in dispatch order, from its
    counter_collection.csv (-f csv) or its rocpd database (-f rocpd).  A
    counter that the profiler reports per hardware instance is summed over
    them."""
    from collections import defaultdict
    acc = defaultdict(float)
    meta = {}
    if path.endswith(".csv"):
        import csv
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                did = int(r["Dispatch_Id"])
                key = (did, r["Kernel_Name"], r["Counter_Name"])
                acc[key] += float(r["Counter_Value"])
                meta[key] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    else:
        import sqlite3
        con = sqlite3.connect(path)
        for did, kn, cn, v, dur in con.execute("select dispatch_id, kernel_name, counter_name, value, duration "
                                               "from counters_collection"):
            acc[(did, kn, cn)] += v
            meta[(did, kn, cn)] = dur
    return sorted((k[0], k[1], k[2], v, meta[k]) for k, v in acc.items())


def kernel_sources_digest():
    """Digest of the sources that define the kernels and their launch plans:
    counter readings stored under profiles/ apply only while it is unchanged."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "plan.h", "layout.cpp", "engine.hip"):
        with open(os.path.join(ROOT, "paper_2212_11973_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, args):
    """HBM bytes per launch of the dominant kernel from the rocprofv3 counter
    summary under profiles/ (FETCH_SIZE + WRITE_SIZE per dispatch, each scaled
    by the factor a copy of known size gives), or None if there is none for
    this kernel and workload or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "counters_%s_%s.txt" % (args.workload, args.precision))
    if not os.path.exists(path):
        return None, "no counter summary for this workload"
    vals = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("sources_digest") != kernel_sources_digest():
        return None, "%s was taken on other kernel sources" % os.path.basename(path)
    key = "traffic_bytes_per_launch[%s]" % kernel
    if key not in vals:
        return None, "%s has no entry for %s" % (os.path.basename(path), kernel)
    return float(vals[key]), os.path.basename(path)


def heff_bench(args, T, WL, torch):
    """The dense effective-Hamiltonian apply at D = --heff-D in each precision of
    --heff-precisions (and the two-site generator at --heff2-D), timed with the
    library's events per stage."""
    # dense effective-Hamiltonian apply at D (microbenchmark)
    heff = {}
    Dh, DH = args.heff_D, 18
    if Dh > 0:
        L, W, A, R = WL.heff_inputs(Dh, DH)
        dev = torch.device("cuda:0")
        tl, tw, ta, tr = (torch.from_numpy(x).to(dev) for x in (L, W, A, R))
        out = torch.empty_like(ta)
        fl = 32.0 * DH * Dh * Dh * (2 * Dh) + 128.0 * DH * DH * Dh * Dh
        sm = torch.cuda.current_stream().cuda_stream
        # MFMA work per FP64-equivalent flop and the roof it runs against: the
        # split-BF16 modes take 3 or 6 BF16 part products per product
        heff_roof = dict(fp64=(1, PEAK["fp64"]), fp32=(1, PEAK["fp32"]), bf16x3=(3, PEAK["bf16"]),
                         bf16x6=(6, PEAK["bf16"]))
        ref64 = None
        for pname in args.heff_precisions.split(","):
            p = PREC[pname]
            T.tt_heff_apply(Dh, Dh, DH, tl.data_ptr(), tw.data_ptr(), ta.data_ptr(), tr.data_ptr(), out.data_ptr(), p, sm)
            torch.cuda.synchronize()
            ms = []
            for _ in range(args.heff_reps):
                T.tt_heff_apply(Dh, Dh, DH, tl.data_ptr(), tw.data_ptr(), ta.data_ptr(), tr.data_ptr(), out.data_ptr(),
                                p, sm)
                ms.append(T.tt_heff_last_timing())
            med = statistics.median(x[3] for x in ms)
            tf = fl / (med * 1e-3) / 1e12
            mult, peak = heff_roof[pname]
            heff[pname] = dict(ms=med, tflops=tf, applies_per_s=1e3 / med, mfma_tflops=tf * mult,
                               frac_mfma_peak=tf * mult / peak, mfma_peak=peak,
                               stage_ms=[statistics.median(x[i] for x in ms) for i in range(3)])
            if pname == "fp64":
                ref64 = out.clone()
            elif ref64 is not None:   # the FP64 apply's result (itself held to 1e-12 of the oracle by the tests)
                heff[pname]["rel_err_vs_fp64"] = (torch.linalg.norm(out - ref64) / torch.linalg.norm(ref64)).item()
        if "fp64" in heff:
            for pname in heff:
                if pname != "fp64":
                    heff[pname]["speedup_vs_fp64"] = heff["fp64"]["ms"] / heff[pname]["ms"]
        del ref64
        print("heff done", file=sys.stderr, flush=True)
        del tl, tw, ta, tr, out
    D2 = args.heff2_D
    if D2 > 0:   # two-site generator: four grouped GEMMs (L.C, W1, W2, .R)
        L, W1, W2, C2, R = WL.heff2_inputs(D2, D2, DH, 20221223)
        dev = torch.device("cuda:0")
        tt_ = [torch.from_numpy(x).to(dev) for x in (L, W1, W2, C2, R)]
        out = torch.empty_like(tt_[3])
        sm = torch.cuda.current_stream().cuda_stream
        ptrs = [x.data_ptr() for x in tt_]
        T.tt_heff2_apply(D2, D2, DH, *ptrs, out.data_ptr(), T.TT_FP64, sm)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(args.heff_reps):
            e0.record()
            T.tt_heff2_apply(D2, D2, DH, *ptrs, out.data_ptr(), T.TT_FP64, sm)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        # flops of the contraction in the paper's order (L.C, W1, W2, .R)
        fl2 = 2.0 * 256 * D2 ** 3 * DH + 2.0 * 2 * 16 * 4 * D2 * D2 * DH * DH * 16 + 2.0 * 256 * D2 ** 3 * DH
        heff["two_site_fp64"] = dict(D=D2, ms=statistics.median(ms),
                                     tflops=fl2 / (statistics.median(ms) * 1e-3) / 1e12)
        print("heff2 done", file=sys.stderr, flush=True)
        del tt_, out
    return heff


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cl4x16")
    ap.add_argument("--D", type=int, default=0, help="override the bond dimension")
    ap.add_argument("--apply-form", type=int, default=2, choices=(0, 1, 2, 4),
                    help="site apply form: 0 the paper's contraction order, 1 the MPO folded into L, "
                         "2 autotuned per site (default), 4 the fused LW.A.R kernel everywhere")
    ap.add_argument("--sector-cap", type=int, default=64,
                    help="largest sector of a padded bond (0: no cap; the headline uses 64)")
    ap.add_argument("--uncapped-steps", type=int, default=1,
                    help="also time this many sweeps with no sector cap (0: skip)")
    ap.add_argument("--precision", default="fp64", choices=sorted(PREC),
                    help="precision of the timed sweep that gives 'value'")
    ap.add_argument("--mixed-precisions", default="bf16x6,fp32",
                    help="further sweep precisions timed after the main one ('' for none)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="copy this many MiB once (a known-size kernel for counter calibration)")
    ap.add_argument("--heff-D", type=int, default=2000)
    ap.add_argument("--heff-reps", type=int, default=5)
    ap.add_argument("--heff-precisions", default="fp64,fp32,bf16x6,bf16x3")
    ap.add_argument("--d4000", default="os10x10",
                    help="D=4000 workloads to time one FP64 and one FP32 sweep of ('' for none; os10x10, cl8x16)")
    ap.add_argument("--heff-only", action="store_true",
                    help="only the dense apply microbenchmark (--heff-D, --heff-precisions), one JSON line")
    ap.add_argument("--heff2-D", type=int, default=256,
                    help="also time the dense two-site 2-TDVP generator at this bond dimension (0: skip)")
    ap.add_argument("--tdvp2-sweeps", type=int, default=2,
                    help="also grow the workload from the bare rho0 with this many 2-TDVP sweeps (0: skip)")
    ap.add_argument("--tdvp2-D", type=int, default=2000, help="D_max of the 2-TDVP growth")
    ap.add_argument("--tdvp2-cutoff", type=float, default=1e-12, help="discarded-weight cutoff of the 2-TDVP splits")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graphs", action="store_true", help="replay captured sweeps (hipGraph) in the timed loop")
    ap.add_argument("--no-observables", action="store_true",
                    help="skip the entropy, specific heat and spin correlations after the timed sweeps")
    ap.add_argument("--mu-scan", type=int, default=8,
                    help="instances of the batched mu-scan on the 6x12 cylinder (0: skip)")
    ap.add_argument("--mu-scan-D", type=int, default=0, help="override the mu-scan bond dimension")
    ap.add_argument("--green-map", action="store_true",
                    help="instead of the headline: beta G(k, beta/2) over a k grid on the 10x10 open square "
                         "(U=8, mu=2, D=4000), one JSON line")
    ap.add_argument("--green-map-T", type=float, default=2.0, help="temperature of --green-map (T = 1/beta_phys)")
    ap.add_argument("--green-map-dbeta", type=float, default=0.05, help="linear step of --green-map")
    ap.add_argument("--green-map-pad", type=float, default=1e-3, help="padding noise amplitude of --green-map")
    ap.add_argument("--green-map-cap", type=int, default=64, help="sector cap of --green-map (0: none)")
    ap.add_argument("--green-map-exp-end", type=float, default=0.25,
                    help="beta where the doubling grid of --green-map hands over to the linear steps")
    ap.add_argument("--pairing-scan", action="store_true",
                    help="instead of the headline: chi_SC = Delta_p / hp on the 4x24 cylinder (U=8, hp=0.01, T=1, "
                         "Sz blocks, D=--D or 2000) for a few mu, one JSON line")
    ap.add_argument("--sweep-only", action="store_true",
                    help="time the sweep alone in a process without torch (the library's own hipMalloc and "
                         "the null stream, one HIP runtime): the form for rocprofv3 counter collection")
    ap.add_argument("--summarize-counters", nargs="+", default=None, metavar="DB",
                    help="write profiles/counters_<workload>_<precision>.txt from rocprofv3 --pmc databases of "
                         "--sweep-only runs (no GPU needed)")
    ap.add_argument("--counter-commands", default="", help="the profiler commands, recorded in the summary")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(args)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU (--gpus 1); the sweep has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.sweep_only:
        sweep_only(args)
        return

    import numpy as np
    import torch
    from paper_2212_11973_amd import tantrg as T
    from paper_2212_11973_amd import workloads as WL

    torch.cuda.set_device(0)
    T.lib()
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.heff_only:
        heff = heff_bench(args, T, WL, torch)
        print(json.dumps({"heff": heff, "D": args.heff_D, "D_H": 18, "data": "synthetic N(0,1) tensors, seeded"}))
        return
    if args.green_map:
        green_map(args, T, WL)
        return
    if args.pairing_scan:
        pairing_scan(args, T)
        return
    c = WL.MODELS[args.workload]
    D = args.D or c["D"]
    m = T.model(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"])

    def timed_sweeps(prec, steps, warmup, profile, cap=None):
        """warmup sweeps, `steps` timed sweeps (value), then with profile the same
        number of sweeps again with HIP events around every grouped launch (the
        events cost host time per launch, so they stay out of the timed value)."""
        o = T.options(D=D, symmetry=1, beta0=c["beta0"], pad_eps=1e-3, seed=1, krylov_dim=c["krylov"],
                      precision=PREC[prec], sector_cap=args.sector_cap if cap is None else cap)
        print("init %s D=%d %s" % (args.workload, D, prec), file=sys.stderr, flush=True)
        st = T.State.init(m, o)
        t_tune = time.perf_counter()
        forms = st.tune_apply(args.apply_form)   # the per-site apply form (autotuned by default)
        t_tune = time.perf_counter() - t_tune
        info = st.info() + (dict(apply_form=args.apply_form,
                                 site_forms_0_1_2=[sum(f & 3 == i for f in forms) for i in (0, 1, 2)],
                                 fused_bonds=sum(f >> 2 for f in forms), tune_s=t_tune),)
        T.tt_sweep_graphs(args.graphs)   # the first sweep of a step captures, later ones replay
        for i in range(warmup):
            st.sweep(c["dbeta"])
            print("warmup %d done" % i, file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        stats = []
        t0 = time.perf_counter()
        for i in range(steps):
            stats.append(st.sweep(c["dbeta"], stats=True))
            print("step %d done" % i, file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof, prof_s, phases = None, None, None
        if profile:
            # one pass with per-phase device timing (events around every phase occurrence)
            T.tt_phase_timing(True)
            ph = [st.sweep(c["dbeta"], stats=True) for _ in range(steps)]
            T.tt_phase_timing(False)
            phases = {k: statistics.mean(getattr(x, k) for x in ph)
                      for k in ("t_heff", "t_bond", "t_lanczos", "t_qr", "t_env", "t_absorb")}
            print("phase-timed steps done", file=sys.stderr, flush=True)
            T.tt_profile_enable(True)
            t2 = time.perf_counter()
            for i in range(steps):
                st.sweep(c["dbeta"])
                print("profiled step %d done" % i, file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            prof_s = (time.perf_counter() - t2) / steps
            T.tt_profile_enable(False)
            prof = T.tt_profile_read()
        else:
            for i in range(2 * steps):   # same final beta as the profiled run, for the observable comparison
                st.sweep(c["dbeta"])
        T.tt_sweep_graphs(False)
        obs = st.observables()
        thermo = None
        if profile and not args.no_observables:   # two more sweeps after the timed region: entropy and specific heat
            series = [obs]
            for _ in range(2):
                st.sweep(c["dbeta"])
                series.append(st.observables())
            bp = [o_["beta_phys"] for o_ in series]
            ce, se = T.tt_thermo_derived(bp, [o_["e"] for o_ in series], [o_["f"] for o_ in series])
            spin = {}
            for d2 in (1, 2, 4):   # spin correlation F(d), d = 1, sqrt 2, 2, at the last beta
                F_, npairs = st.spin_correlation(d2)
                spin["d2=%d" % d2] = dict(F=F_, pairs=npairs)
            green = {}   # G(k, beta_phys/2) at a few momenta (x along the length, y around the cylinder)
            tg = time.perf_counter()
            for name, kx, ky in (("0,0", 0.0, 0.0), ("pi/2,pi/2", math.pi / 2, math.pi / 2),
                                 ("pi,0", math.pi, 0.0), ("pi,pi/2", math.pi, math.pi / 2)):
                G_ = st.green_function(kx, ky)
                green[name] = dict(G=G_, beta_G=bp[-1] * G_)
            green["seconds_per_k"] = (time.perf_counter() - tg) / 4
            thermo = dict(beta_phys=bp, e=[o_["e"] for o_ in series], f=[o_["f"] for o_ in series],
                          c_e=ce, s_e=se, spin_correlation=spin, green_k=green)
        st.free()
        return (t1 - t0) / steps, stats, (prof, prof_s, phases), obs, info, thermo

    s_per_step, stats, (prof, prof_s_per_step, phases), obs, (n_sites, dims, forms_info), thermo = timed_sweeps(
        args.precision, args.steps, args.warmup, True)
    flops_step = statistics.mean(s.flops_alg for s in stats)
    applies_step = statistics.mean(s.n_applies for s in stats)
    bytes_min_step = statistics.mean(s.bytes_min for s in stats)
    launches_step = statistics.mean(s.n_launches for s in stats)
    mixed = {}
    for pname in [x for x in args.mixed_precisions.split(",") if x and x != args.precision]:
        sp, st2, _, ob2, _, _ = timed_sweeps(pname, args.steps, args.warmup, False)
        mixed[pname] = dict(s_per_step=sp, f=ob2["f"], e=ob2["e"],
                            rel_df_vs_main=abs(ob2["f"] - obs["f"]) / max(abs(obs["f"]), 1e-2),
                            rel_de_vs_main=abs(ob2["e"] - obs["e"]) / max(abs(obs["e"]), 1e-2))
    # the same sweep with the sectors uncapped (every sector at its share of D
    # up to its maximal dimension): the method's bond space without the cap,
    # at the cost the cap saves
    uncapped = None
    if args.uncapped_steps > 0 and args.sector_cap != 0:
        su, stu, _, obu, (_, dims_u, _), _ = timed_sweeps(args.precision, args.uncapped_steps, 1, False, cap=0)
        uncapped = dict(s_per_step=su, steps=args.uncapped_steps, warmup=1, max_bond=max(dims_u),
                        flops_alg_per_step=statistics.mean(x.flops_alg for x in stu), f=obu["f"], e=obu["e"])

    # the D=4000 lattices (the 10x10 open square by default): one sweep in FP64
    # and one in the FP32 mode, each after a warmup sweep and from a state of its
    # own (12-13 GB of site tensors and environments, resident in HBM)
    d4000 = {}
    for wname in [x for x in args.d4000.split(",") if x]:
        c5 = WL.MODELS[wname]
        m5 = T.model(c5["W"], c5["L"], c5["geometry"], c5["t"], c5["U"], c5["mu"])
        res = dict(workload="%s, U=%g, mu=%g, U(1)xU(1) D=%d (sector cap %d), d_beta=%g, Krylov %d"
                   % (wname, c5["U"], c5["mu"], c5["D"], args.sector_cap, c5["dbeta"], c5["krylov"]))
        for pname in ("fp64", "fp32"):
            o5 = T.options(D=c5["D"], symmetry=1, beta0=c5["beta0"], pad_eps=1e-3, seed=1, krylov_dim=c5["krylov"],
                           precision=PREC[pname], sector_cap=args.sector_cap)
            print("init %s D=%d %s" % (wname, c5["D"], pname), file=sys.stderr, flush=True)
            st5 = T.State.init(m5, o5)
            st5.tune_apply(args.apply_form)
            st5.sweep(c5["dbeta"])
            torch.cuda.synchronize()
            t5 = time.perf_counter()
            s5 = st5.sweep(c5["dbeta"], stats=True)
            torch.cuda.synchronize()
            dt5 = time.perf_counter() - t5
            ob5 = st5.observables()
            res[pname] = dict(s_per_step=dt5, tflops_alg=s5.flops_alg / dt5 / 1e12,
                              frac_fp64_mfma=s5.flops_alg / dt5 / 1e12 / PEAK["fp64"], f=ob5["f"], e=ob5["e"],
                              max_bond=max(st5.info()[1]))
            st5.free()
            print("%s %s sweep: %.2f s" % (wname, pname, dt5), file=sys.stderr, flush=True)
        res["fp32"]["speedup_vs_fp64"] = res["fp64"]["s_per_step"] / res["fp32"]["s_per_step"]
        res["fp32"]["rel_de_vs_fp64"] = abs(res["fp32"]["e"] - res["fp64"]["e"]) / max(abs(res["fp64"]["e"]), 1e-2)
        res["fp32"]["rel_df_vs_fp64"] = abs(res["fp32"]["f"] - res["fp64"]["f"]) / max(abs(res["fp64"]["f"]), 1e-2)
        d4000[wname] = res

    # dominant single kernel of the timed region and its roofline.  A
    # contraction kernel (grouped GEMM) is priced against the MFMA peak of the
    # type it multiplies in (algorithmic flops, sum of 2mnk, over its event
    # time); the W stage against HBM (its algorithmic bytes); the QR against
    # the FP64 vector peak
    singles = [k for k in prof if k.startswith("k_gemm_") or k in ("k_wgemm", "k_fused", "wstage", "qr")]
    kind = max(singles, key=lambda k: prof[k]["ms"])
    pk = prof[kind]
    sec = pk["ms"] * 1e-3
    is_mfma = (kind.startswith("k_gemm_") and kind != "k_gemm_reduce") or kind in ("k_wgemm", "k_fused")
    if is_mfma:
        # the wave GEMM multiplies in FP64 in every mode; the fused apply runs in FP64 states only
        pname = "fp64" if (args.precision == "fp64" or kind in ("k_wgemm", "k_fused")) else (
            "fp32" if args.precision == "fp32" else "bf16")
        roof = dict(bound="mfma", unit="TFLOP/s", peak=PEAK[pname], achieved=pk["flops"] / sec / 1e12)
    elif kind == "qr":
        roof = dict(bound="alu", unit="TFLOP/s", peak=PEAK_FP64_VALU, achieved=pk["flops"] / sec / 1e12)
    else:
        roof = dict(bound="hbm", unit="GB/s", peak=PEAK_HBM_GBS, achieved=pk["bytes"] / sec / 1e9)
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = kernel_name(kind, PREC[args.precision])
    roof["avg_launch_ms"] = pk["ms"] / max(pk["launches"], 1)
    roof["launches"] = pk["launches"]
    roof["alg_flops_per_launch"] = pk["flops"] / max(pk["launches"], 1)
    roof["alg_bytes_per_launch"] = pk["bytes"] / max(pk["launches"], 1)
    roof["share_of_step"] = pk["ms"] / (prof_s_per_step * 1e3 * args.steps)
    roof["profiled_s_per_step"] = prof_s_per_step
    roof["traffic"], roof["traffic_source"] = measured_traffic(roof["kernel"], args)
    kernels = {k: dict(ms_per_step=v["ms"] / args.steps, launches_per_step=v["launches"] / args.steps,
                       tflops=(v["flops"] / (v["ms"] * 1e-3) / 1e12) if v["ms"] > 0 else 0.0,
                       gbs=(v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else 0.0)
               for k, v in prof.items()}

    # batched mu-scan: instances with identical plans advance in shared launches
    mu_scan = None
    if args.mu_scan > 0:
        c4 = WL.MODELS["cl6x12"]
        D4 = args.mu_scan_D or c4["D"]
        mus = WL.MU_SCAN[:args.mu_scan]
        o4 = T.options(D=D4, symmetry=1, beta0=c4["beta0"], pad_eps=1e-3, seed=1, krylov_dim=c4["krylov"],
                       precision=PREC[args.precision])
        print("init mu-scan: %d x 6x12 cylinder D=%d" % (len(mus), D4), file=sys.stderr, flush=True)
        sts = [T.State.init(T.model(c4["W"], c4["L"], c4["geometry"], c4["t"], c4["U"], mu), o4) for mu in mus]
        forms4 = sts[0].tune_apply(args.apply_form)   # one instance's choice for the whole batch
        for st in sts[1:]:
            st.tune_apply(3, forms4)
        hs = [st.h for st in sts]
        T.tdvp_sweep_batch(hs, c4["dbeta"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fl = 0.0
        for i in range(args.steps):
            fl += T.tdvp_sweep_batch(hs, c4["dbeta"], stats=True).flops_alg
        torch.cuda.synchronize()
        s_batch = (time.perf_counter() - t0) / args.steps
        print("mu-scan batch done", file=sys.stderr, flush=True)
        # observables of every instance at the same beta, before instance 0 is timed alone
        dens = [st.observables() for st in sts]
        locs = [st.local_observables() for st in sts]
        f_nn = [st.spin_correlation(1)[0] for st in sts]
        t0 = time.perf_counter()
        for i in range(args.steps):
            sts[0].sweep(c4["dbeta"])
        torch.cuda.synchronize()
        s_single = (time.perf_counter() - t0) / args.steps
        for st in sts:
            st.free()
        # compressibility chi = dn/dmu from neighbouring instances (centred differences)
        ns = [lo["n"] for lo in locs]
        chi = [(ns[i + 1] - ns[i - 1]) / (mus[i + 1] - mus[i - 1]) for i in range(1, len(mus) - 1)]
        mu_scan = dict(workload="Hubbard 6x12 cylinder, U=8, U(1)xU(1) D=%d, d_beta=%g, mu = %s"
                       % (D4, c4["dbeta"], ", ".join("%.4g" % m for m in mus)),
                       instances=len(mus), site_forms_0_1_2=[sum(f & 3 == i for f in forms4) for i in (0, 1, 2)],
                       fused_bonds=sum(f >> 2 for f in forms4),
                       batched_s_per_step=s_batch, s_per_instance_step=s_batch / len(mus),
                       single_instance_s_per_step=s_single, speedup_vs_one_at_a_time=s_single * len(mus) / s_batch,
                       tflops_alg=fl / args.steps / s_batch / 1e12,
                       frac_fp64_mfma=fl / args.steps / s_batch / 1e12 / PEAK["fp64"],
                       beta_phys=dens[0]["beta_phys"], e_per_site=[d["e"] for d in dens],
                       s_per_site=[d["beta_phys"] * (d["e"] - d["f"]) for d in dens], n_per_site=ns,
                       docc_per_site=[lo["docc"] for lo in locs], chi_dn_dmu=chi, spin_corr_nn=f_nn)
        if args.precision == "fp64":
            # the mixed-precision batched form: the same scan with FP32 contractions
            o32 = T.options(D=D4, symmetry=1, beta0=c4["beta0"], pad_eps=1e-3, seed=1, krylov_dim=c4["krylov"],
                            precision=PREC["fp32"])
            print("init mu-scan fp32", file=sys.stderr, flush=True)
            s32 = [T.State.init(T.model(c4["W"], c4["L"], c4["geometry"], c4["t"], c4["U"], mu), o32) for mu in mus]
            f32 = s32[0].tune_apply(args.apply_form)
            for st in s32[1:]:
                st.tune_apply(3, f32)
            h32 = [st.h for st in s32]
            T.tdvp_sweep_batch(h32, c4["dbeta"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fl32 = 0.0
            for i in range(args.steps):
                fl32 += T.tdvp_sweep_batch(h32, c4["dbeta"], stats=True).flops_alg
            torch.cuda.synchronize()
            s_b32 = (time.perf_counter() - t0) / args.steps
            e32 = [st.observables()["e"] for st in s32]
            for st in s32:
                st.free()
            print("mu-scan fp32 batch done", file=sys.stderr, flush=True)
            tf32 = fl32 / args.steps / s_b32 / 1e12
            mu_scan.update(fp32_batched_tflops_alg=tf32,
                           # the wave GEMM multiplies in FP64 in both forms: the FP64 MFMA roof
                           fp32_batched_frac_fp64_mfma=tf32 / PEAK["fp64"],
                           fp32_batched_s_per_instance_step=s_b32 / len(mus),
                           fp32_batched_speedup_vs_fp64_one_at_a_time=s_single * len(mus) / s_b32,
                           fp32_max_rel_de_vs_fp64=max(abs(a - b) / max(abs(b), 1e-2)
                                                       for a, b in zip(e32, [d_["e"] for d_ in dens])))

    heff = heff_bench(args, T, WL, torch)

    # 2-TDVP growth (the exponential stage's bond growth): the headline lattice
    # from the bare rho0, steps of d_beta doubling from beta0, D_max and the
    # discarded-weight cutoff as given
    tdvp2 = None
    if args.tdvp2_sweeps > 0:
        o2 = T.options(D=1, symmetry=1, beta0=c["beta0"], pad_eps=0.0, krylov_dim=c["krylov"])
        st2 = T.State.init(m, o2)
        recs = []
        b = c["beta0"]
        for i in range(args.tdvp2_sweeps):
            torch.cuda.synchronize()
            T.tt_phase_timing(i == args.tdvp2_sweeps - 1)   # device time per phase in the last sweep
            t0 = time.perf_counter()
            s2 = st2.sweep2(b, args.tdvp2_D, args.tdvp2_cutoff, stats=True)   # synchronises
            dt = time.perf_counter() - t0
            T.tt_phase_timing(False)
            b *= 2.0
            recs.append(dict(seconds=dt, max_bond=max(st2.info()[1]), discarded=s2.discarded,
                             flops_alg=s2.flops_alg, n_launches=s2.n_launches,
                             device_ms={k: getattr(s2, k) for k in ("t_heff", "t_bond", "t_lanczos", "t_qr",
                                                                    "t_env", "t_absorb")}))
            print("tdvp2 sweep %d: %.2f s, max bond %d" % (i, dt, recs[-1]["max_bond"]), file=sys.stderr, flush=True)
        o = st2.observables()
        t0 = time.perf_counter()
        st2.sweep(c["dbeta"])   # the one-site sweep on the grown bonds
        torch.cuda.synchronize()
        t_one = time.perf_counter() - t0
        tdvp2 = dict(workload="%s from the bare rho0 (beta0 = %g), d_beta doubling, D_max %d, cutoff %g"
                     % (args.workload, c["beta0"], args.tdvp2_D, args.tdvp2_cutoff),
                     sweeps=recs, beta_phys=o["beta_phys"], f=o["f"], e=o["e"],
                     bond_dims=st2.info()[1], one_site_sweep_s_after=t_one)
        st2.free()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(c, D, args.sector_cap)

    line = {
        "metric": "TDVP beta-sweep s/step & H_eff TFLOP/s (FP64 vs split-BF16) at D=2000",
        "value": s_per_step,
        "unit": "s/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": s_per_step * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64", "bf16x6": "bf16x6+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "Hubbard %dx%d %s, U=%g, mu=%g, U(1)xU(1) D=%d (%s), d_beta=%g, Krylov %d"
                   % (c["W"], c["L"], "cylinder" if c["geometry"] == 1 else "open square", c["U"], c["mu"], D,
                      "sector cap %d" % args.sector_cap if args.sector_cap else "no sector cap",
                      c["dbeta"], c["krylov"]),
                   "sector_cap": args.sector_cap,
                   "n_sites": n_sites, "max_bond": max(dims), "parallelism": "single GPU"},
        "sweep": {"precision": args.precision, "flops_alg_per_step": flops_step,
                  "tflops_alg": flops_step / s_per_step / 1e12,
                  "applies_per_step": applies_step, "applies_per_s": applies_step / s_per_step,
                  "launches_per_step": launches_step,
                  "apply_min_bytes_per_step": bytes_min_step,
                  "phase_ms_per_step": phases,
                  "apply_forms": forms_info,
                  "kernels": kernels, "beta_end": obs["beta"], "f": obs["f"], "e": obs["e"],
                  "thermo": thermo, "other_precisions": mixed, "uncapped": uncapped, "d4000": d4000},
        "heff": {"D": args.heff_D, "D_H": 18, **heff},
        "mu_scan": mu_scan,
        "tdvp2": tdvp2,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
