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
    return {"k_gemm_reduce": "tt::k_gemm_reduce", "k_wgemm": "tt::k_wgemm", "wstage": "tt::k_wstage",
            "qr": "tt::k_qr_chunk + k_qr_stack + k_qr_combine + k_qr_wide"}[kind]


def dense_sweep_flops(dims, DH, K):
    """Dense-equivalent flops of one sweep (what a dense contraction of the same
    bond dimensions costs): site applies, bond applies, environments, QR."""
    N = len(dims) - 1
    def h1(Dl, Dr):
        return 32.0 * DH * Dl * Dr * (Dl + Dr) + 128.0 * DH * DH * Dl * Dr
    f = 0.0
    for k in range(N):                       # 2N-1 site exponentials
        f += (2 if k < N - 1 else 1) * K * h1(dims[k], dims[k + 1])
    for k in range(1, N):                    # 2N-2 bond exponentials, 2N-2 environments, QR
        D = dims[k]
        f += 2 * K * 4.0 * D ** 3 * DH
        f += h1(dims[k - 1], dims[k]) + h1(dims[k], dims[k + 1])
        f += 2 * (4.0 * 16 * D * D * D)
    return f


def cpu_baseline(D, DH):
    """The oracle's dense apply at D on the host (bounded sample)."""
    import numpy as np
    from oracle import tdvp as otd
    from paper_2212_11973_amd import workloads as WL
    L, W, A, R = WL.heff_inputs(D, DH)
    t0 = time.perf_counter()
    otd.heff1(L, W, R, A)
    t = time.perf_counter() - t0
    flops = 32.0 * DH * D * D * (2 * D) + 128.0 * DH * DH * D * D
    return t, flops


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
    --calib-copy-mib, one device-to-device copy of that size runs first (the
    runtime's own copy kernel), the reference for HBM byte counters."""
    import ctypes
    from paper_2212_11973_amd import tantrg as T
    from paper_2212_11973_amd import workloads as WL
    T.lib(init_torch=False)
    if args.calib_copy_mib > 0:
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
    c = WL.MODELS[args.workload]
    D = args.D or c["D"]
    m = T.model(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"])
    o = T.options(D=D, symmetry=1, beta0=c["beta0"], pad_eps=1e-3, seed=1, krylov_dim=c["krylov"],
                  precision=PREC[args.precision], sector_cap=args.sector_cap)
    print("init %s D=%d %s (no torch)" % (args.workload, D, args.precision), file=sys.stderr, flush=True)
    st = T.State.init(m, o)
    for i in range(args.warmup):
        st.sweep(c["dbeta"], stats=True)
        print("warmup %d done" % i, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        stats.append(st.sweep(c["dbeta"], stats=True))   # returns after the stream is synchronised
        print("step %d done" % i, file=sys.stderr, flush=True)
    s_step = (time.perf_counter() - t0) / args.steps
    obs = st.observables()
    st.free()
    print(json.dumps({"metric": "s/step (sweep only, no torch)", "value": s_step, "unit": "s/step",
                      "steps": args.steps, "warmup": args.warmup, "precision": args.precision,
                      "sector_cap": args.sector_cap,
                      "workload": "%s D=%d" % (args.workload, D),
                      "flops_alg_per_step": statistics.mean(x.flops_alg for x in stats),
                      "applies_per_step": statistics.mean(x.n_applies for x in stats),
                      "f": obs["f"], "e": obs["e"]}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cl4x16")
    ap.add_argument("--D", type=int, default=0, help="override the bond dimension")
    ap.add_argument("--sector-cap", type=int, default=64,
                    help="largest sector of a padded bond (0: no cap; the headline uses 64)")
    ap.add_argument("--precision", default="fp64", choices=sorted(PREC),
                    help="precision of the timed sweep that gives 'value'")
    ap.add_argument("--mixed-precisions", default="bf16x6,fp32",
                    help="further sweep precisions timed after the main one ('' for none)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="copy this many MiB once (a known-size kernel for counter calibration)")
    ap.add_argument("--heff-D", type=int, default=2000)
    ap.add_argument("--heff-reps", type=int, default=5)
    ap.add_argument("--heff-precisions", default="fp64,fp32,bf16x6,bf16x3")
    ap.add_argument("--heff2-D", type=int, default=256,
                    help="also time the dense two-site 2-TDVP generator at this bond dimension (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graphs", action="store_true", help="replay captured sweeps (hipGraph) in the timed loop")
    ap.add_argument("--no-observables", action="store_true",
                    help="skip the entropy, specific heat and spin correlations after the timed sweeps")
    ap.add_argument("--cpu-D", type=int, default=1500, help="bond dimension of the oracle sample")
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
    args = ap.parse_args()
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
    if args.green_map:
        green_map(args, T, WL)
        return
    if args.pairing_scan:
        pairing_scan(args, T)
        return
    c = WL.MODELS[args.workload]
    D = args.D or c["D"]
    m = T.model(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"])

    def timed_sweeps(prec, steps, warmup, profile):
        """warmup sweeps, `steps` timed sweeps (value), then with profile the same
        number of sweeps again with HIP events around every grouped launch (the
        events cost host time per launch, so they stay out of the timed value)."""
        o = T.options(D=D, symmetry=1, beta0=c["beta0"], pad_eps=1e-3, seed=1, krylov_dim=c["krylov"],
                      precision=PREC[prec])
        print("init %s D=%d %s" % (args.workload, D, prec), file=sys.stderr, flush=True)
        st = T.State.init(m, o)
        info = st.info()
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
        prof, prof_s = None, None
        if profile:
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
            for i in range(steps):   # same final beta as the profiled run, for the observable comparison
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
        return (t1 - t0) / steps, stats, (prof, prof_s), obs, info, thermo

    s_per_step, stats, (prof, prof_s_per_step), obs, (n_sites, dims), thermo = timed_sweeps(
        args.precision, args.steps, args.warmup, True)
    flops_step = statistics.mean(s.flops_alg for s in stats)
    applies_step = statistics.mean(s.n_applies for s in stats)
    mixed = {}
    for pname in [x for x in args.mixed_precisions.split(",") if x and x != args.precision]:
        sp, st2, _, ob2, _, _ = timed_sweeps(pname, args.steps, args.warmup, False)
        mixed[pname] = dict(s_per_step=sp, f=ob2["f"], e=ob2["e"],
                            rel_df_vs_main=abs(ob2["f"] - obs["f"]) / max(abs(obs["f"]), 1e-2),
                            rel_de_vs_main=abs(ob2["e"] - obs["e"]) / max(abs(obs["e"]), 1e-2))

    # dominant single kernel of the timed region and its roofline: the binding
    # roof is the lower of the compute peak and arithmetic intensity x HBM peak
    singles = [k for k in prof if k.startswith("k_gemm_") or k in ("k_wgemm", "wstage", "qr")]
    kind = max(singles, key=lambda k: prof[k]["ms"])
    pk = prof[kind]
    sec = pk["ms"] * 1e-3
    is_mfma = (kind.startswith("k_gemm_") and kind != "k_gemm_reduce") or kind == "k_wgemm"
    if is_mfma:
        # the wave GEMM multiplies in FP64 in every mode
        pname = "fp64" if (args.precision == "fp64" or kind == "k_wgemm") else (
            "fp32" if args.precision == "fp32" else "bf16")
        peak_f = PEAK[pname]
    else:
        peak_f = PEAK_FP64_VALU
    ai = pk["flops"] / max(pk["bytes"], 1.0)
    if pk["flops"] > 0 and peak_f <= ai * PEAK_HBM_GBS / 1e3:
        roof = dict(bound="mfma" if is_mfma else "alu", unit="TFLOP/s", peak=peak_f,
                    achieved=pk["flops"] / sec / 1e12)
    else:
        roof = dict(bound="hbm", unit="GB/s", peak=PEAK_HBM_GBS, achieved=pk["bytes"] / sec / 1e9)
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = kernel_name(kind, PREC[args.precision])
    roof["avg_launch_ms"] = pk["ms"] / max(pk["launches"], 1)
    roof["launches"] = pk["launches"]
    roof["alg_flops_per_launch"] = pk["flops"] / max(pk["launches"], 1)
    roof["alg_bytes_per_launch"] = pk["bytes"] / max(pk["launches"], 1)
    roof["intensity_flop_per_byte"] = ai
    roof["share_of_step"] = pk["ms"] / (prof_s_per_step * 1e3 * args.steps)
    roof["profiled_s_per_step"] = prof_s_per_step
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
                       instances=len(mus), batched_s_per_step=s_batch, s_per_instance_step=s_batch / len(mus),
                       single_instance_s_per_step=s_single, speedup_vs_one_at_a_time=s_single * len(mus) / s_batch,
                       tflops_alg=fl / args.steps / s_batch / 1e12,
                       beta_phys=dens[0]["beta_phys"], e_per_site=[d["e"] for d in dens],
                       s_per_site=[d["beta_phys"] * (d["e"] - d["f"]) for d in dens], n_per_site=ns,
                       docc_per_site=[lo["docc"] for lo in locs], chi_dn_dmu=chi, spin_corr_nn=f_nn)
        if args.precision == "fp64":
            # the mixed-precision batched form: the same scan with FP32 contractions
            o32 = T.options(D=D4, symmetry=1, beta0=c4["beta0"], pad_eps=1e-3, seed=1, krylov_dim=c4["krylov"],
                            precision=PREC["fp32"])
            print("init mu-scan fp32", file=sys.stderr, flush=True)
            s32 = [T.State.init(T.model(c4["W"], c4["L"], c4["geometry"], c4["t"], c4["U"], mu), o32) for mu in mus]
            h32 = [st.h for st in s32]
            T.tdvp_sweep_batch(h32, c4["dbeta"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(args.steps):
                T.tdvp_sweep_batch(h32, c4["dbeta"])
            torch.cuda.synchronize()
            s_b32 = (time.perf_counter() - t0) / args.steps
            e32 = [st.observables()["e"] for st in s32]
            for st in s32:
                st.free()
            print("mu-scan fp32 batch done", file=sys.stderr, flush=True)
            mu_scan.update(fp32_batched_s_per_instance_step=s_b32 / len(mus),
                           fp32_batched_speedup_vs_fp64_one_at_a_time=s_single * len(mus) / s_b32,
                           fp32_max_rel_de_vs_fp64=max(abs(a - b) / max(abs(b), 1e-2)
                                                       for a, b in zip(e32, [d_["e"] for d_ in dens])))

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
            heff[pname] = dict(ms=med, tflops=fl / (med * 1e-3) / 1e12, applies_per_s=1e3 / med,
                               stage_ms=[statistics.median(x[i] for x in ms) for i in range(3)])
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

    cpu = None
    if not args.no_cpu_baseline:
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t_apply, fl_apply = cpu_baseline(args.cpu_D, DH)
        rate = fl_apply / t_apply
        est = dense_sweep_flops(dims, DH, c["krylov"]) / rate
        cpu = dict(value=est, unit="s/step", cores=nthreads, kind="oracle",
                   sample="one dense oracle H_eff apply at D=%d (%.3g flop, %.2f s, %.3g flop/s) scaled by the "
                          "dense-equivalent flops of one sweep of the same bond dimensions (%.3g flop)"
                          % (args.cpu_D, fl_apply, t_apply, rate, dense_sweep_flops(dims, DH, c["krylov"])))

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
        "config": {"workload": "Hubbard %dx%d %s, U=%g, mu=%g, U(1)xU(1) D=%d, d_beta=%g, Krylov %d"
                   % (c["W"], c["L"], "cylinder" if c["geometry"] == 1 else "open square", c["U"], c["mu"], D,
                      c["dbeta"], c["krylov"]),
                   "n_sites": n_sites, "max_bond": max(dims), "parallelism": "single GPU"},
        "sweep": {"precision": args.precision, "flops_alg_per_step": flops_step,
                  "tflops_alg": flops_step / s_per_step / 1e12,
                  "applies_per_step": applies_step, "applies_per_s": applies_step / s_per_step,
                  "kernels": kernels, "beta_end": obs["beta"], "f": obs["f"], "e": obs["e"],
                  "thermo": thermo, "other_precisions": mixed},
        "heff": {"D": Dh, "D_H": DH, **heff},
        "mu_scan": mu_scan,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
