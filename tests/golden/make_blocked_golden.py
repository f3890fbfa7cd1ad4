"""Write the stored reference values of the block-sparse oracle on the
headline workload (calls only ``oracle/``; no value comes from the HIP path).

Workload: Hubbard 4x16 cylinder (periodic across the width of 4, open along
the length of 16), t = 1, U = 8, mu = 1.5, U(1)charge x U(1)spin bonds of
D = 2000 with sector cap 64 (or none), rho0 = 1 - beta0 H at beta0 = 0.05 * 2^-12,
padding noise 1e-3 from SplitMix64 seed 1; then two symmetric 1-TDVP sweeps of
d_beta = 0.05 with Krylov dimension 8 (SM Sec. II.F, II.H), the bilayer
observables (SM Sec. II.A) after the start and after each sweep.

Run:  python tests/golden/make_blocked_golden.py [CAP]   (CAP 64 or 0, default
64; about half an hour on 8 cores; writes blocked_cl4x16_d2000.json for cap 64
and blocked_cl4x16_d2000_cap0.json for no cap, next to this file)
"""
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import blocked, mpo  # noqa: E402

CASE = dict(W=4, L=16, geometry=1, t=1.0, U=8.0, mu=1.5, D=2000, sector_cap=64,
            beta0=0.05 * 2.0 ** -12, pad_eps=1e-3, seed=1, dbeta=0.05, krylov=8, sweeps=2)


def main():
    c = dict(CASE)
    if len(sys.argv) > 1:
        c["sector_cap"] = int(sys.argv[1])
    model = mpo.HubbardMPO(c["W"], c["L"], c["geometry"], t=c["t"], U=c["U"], mu=c["mu"])
    t0 = time.perf_counter()
    st = blocked.initial_state(model, c["beta0"], c["D"], pad_eps=c["pad_eps"], seed=c["seed"],
                               sector_cap=c["sector_cap"])
    t_init = time.perf_counter() - t0
    rec = [dict(sweeps=0, **{k: float(v) for k, v in st.observables().items()}, lam=float(st.lam))]
    print("start done (%.0f s)" % t_init, file=sys.stderr, flush=True)
    secs = []
    for i in range(c["sweeps"]):
        t0 = time.perf_counter()
        st.sweep(c["dbeta"], K=c["krylov"])
        secs.append(time.perf_counter() - t0)
        rec.append(dict(sweeps=i + 1, **{k: float(v) for k, v in st.observables().items()}, lam=float(st.lam),
                        max_krylov_err=float(st.max_krylov_err)))
        print("sweep %d done (%.0f s)" % (i + 1, secs[-1]), file=sys.stderr, flush=True)
    out = dict(source="oracle.blocked (block-sparse FP64 oracle); script tests/golden/make_blocked_golden.py",
               case=c, bond_dims=[b.dim for b in st.bonds], records=rec,
               oracle_seconds=dict(start=t_init, per_sweep=secs,
                                   host=platform.processor() or platform.machine(),
                                   cpus=os.cpu_count()))
    name = "blocked_cl4x16_d2000.json" if c["sector_cap"] == 64 else "blocked_cl4x16_d2000_cap%d.json" % c["sector_cap"]
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote %s" % path, file=sys.stderr)


if __name__ == "__main__":
    main()
