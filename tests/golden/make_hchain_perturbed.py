"""Write the FP64 oracle run of the 64-walker, 1000-step hydrogen-chain
population (comb every 20 steps, field seed 1) started from the reference
determinant with one orbital entry of every walker changed by one unit in
the last place, phi[w, 0, 0] *= 1 + 2**-52.  Compared with the unperturbed
run in hchain-M50_W64_T1000.txt it shows how far the population-controlled
trajectory carries a rounding-sized difference: the mixed energies agree to
rounding for a while and then part, when a walker near a node amplifies the
difference and later combs pick different parents.  Only the oracle is
called.

    python tests/golden/make_hchain_perturbed.py
"""
from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SEED = 1
WORKLOAD = "hchain-M50"


def main():
    sys.path.insert(0, ROOT)
    import numpy as np

    import afqmc_synth as syn
    from oracle import Oracle, Options

    wl = syn.WORKLOADS[WORKLOAD]
    o = Oracle.from_inputs(syn.workload_system(wl))
    st = o.init_walkers(64)
    et = float(st.eloc.real[0])
    st.phi[:, 0, 0] *= 1.0 + 2.0 ** -52
    opt = Options(taylor_order=wl.taylor_order, ortho_every=wl.ortho_every,
                  pc_every=wl.pc_every, e_trial=et)
    n = 1000
    num, den = np.zeros(n), np.zeros(n)
    m = o.measure(st.phi)
    st.logS, st.eloc, st.v = m["logS"], m["eloc"], m["v"]
    for t in range(n):
        with np.errstate(all="ignore"):
            o.step(st, t, SEED, wl.dt, opt)
        num[t] = np.sum(st.weight * st.eloc.real)
        den[t] = np.sum(st.weight)
        if (t + 1) % wl.ortho_every == 0:
            o.orthonormalize(st)
        if (t + 1) % wl.pc_every == 0:
            o.reconfigure(st, SEED, t)
        if t % 50 == 0:
            print(f"step {t}", flush=True)
    with open(os.path.join(HERE, "hchain-M50_W64_T1000_ulp.txt"), "w") as f:
        f.write("# 64 walkers, 1000 steps, comb every 20 steps (pc_index = step), started from\n")
        f.write("# D_0 with phi[w, 0, 0] *= 1 + 2**-52; columns: step, sum W Re E_L, sum W\n")
        f.write(f"# FP64 oracle, workload {WORKLOAD}, field seed {SEED}; written by "
                "tests/golden/make_hchain_perturbed.py\n")
        f.write(f"e_trial {et!r}\n")
        for t in range(n):
            f.write(f"step {t} {float(num[t])!r} {float(den[t])!r}\n")


if __name__ == "__main__":
    main()
