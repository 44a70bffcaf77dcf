"""Write the FP64 oracle references of the hydrogen-chain workload (M = 50,
25 + 25 electrons, 250 vectors, dt = 0.005, Taylor order 6, orthonormalised
every 10 steps).

* ``hchain-M50_W1024_T100.txt``: all 1024 walkers, 100 steps, population
  control off; per step the sums sum_w W_w Re E_L,w and sum_w W_w, so
  E_mix(t) is their ratio.  Walkers are split into chunks run in separate
  processes: with no population control coupling them, the chunked run is
  the same computation as one run over all walkers.
* ``hchain-M50_W64_T1000.txt``: a population of 64 walkers, all 1000 steps,
  comb every 20 steps as in the workload; the same sums per step (taken
  before the comb), then each walker's final weight and E_L.

E_T is the reference determinant's E_L (every walker starts there), field
seed 1.  Only the oracle is called.

    python tests/golden/make_hchain_reference.py [--procs 8]
"""
from __future__ import annotations

import argparse
import os
import sys

# one BLAS thread per worker process unless the caller says otherwise (set
# before numpy is first imported)
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))

SEED = 1
WORKLOAD = "hchain-M50"


def _chunk(args):
    lo, hi, n_steps, pc = args
    sys.path.insert(0, ROOT)
    import numpy as np

    import afqmc_synth as syn
    from oracle import Oracle, Options

    wl = syn.WORKLOADS[WORKLOAD]
    o = Oracle.from_inputs(syn.workload_system(wl))
    st = o.init_walkers(hi - lo, index=np.arange(lo, hi))
    et = float(st.eloc.real[0])
    pc_every = wl.pc_every if pc else 0
    opt = Options(taylor_order=wl.taylor_order, ortho_every=wl.ortho_every, pc_every=pc_every,
                  e_trial=et)
    num = np.zeros(n_steps)
    den = np.zeros(n_steps)
    # the loop of Oracle.propagate, recording the weighted sums after every step
    for t in range(n_steps):
        with np.errstate(all="ignore"):  # a chunk whose walkers all died has no E_mix
            o.step(st, t, SEED, wl.dt, opt)
        num[t] = np.sum(st.weight * st.eloc.real)
        den[t] = np.sum(st.weight)
        if (t + 1) % wl.ortho_every == 0:
            o.orthonormalize(st)
        if pc_every and (t + 1) % pc_every == 0:
            o.reconfigure(st, SEED, t)
    return et, num, den, st.weight.copy(), st.eloc.copy()


def _run(W, n_steps, procs, pc=False):
    import multiprocessing as mp

    import numpy as np
    if pc:  # the comb couples all walkers: one process
        procs = 1
    bounds = np.linspace(0, W, min(procs, W) + 1).astype(int)
    jobs = [(int(bounds[i]), int(bounds[i + 1]), n_steps, pc) for i in range(len(bounds) - 1)]
    with mp.get_context("fork").Pool(len(jobs)) as pool:
        parts = pool.map(_chunk, jobs)
    et = parts[0][0]
    num = sum(p[1] for p in parts)
    den = sum(p[2] for p in parts)
    wts = np.concatenate([p[3] for p in parts])
    els = np.concatenate([p[4] for p in parts])
    return et, num, den, wts, els


def _write(path, header, et, num, den, wts=None, els=None):
    with open(path, "w") as f:
        for line in header:
            f.write(f"# {line}\n")
        f.write(f"e_trial {float(et)!r}\n")
        for t in range(len(num)):
            f.write(f"step {t} {float(num[t])!r} {float(den[t])!r}\n")
        if wts is not None:
            for k in range(len(wts)):
                f.write(f"walker {k} {float(wts[k])!r} {float(els[k].real)!r} "
                        f"{float(els[k].imag)!r}\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    ap.add_argument("--only", choices=["full", "subset"], default=None)
    a = ap.parse_args()
    common = [f"FP64 oracle, workload {WORKLOAD}, field seed {SEED},",
              "E_mix(t) = num / den; written by tests/golden/make_hchain_reference.py"]
    if a.only in (None, "full"):
        et, num, den, _, _ = _run(1024, 100, a.procs)
        _write(os.path.join(HERE, "hchain-M50_W1024_T100.txt"),
               ["walkers 0..1023, 100 steps, population control off;",
                "columns: step, sum W Re E_L, sum W"] + common, et, num, den)
    if a.only in (None, "subset"):
        et, num, den, wts, els = _run(64, 1000, a.procs, pc=True)
        _write(os.path.join(HERE, "hchain-M50_W64_T1000.txt"),
               ["64 walkers, 1000 steps, comb every 20 steps (pc_index = step);",
                "step lines as above (before the comb), then walker k: weight, Re E_L, Im E_L"]
               + common, et, num, den, wts, els)


if __name__ == "__main__":
    main()
