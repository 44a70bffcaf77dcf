"""Benchmark: walker-steps per second of the batched phaseless AFQMC walker update.

Workload (default): hydrogen-chain-shaped system, M = 50 orbitals, 25 + 25
electrons, 250 Cholesky vectors, 1024 walkers, dt = 0.005, 6th-order Taylor
propagator, FP32 contractions (propagator build, Ltil Theta, Taylor and B1
products) with FP64 overlaps / inverses / determinants / MGS and FP64 sums,
MGS every 10 steps, comb every 20 steps.  A step is one pass of the whole
walker update over all walkers.  Inputs are synthetic (seeded generators).

Prints one JSON line.  `value` is walker-steps/s over the timed steps with all
inputs resident in HBM.  `roofline` reports the fused exchange / force-bias
kernel (the dominant one): algorithmic flops per launch divided by its average
duration, measured with HIP events on the launch stream over the timed region.
`cpu_baseline` times the FP64 numpy oracle on a bounded sample of the same
workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def exchange_flops_per_walker(M, n_up, n_dn, G):
    """X_g = Ltil_g Theta (real N x M times complex M x N: 4 N^2 M flops) and
    Tr(X_g X_g) (N^2 complex multiply-adds: 8 N^2 flops), per spin and g."""
    return sum(G * (4 * n * n * M + 8 * n * n) for n in (n_up, n_dn))


def cpu_baseline(wl, inp, sample_walkers, sample_steps):
    from oracle import Oracle, Options as OOptions
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    o = Oracle.from_inputs(inp)
    st = o.init_walkers(sample_walkers)
    et = o.mixed_energy(st)
    opt = OOptions(taylor_order=wl.taylor_order, ortho_every=wl.ortho_every, pc_every=0, e_trial=et)
    o.propagate(st, 1, wl.dt, 0, 0, opt)  # warm caches (B1, allocations)
    t0 = time.perf_counter()
    o.propagate(st, sample_steps, wl.dt, 0, 1, opt)
    dt = time.perf_counter() - t0
    return {"value": sample_walkers * sample_steps / dt, "unit": "walker-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{sample_walkers} walkers x {sample_steps} steps of {wl.name} "
                      f"(FP64 numpy oracle, comb off), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="hchain-M50")
    ap.add_argument("--walkers", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-walkers", type=int, default=16)
    ap.add_argument("--cpu-steps", type=int, default=80)
    ap.add_argument("--tte-repeats", type=int, default=5)
    ap.add_argument("--tte-steps", type=int, default=50)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain elementwise copy of 256 MiB (reads 256 MiB, writes "
                         "256 MiB) so that HBM byte counters can be scaled")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(walker sharding is described in DESIGN.md but not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import afqmc_synth as syn
    import paper_1804_03310_amd as afq

    wl = syn.WORKLOADS[args.workload]
    W = args.walkers or wl.n_walkers
    inp = syn.workload_system(wl)
    torch.cuda.set_device(0)
    ham = afq.Hamiltonian(inp.h, inp.L, inp.e_core)
    trial = afq.Trial(ham, inp.n_up, inp.n_dn, inp.C_up, inp.C_dn)
    w = afq.Walkers(trial, W)
    afq.walkers_from_trial(ham, trial, w)
    et = afq.local_energy(ham, trial, w)
    opt = afq.Options(taylor_order=wl.taylor_order, ortho_every=wl.ortho_every,
                      pc_every=wl.pc_every, e_trial=et, chol_prec=wl.chol_prec,
                      taylor_prec=wl.taylor_prec)
    emix = torch.empty(max(args.steps, args.warmup, args.tte_steps, 1), dtype=torch.float64,
                       device="cuda")
    # warmup
    if args.warmup:
        afq.propagate(ham, trial, w, args.warmup, wl.dt, 1, 0, opt, emix=emix)
    torch.cuda.synchronize()
    for k in afq._abi.KERNEL_CLASSES:
        afq.timing_read(ham, k)
    # timed region: exactly `steps` steps in one call, kernel events on the launch stream
    afq.timing_enable(ham, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    afq.propagate(ham, trial, w, args.steps, wl.dt, 1, args.warmup, opt, emix=emix)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    afq.timing_enable(ham, False)
    ktimes = {k: afq.timing_read(ham, k) for k in afq._abi.KERNEL_CLASSES}
    e_last = float(emix[args.steps - 1].item()) if args.steps else float("nan")
    alive = int((w.weight > 0).sum().item())

    # time to energy: propagate start -> final E_mix on the host
    tte = []
    for r in range(args.tte_repeats):
        afq.walkers_from_trial(ham, trial, w)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        e = afq.propagate(ham, trial, w, args.tte_steps, wl.dt, 100 + r, 0, opt, emix=emix)
        _ = float(e[args.tte_steps - 1].item())
        tte.append(time.perf_counter() - t1)

    n_ex, ms_ex = ktimes["exchange"]
    flops = exchange_flops_per_walker(wl.M, wl.n_up, wl.n_dn, wl.n_chol) * W
    avg_s = (ms_ex / n_ex) / 1e3 if n_ex else float("nan")
    peak = FP32_PEAK_TFLOPS if wl.chol_prec == "fp32" else FP64_PEAK_TFLOPS
    achieved = flops / avg_s / 1e12 if n_ex else float("nan")
    value = W * args.steps / elapsed
    out = {
        "metric": "walker-steps/sec on 1 MI355X at <=0.1 mHa vs FP64 oracle; p50/p99 time-to-energy",
        "value": value,
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / max(args.steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl.chol_prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "M": wl.M, "n_up": wl.n_up, "n_dn": wl.n_dn,
                   "n_chol": wl.n_chol, "n_walkers": W, "dt": wl.dt,
                   "taylor_order": wl.taylor_order, "ortho_every": wl.ortho_every,
                   "pc_every": wl.pc_every,
                   "precision": f"contractions {wl.chol_prec}, Taylor/B1 {wl.taylor_prec}, "
                                "overlap/inverse/det/MGS/sums fp64",
                   "e_mix_last": e_last, "alive_walkers": alive},
        "roofline": {"bound": "mfma", "kernel": "k_exchange (fused Ltil*Theta, Tr X, Tr XX)",
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "flops_per_launch": flops, "avg_launch_ms": avg_s * 1e3, "launches": n_ex},
        "kernel_ms_per_step": {k: (v[1] / max(args.steps, 1)) for k, v in ktimes.items() if v[0]},
        "time_to_energy_s": {"p50": float(np.percentile(tte, 50)) if tte else None,
                             "p99": float(np.percentile(tte, 99)) if tte else None,
                             "repeats": len(tte), "steps": args.tte_steps},
    }
    if args.calibrate_copy:
        x = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"kernel": "torch elementwise mul (x * 1.0 -> y)",
                                   "bytes_read": x.numel() * 8, "bytes_written": y.numel() * 8}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, inp, args.cpu_walkers, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
