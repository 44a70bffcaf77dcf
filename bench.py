"""Benchmark: walker-steps per second of the batched phaseless AFQMC walker update.

Workload (default): hydrogen-chain-shaped system, M = 50 orbitals, 25 + 25
electrons, 250 Cholesky vectors, 1024 walkers, dt = 0.005, 6th-order Taylor
propagator, FP32 contractions (propagator build, Ltil Theta, Taylor and B1
products) with FP64 overlaps / inverses / determinants / MGS and FP64 sums,
MGS every 10 steps, comb every 20 steps.  A step is one pass of the whole
walker update over all walkers.  Inputs are synthetic (seeded generators).

Prints one JSON line.  `value` is walker-steps/s over the timed steps with all
inputs resident in HBM.  `roofline` reports whichever of the two matrix-core
classes takes more time per step, the exchange (quadratic form, per-vector
exchange or multi-determinant energy kernel) or the Taylor propagation (the
fused kernel, or the chain of walker-batched GEMMs where the operands do not
fit one CU): algorithmic flops per launch divided by the average launch
duration, measured with HIP events on the launch stream over the timed region;
the other class is under `roofline_other`.
`accuracy` (hydrogen-chain workload) runs all walkers for 100 steps with
population control off and compares E_mix per step with the stored FP64
oracle run under tests/golden.  `cpu_baseline` times the FP64 numpy oracle on
a bounded sample of the same workload on the host cores (BLAS threads as
the host gives them), and beside it on one thread.
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
BF16_PEAK_TFLOPS = 2500.0


def exchange_flops_per_walker(M, n_up, n_dn, G):
    """X_g = Ltil_g Theta (real N x M times complex M x N: 4 N^2 M flops) and
    Tr(X_g X_g) (N^2 complex multiply-adds: 8 N^2 flops), per spin and g."""
    return sum(G * (4 * n * n * M + 8 * n * n) for n in (n_up, n_dn))


def taylor_flops_per_walker(M, Nt, order):
    """B1 exp(A) B1 phi with the Taylor series: two real M x M times complex
    M x Nt products (4 M^2 Nt flops each) and `order` complex M x M times
    complex M x Nt products (8 M^2 Nt flops each)."""
    return (8 * order + 8) * M * M * Nt


def taylor_fused(M, Nt, prec, lds_bytes=160 * 1024):
    """Whether the propagation runs as the one fused kernel per step (its LDS
    operands fit one CU, at most 64 output tiles)."""
    mp4 = (M + 3) // 4 * 4
    ldk = mp4 if (mp4 // 4) % 2 else mp4 + 4
    elem = 4 if prec == "fp32" else 8
    ntile = ((M + 15) // 16) * ((Nt + 15) // 16)
    return (3 * M + 4 * Nt) * ldk * elem <= lds_bytes and ntile <= 64


def qform_flops_per_walker(M, n_up, n_dn):
    """Q route exchange: per spin theta^T Q theta over the K = M N_sigma index
    with Q symmetric (K (K + 1) / 2 distinct entries, each a complex-by-real
    multiply-add: 2 K (K + 1) flops)."""
    return sum(2 * (M * n) * (M * n + 1) for n in (n_up, n_dn))


def fbias_flops_per_walker(M, n_up, n_dn, G):
    """Force bias v_g = sum_k theta_k Lq[k][g] (complex 1 x M Nt times real
    M Nt x G: 4 M Nt G flops)."""
    return 4 * M * (n_up + n_dn) * G


def multidet_flops_per_walker(M, n_up, n_dn, G, rows=None):
    """Multi-determinant energy: per spin and per g (the G vectors and h),
    P_g = (C^T L_g) Theta_0 over the rows formed (all M, or the R = N +
    distinct-particle rows of the compact-row kernel: real R x M times complex
    M x N, 4 R M N flops) and X0^2 = P[:N] P[:N] (complex N x N x N: 8 N^3);
    the compact-row kernel also forms Ghat at its particle rows once (4 (R - N)
    M N).  The per-determinant corrections are O(E^2 N) and not counted."""
    f = 0
    for s, n in enumerate((n_up, n_dn)):
        if not n:
            continue
        r = M if rows is None else rows[s]
        f += (G + 1) * (4 * r * M * n + 8 * n ** 3)
        if rows is not None:
            f += 4 * (r - n) * M * n
    return f


def multidet_compact_rows(M, n_up, n_dn, exc, chol_prec):
    """Rows per spin that the FP32 compact-row energy kernel forms (N plus the
    distinct particle orbitals of the determinants), or None where the
    full-row kernel runs (FP64, or past the compact kernel's limits: M <= 128,
    N <= 16, at most 256 determinants, 4 KS RP <= 12288 with KS = 16 for
    M <= 64, else 32, and RP = R rounded up to 16)."""
    n_det = exc.shape[0]
    if chol_prec != "fp32" or M > 128 or max(n_up, n_dn) > 16 or n_det > 256:
        return None
    ks = 16 if M <= 64 else 32
    max_exc = (exc.shape[2] - 1) // 2
    rows = []
    for s, n in enumerate((n_up, n_dn)):
        parts = {int(exc[i, s, 1 + max_exc + e]) for i in range(n_det) for e in range(int(exc[i, s, 0]))}
        r = n + len(parts)
        if 4 * ks * (-(-r // 16) * 16) > 12288:
            return None
        rows.append(r)
    return rows


def resident_flops_per_walker(M, n_up, n_dn, G, order):
    """Algorithmic flops of one walker-step of the walker-resident kernel
    (real flops, complex walkers): A = sum_g c_g L_g, complex coefficients
    times real M x M (4 M^2 G); B1 twice and `order` Taylor terms
    ((8 order + 8) M^2 Nt); per spin the overlap D_0^T phi (4 M N^2), its
    inverse (8 N^3) and Theta = phi S^-1 (8 M N^2); per spin and g the
    exchange X = Ltil_g Theta (4 N^2 M) and Tr(X X) (8 N^2)."""
    Nt = n_up + n_dn
    f = 4 * M * M * G + (8 * order + 8) * M * M * Nt
    for n in (n_up, n_dn):
        f += 4 * M * n * n + 8 * n ** 3 + 8 * M * n * n + G * (4 * n * n * M + 8 * n * n)
    return f


# Systems of a batched group: (label, M, n_up, n_dn, n_chol, walkers, tau_d,
# health-scaled, ortho_every, pc_every, hamiltonian seed, field seed, system id).
# The two M = 12 members are a neutral / cation correlated-sampling pair on
# one Hamiltonian sharing one field stream (same seed and system id).
BATCHED_MIX = [
    ("plain-M10", 10, 5, 5, 40, 64, 8.0, False, 2, 0, 0, 0, 0),
    ("M12-neutral", 12, 6, 6, 36, 512, 8.0, False, 2, 0, 12, 11, 1),
    ("M12-cation", 12, 6, 5, 36, 512, 8.0, False, 2, 0, 12, 11, 1),
    ("M8", 8, 4, 4, 24, 256, 8.0, False, 2, 20, 8, 12, 2),
    ("M14", 14, 4, 3, 30, 33, 8.0, False, 3, 20, 14, 13, 3),
]


GOLDEN = {"hchain-M50": ("hchain-M50_W1024_T100.txt", 1024, 100, 1)}

TRAFFIC = {("hchain-M50", "exchange"): "hchain-M50_qform_traffic.json",
           ("hchain-M50", "taylor_b1"): "hchain-M50_taylor_traffic.json",
           ("tm-multidet-M120", "exchange"): "tm-multidet-M120_md_traffic.json",
           ("sweep-M200", "exchange"): "sweep-M200_bf16x3_exchange_traffic.json"}


def measured_traffic(wl_name, cls, chol_prec, taylor_prec):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (scaled by the copy-kernel calibration), or
    None when there is none for this workload and precision or the kernel
    source has changed since the counters were taken."""
    import hashlib
    name = TRAFFIC.get((wl_name, cls))
    path = os.path.join(ROOT, "profiles", name) if name else None
    if path is None or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    prec = taylor_prec if cls == "taylor_b1" else chol_prec
    if rec["prec"] != prec or rec["source_sha256"] != digest:
        return None
    return rec["hbm_bytes_per_launch"]


def read_golden(fname):
    et, num, den = None, [], []
    with open(os.path.join(ROOT, "tests", "golden", fname)) as f:
        for line in f:
            p = line.split()
            if not p or p[0] == "#":
                continue
            if p[0] == "e_trial":
                et = float(p[1])
            elif p[0] == "step":
                num.append(float(p[2]))
                den.append(float(p[3]))
    return et, np.array(num) / np.array(den)


def accuracy_check(afq, torch, wl, inp, ham, trial, opt_kw):
    """E_mix per step, all walkers, population control off, vs the stored
    FP64 oracle run of the same workload and fields."""
    fname, W, n_steps, seed = GOLDEN[wl.name]
    et, ref = read_golden(fname)
    w = afq.Walkers(trial, W)
    afq.walkers_from_trial(ham, trial, w)
    opt = afq.Options(e_trial=et, pc_every=0, **opt_kw)
    em = afq.propagate(ham, trial, w, n_steps, wl.dt, seed, 0, opt).cpu().numpy()
    err = np.abs(em - ref)
    return {"max_abs_dEmix_Ha": float(err.max()), "final_abs_dEmix_Ha": float(err[-1]),
            "gate_Ha": 1e-4, "pass": bool(err.max() <= 1e-4),
            "walkers": W, "steps": n_steps, "pc": "off", "field_seed": seed,
            "e_mix_final": float(em[-1]), "alive_final": int((w.weight > 0).sum().item()),
            "reference": "FP64 oracle sums stored in tests/golden/" + fname}


def kernel_error_check(afq, torch, wl, inp, ham, trial, opt_kw, W, n_steps=5):
    """Per-step E_L error of the run's precision where no stored oracle run
    exists: the walkers after n_steps FP64 steps (population control off)
    are measured once with the run's contraction precision and once in FP64
    (the FP64 path is held to the oracle by the parity tests at this size);
    the largest |dE_L| over the live walkers, in Ha, against the 0.1 mHa
    gate."""
    w = afq.Walkers(trial, W)
    afq.walkers_from_trial(ham, trial, w)
    kw = dict(opt_kw)
    prec = kw.pop("chol_prec")
    kw.pop("taylor_prec")
    kw.pop("weight_mode", None)
    kw.pop("meas_every", None)
    base = afq.Options(e_trial=0.0, pc_every=0, chol_prec="fp64", taylor_prec="fp64", **kw)
    afq.propagate(ham, trial, w, n_steps, wl.dt, 7, 0, base)
    torch.cuda.synchronize()
    el64 = w.eloc[0].cpu().numpy().copy()
    alive = (w.weight > 0).cpu().numpy()
    phi_re, phi_im = w.phi_re.clone(), w.phi_im.clone()
    route = trial.exchange_route
    if prec in ("bf16", "bf16x3"):
        trial.exchange_route = "ltilde"
    afq.propagate(ham, trial, w, 0, wl.dt, 7, n_steps,
                  afq.Options(e_trial=0.0, pc_every=0, chol_prec=prec, taylor_prec="fp64", **kw))
    trial.exchange_route = route
    el = w.eloc[0].cpu().numpy()
    w.phi_re.copy_(phi_re)
    w.phi_im.copy_(phi_im)
    d = np.abs(el - el64)[alive]
    err = float(d.max()) if d.size else float("nan")
    return {"max_abs_dEL_Ha": err, "gate_Ha": 1e-4, "pass": bool(err <= 1e-4),
            "walkers": int(W), "after_steps": n_steps, "contraction_prec": prec,
            "reference": "the FP64 GPU path on the same walkers (pinned to the FP64 oracle by the "
                         "parity tests); one measurement in the run's contraction precision"}


def serving_bench(args):
    """Mixed request stream through the serving loop (paper_1804_03310_amd.serving):
    Poisson arrivals at 20 requests/s, M uniform over {20, 40, 80, 120, 160}
    with N = M/4 electrons per spin and 5M Cholesky vectors (health-scaled
    tau_d = 50 generator), W uniform over {128, 512, 2048}, FP32 contractions,
    comb every 20 steps; half the requests are neutral/cation correlated-sampling
    pairs (cation: one down electron fewer) sharing the Hamiltonian, field seed
    and system id, without population control.  Two distinct systems per M.
    Reports walker-steps/s over the whole stream, p50/p99 arrival-to-result
    latency, and whether a few requests rerun alone reproduce their mixed
    results bitwise."""
    import torch

    import afqmc_synth as syn
    from paper_1804_03310_amd.serving import Request, Server

    rng = np.random.default_rng(args.serve_seed)
    n = args.requests
    systems = {}

    def system(M, k):
        if (M, k) not in systems:
            systems[(M, k)] = syn.make_system(M, M // 4, M // 4, 5 * M, 50.0, seed=1000 * M + k,
                                              l_scale=syn.health_scale(M))
        return systems[(M, k)]

    gaps = rng.exponential(1.0 / args.rate, n)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    i = 0
    sys_id = 0
    while i < n:
        M = int(rng.choice([20, 40, 80, 120, 160]))
        W = int(rng.choice([128, 512, 2048]))
        inp = system(M, int(rng.integers(2)))
        pair = (i + 1 < n) and (i % 4 < 2)  # half of the requests, in pairs
        seed = int(rng.integers(1 << 30))
        base = dict(h=inp.h, L=inp.L, e_core=0.0, C_up=inp.C_up, C_dn=inp.C_dn, n_walkers=W,
                    n_steps=args.serve_steps, dt=0.005, seed=seed, chol_prec="fp32",
                    taylor_prec="fp32", ortho_every=2)
        if pair:
            sys_id += 1
            for n_dn in (inp.n_dn, inp.n_dn - 1):
                reqs.append(Request(n_up=inp.n_up, n_dn=n_dn, system_id=sys_id, pc_every=0,
                                    arrival=float(arrivals[i]), tag=("pair", sys_id, n_dn), **base))
                i += 1
        else:
            reqs.append(Request(n_up=inp.n_up, n_dn=inp.n_dn, system_id=0, pc_every=20,
                                arrival=float(arrivals[i]), tag=("single", i), **base))
            i += 1
    torch.cuda.set_device(0)
    srv = Server(args.serve_budget_gb << 30, max_active=args.serve_slots,
                 chunk_steps=args.serve_chunk)
    ids = [srv.submit(r) for r in reqs]
    t0 = time.perf_counter()
    reported = 0
    while srv.step():  # the server's run loop, with a progress line every 16 results
        if len(srv.results) >= reported + 16:
            reported = len(srv.results)
            print(f"[serving] {reported}/{n} done at {time.perf_counter() - t0:.1f} s, "
                  f"{len(srv.active)} active", file=sys.stderr, flush=True)
        if not srv.active and srv.pending:
            wait = srv.requests[srv.pending[0]].arrival - srv.now()
            if wait > 0:
                time.sleep(min(wait, 0.05))
        else:
            time.sleep(0.0005)
    wall = time.perf_counter() - t0
    st = srv.stats()
    res = [srv.poll(k) for k in ids]
    # alone vs mix: args.serve_check requests rerun one at a time (correlated
    # pairs' members and single requests, the smaller ones first to bound the
    # time), each E_mix series compared bitwise with its run in the mix
    pairs = [k for k, r in enumerate(reqs) if r.tag[0] == "pair"]
    singles = [k for k, r in enumerate(reqs) if r.tag[0] == "single"]
    cost = lambda k: reqs[k].M ** 4 * reqs[k].n_walkers
    half = args.serve_check // 2
    check = sorted(pairs, key=cost)[:half] + sorted(singles, key=cost)[:args.serve_check - half]
    same = True
    for k in check:
        r = reqs[k]
        r1 = Request(**{f: getattr(r, f) for f in r.__dataclass_fields__})
        r1.arrival = 0.0
        s1 = Server(args.serve_budget_gb << 30, max_active=1, chunk_steps=args.serve_chunk)
        rid = s1.submit(r1)
        s1.run()
        same = same and res[k] is not None and np.array_equal(s1.poll(rid).emix, res[k].emix)
        print(f"[serving] alone vs mix: request {k} (M={r.M}, W={r.n_walkers}) "
              f"{'same' if same else 'DIFFERENT'}", file=sys.stderr, flush=True)
    ws = sum(r.n_walkers * r.n_steps for r, x in zip(reqs, res) if x is not None and x.error is None)
    out = {"metric": "serving: walker-steps/s over a mixed request stream; p50/p99 arrival-to-result latency",
           "value": ws / wall, "unit": "walker-steps/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "serving-mix", "requests": n, "rate_per_s": args.rate,
                      "steps_per_request": args.serve_steps, "M": [20, 40, 80, 120, 160],
                      "walkers": [128, 512, 2048], "cs_pairs": sum(1 for r in reqs if r.tag[0] == "pair") // 2,
                      "budget_gib": args.serve_budget_gb, "max_active": args.serve_slots,
                      "chunk_steps": args.serve_chunk},
           "wall_s": wall, "completed": st.get("completed"), "rejected": st.get("rejected"),
           "p50_s": st.get("p50_s"), "p99_s": st.get("p99_s"), "peak_bytes": st.get("peak_bytes"),
           "makespan_s": st.get("makespan_s"),
           "latency_by_M": {str(M): {"p50_s": float(np.percentile(
               [x.latency for x, r in zip(res, reqs) if x is not None and r.M == M], 50))}
               for M in sorted({r.M for r in reqs})},
           "alone_vs_mix_bitwise": bool(same), "alone_vs_mix_checked": len(check),
           "alone_vs_mix_requests": [{"M": reqs[k].M, "W": reqs[k].n_walkers, "kind": reqs[k].tag[0]}
                                     for k in check]}
    print(json.dumps(out), flush=True)


def precision_report(args):
    """Per-step E_L error of the reduced-precision contraction modes on the
    FP64 trajectory's walkers (kernel error) and E_mix drift over a short
    trajectory with the same fields (includes the trajectories' divergence),
    both against the FP64 path, which the parity tests pin to the FP64 oracle
    at this size.  Only the contraction precision varies; Taylor, B1,
    overlaps, inverses, determinants and MGS stay FP64.  The modes run the
    per-vector (Ltil) exchange route, whose contractions take the mode's
    precision; "<prec>+q" runs the Q route (FP32 contractions only while
    M max(N) <= AFQMC_QROUTE_FP32_MAX_K, else FP64)."""
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
    base = dict(taylor_order=wl.taylor_order, ortho_every=wl.ortho_every, pc_every=0, e_trial=et,
                taylor_prec="fp64")
    steps = args.steps
    # FP64 reference trajectory; keep the walkers after `steps` steps
    em64 = afq.propagate(ham, trial, w, steps, wl.dt, 7, 0, afq.Options(chol_prec="fp64", **base))
    em64 = em64.cpu().numpy()
    phi_re, phi_im = w.phi_re.clone(), w.phi_im.clone()
    wt = w.weight.clone()
    el64 = w.eloc[0].cpu().numpy().copy()
    alive = (wt > 0).cpu().numpy()
    out = {"metric": "per-step E_L error and E_mix drift of the contraction precisions vs FP64",
           "unit": "Ha", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": wl.name, "M": wl.M, "n_up": wl.n_up, "n_dn": wl.n_dn,
                      "n_chol": wl.n_chol, "n_walkers": W, "steps": steps, "l_scale": wl.l_scale,
                      "varied": "propagator build and L~ Theta contractions (Ltil route); "
                                "+q: the Q route's contractions per the FP32 size limit",
                      "fixed_fp64": "Taylor, B1, overlaps, inverses, determinants, MGS, sums"},
           "e_mix_fp64_last": float(em64[-1]), "modes": {}}
    q_ok = trial.exchange_route == "q"
    for mode in args.sweep_precs.split(","):
        prec, _, rt = mode.partition("+")
        if rt == "q" and not q_ok:
            continue
        trial.exchange_route = "q" if rt == "q" else "ltilde"
        # (i) kernel error: E_L on the FP64 trajectory's walkers
        w.phi_re.copy_(phi_re)
        w.phi_im.copy_(phi_im)
        w.weight.copy_(wt)
        afq.propagate(ham, trial, w, 0, wl.dt, 7, steps, afq.Options(chol_prec=prec, **base))
        el = w.eloc[0].cpu().numpy()
        d = np.abs(el - el64)[alive]
        # (ii) trajectory drift from the same start and fields
        afq.walkers_from_trial(ham, trial, w)
        em = afq.propagate(ham, trial, w, steps, wl.dt, 7, 0,
                           afq.Options(chol_prec=prec, **base)).cpu().numpy()
        out["modes"][mode] = {"el_max_abs_err": float(d.max()), "el_mean_abs_err": float(d.mean()),
                              "el_max_rel_err": float((d / np.abs(el64[alive])).max()),
                              "emix_max_abs_drift": float(np.abs(em - em64).max()),
                              "emix_drift_last": float(abs(em[-1] - em64[-1]))}
    print(json.dumps(out), flush=True)


def group_bench(args):
    """Walker-resident group path (afqmc_group_*): several systems in one
    launch per segment, segments replayed as HIP graphs.  --workload W with
    --path resident runs that workload's system as a group of one; --batched
    runs the uneven BATCHED_MIX group.  Reports walker-steps/s over all
    members, the resident kernel's roofline (algorithmic flops per launch over
    its HIP-event-timed average duration against the FP64 peak: the kernel
    computes in FP64 on the vector ALUs, whose peak equals the FP64 matrix
    peak), the same members run one after the other through the per-kernel
    chain, and (batched) each member's E_mix alone vs in the group."""
    import torch

    import afqmc_synth as syn
    import paper_1804_03310_amd as afq

    torch.cuda.set_device(0)
    if args.tune_cache:
        afq.tune_cache_path(args.tune_cache)
    if args.batched:
        spec = BATCHED_MIX
        name = "batched-mix"
    else:
        wl = syn.WORKLOADS[args.workload]
        spec = [(wl.name, wl.M, wl.n_up, wl.n_dn, wl.n_chol, args.walkers or wl.n_walkers, wl.tau_d,
                 wl.l_scale != 1.0, wl.ortho_every, wl.pc_every, wl.ham_seed, wl.field_seed, 0)]
        name = wl.name
    systems = {}

    def system(M, nu, nd, G, tau, scaled, hseed):
        key = (M, G, tau, scaled, hseed)
        if key not in systems:
            systems[key] = syn.make_system(M, nu, nu, G, tau, seed=hseed,
                                           l_scale=syn.health_scale(M) if scaled else 1.0)
        return systems[key]

    def members():
        out = []
        for (lab, M, nu, nd, G, W, tau, scaled, oe, pc, hseed, fseed, sid) in spec:
            inp = system(M, nu, nd, G, tau, scaled, hseed)
            ham = afq.Hamiltonian(inp.h, inp.L, inp.e_core)
            trial = afq.Trial(ham, nu, nd, inp.C_up, inp.C_dn)
            w = afq.Walkers(trial, W, system_id=sid)
            afq.walkers_from_trial(ham, trial, w)
            et = afq.local_energy(ham, trial, w)
            opt = afq.Options(taylor_order=6, ortho_every=oe, pc_every=pc, e_trial=et,
                              chol_prec="fp64", taylor_prec="fp64")
            out.append(afq.GroupMember(ham, trial, w, 0.005, fseed, opt))
        return out

    mem = members()
    g = afq.Group(mem)
    tuned_us = g.tune(steps=max(2 * g.config[1], 40)) if args.tune else None
    threads, K, tuned = g.config
    n_ws = sum(m.walkers.n_walkers for m in mem)
    if args.warmup:
        g.propagate(args.warmup, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    em = g.propagate(args.steps, args.warmup)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    e_last = [float(e[args.steps - 1].item()) for e in em]
    # kernel timing pass (direct launches with events) for the roofline
    g.timing(True)
    g.propagate(args.steps, args.warmup + args.steps)
    torch.cuda.synchronize()
    n_l, n_s, ms = g.timing_read()
    g.timing(False)
    flops_step = sum(resident_flops_per_walker(m.ham.M, m.trial.n_up, m.trial.n_dn,
                                               m.ham.n_chol, m.opt.taylor_order)
                     * m.walkers.n_walkers for m in mem)
    per_launch = flops_step * n_s / max(n_l, 1)
    avg_s = ms / max(n_l, 1) / 1e3
    ach = per_launch / avg_s / 1e12 if n_l else float("nan")
    # the same members, one after the other, through the per-kernel chain
    cm = members()
    for m in cm:
        afq.propagate(m.ham, m.trial, m.walkers, args.warmup, m.dt, m.seed, 0, m.opt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for m in cm:
        afq.propagate(m.ham, m.trial, m.walkers, args.steps, m.dt, m.seed, args.warmup, m.opt)
    torch.cuda.synchronize()
    chain_s = time.perf_counter() - t1
    same = None
    if args.batched:
        same = True
        fresh = members()
        gm = afq.Group(fresh)
        ref = [e.cpu().numpy() for e in gm.propagate(args.steps, 0)]
        for k in range(len(fresh)):
            one = members()[k]
            e1 = afq.Group([one]).propagate(args.steps, 0)[0].cpu().numpy()
            same = same and bool(np.array_equal(e1, ref[k]))
    value = n_ws * args.steps / elapsed
    out = {"metric": "walker-steps/sec on 1 MI355X, walker-resident group path (FP64)",
           "value": value, "unit": "walker-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / max(args.steps, 1),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": name, "members": [
               {"label": x[0], "M": x[1], "n_up": x[2], "n_dn": x[3], "n_chol": x[4],
                "walkers": x[5], "ortho_every": x[8], "pc_every": x[9], "system_id": x[12]}
               for x in spec],
               "launch": {"threads_per_walker": threads, "segment_steps": K,
                          "tuned": ["default", "measured", "cache"][tuned], "tune_us_per_step": tuned_us},
               "e_mix_last": e_last},
           "roofline": {"bound": "fp64", "kernel": "k_res_steps (walker-resident, one workgroup "
                        "per walker, a segment of steps per launch)",
                        "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": ach / FP64_PEAK_TFLOPS, "traffic": None,
                        "flops_per_launch": per_launch, "avg_launch_ms": avg_s * 1e3,
                        "launches": n_l, "steps_per_launch": n_s / max(n_l, 1)},
           "per_kernel_chain": {"value": n_ws * args.steps / chain_s,
                                "ms_per_step": 1e3 * chain_s / max(args.steps, 1),
                                "note": "the same members run one after the other through "
                                        "afqmc_propagate's per-kernel chain, FP64"},
           "speedup_vs_chain": chain_s / elapsed,
           "alone_vs_group_bitwise": same}
    print(json.dumps(out), flush=True)


def cs_report(args):
    """Correlated sampling (Sec. I, Sec. V) on the hydrogen-chain workload:
    the neutral system (N_up = N_dn) and its cation (one down electron fewer)
    propagated from their trial states with the same seed and system id, so
    that every step draws the same fields for both, in `cs_repeats`
    independent repeats (population control off, as in correlated sampling);
    the cumulative average of E_cation - E_neutral over the repeats with its
    error bar (afqmc_cs_difference), beside the same difference from
    independent fields.  Then a long population-controlled run of the neutral
    system whose E_mix series gets a reblocking error bar (afqmc_reblock).
    All propagation on the GPU; the statistics on the host through the
    C ABI."""
    import torch

    import afqmc_synth as syn
    import paper_1804_03310_amd as afq

    wl = syn.WORKLOADS[args.workload]
    inp = syn.workload_system(wl)
    torch.cuda.set_device(0)
    ham = afq.Hamiltonian(inp.h, inp.L, inp.e_core)
    nu, nd = wl.n_up, wl.n_dn
    systems = {"neutral": afq.Trial(ham, nu, nd, inp.C_up, inp.C_dn),
               "cation": afq.Trial(ham, nu, nd - 1, inp.C_up, inp.C_dn)}
    W, T, R = args.cs_walkers, args.cs_steps, args.cs_repeats
    walkers, etrial = {}, {}
    for k, tr in systems.items():
        walkers[k] = afq.Walkers(tr, W)
        afq.walkers_from_trial(ham, tr, walkers[k])
        etrial[k] = afq.local_energy(ham, tr, walkers[k])
    emix = torch.empty(T, dtype=torch.float64, device="cuda")

    def run(k, seed):
        o = afq.Options(taylor_order=wl.taylor_order, ortho_every=wl.ortho_every, pc_every=0,
                        e_trial=etrial[k])
        afq.walkers_from_trial(ham, systems[k], walkers[k])
        afq.propagate(ham, systems[k], walkers[k], T, wl.dt, seed, 0, o, emix=emix)
        return emix.cpu().numpy().copy()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    neu = np.array([run("neutral", 1000 + r) for r in range(R)])
    cat = np.array([run("cation", 1000 + r) for r in range(R)])
    cat_ind = np.array([run("cation", 5000 + r) for r in range(R)])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    first = min(T // 10, 10)
    m_cs, s_cs = afq.cs_difference(neu, cat, first)
    m_in, s_in = afq.cs_difference(neu, cat_ind, first)
    # long run with population control: reblocking of the E_mix series
    L = args.cs_long_steps
    wl_long = afq.Walkers(systems["neutral"], wl.n_walkers)
    afq.walkers_from_trial(ham, systems["neutral"], wl_long)
    e_long = torch.empty(L, dtype=torch.float64, device="cuda")
    o = afq.Options(taylor_order=wl.taylor_order, ortho_every=wl.ortho_every,
                    pc_every=wl.pc_every, e_trial=etrial["neutral"])
    afq.propagate(ham, systems["neutral"], wl_long, L, wl.dt, 77, 0, o, emix=e_long)
    series = e_long.cpu().numpy()[L // 5:]
    mean, sems, plateau = afq.reblock(series)
    out = {"metric": "correlated-sampling energy difference and reblocking error bars",
           "unit": "Ha", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": wl.name, "neutral": [nu, nd], "cation": [nu, nd - 1],
                      "repeats": R, "walkers": W, "steps": T, "dt": wl.dt,
                      "averaged_from_step": first, "pc": "off (correlated sampling)",
                      "long_run": {"walkers": wl.n_walkers, "steps": L, "pc_every": wl.pc_every,
                                   "discarded": L // 5}},
           "e_trial": etrial,
           "delta_e_cs": float(m_cs[-1]), "sem_cs": float(s_cs[-1]),
           "delta_e_independent": float(m_in[-1]), "sem_independent": float(s_in[-1]),
           "sem_ratio_independent_over_cs": float(s_in[-1] / s_cs[-1]),
           # correlation over the repeats of the two systems' E_mix at a few steps
           "corr_neutral_cation": {str(t): float(np.corrcoef(neu[:, t], cat[:, t])[0, 1])
                                   for t in sorted({0, 4, 9, 19, 49, 99, T - 1}) if t < T},
           "corr_neutral_cation_independent": {
               str(t): float(np.corrcoef(neu[:, t], cat_ind[:, t])[0, 1])
               for t in sorted({0, 4, 9, 19, 49, 99, T - 1}) if t < T},
           "walker_steps_per_s": 3 * R * W * T / elapsed,
           "reblock": {"mean": mean, "sem_by_level": sems, "plateau": plateau,
                       "sem": sems[plateau] if plateau >= 0 else None, "naive_sem": sems[0]}}
    print(json.dumps(out), flush=True)


def _oracle_rate(wl, inp, sample_walkers, sample_steps):
    from oracle import Oracle, Options as OOptions
    o = Oracle.from_inputs(inp)
    st = o.init_walkers(sample_walkers)
    et = o.mixed_energy(st)
    opt = OOptions(taylor_order=wl.taylor_order, ortho_every=wl.ortho_every, pc_every=0, e_trial=et)
    o.propagate(st, 1, wl.dt, 0, 0, opt)  # warm caches (B1, allocations)
    t0 = time.perf_counter()
    o.propagate(st, sample_steps, wl.dt, 0, 1, opt)
    dt = time.perf_counter() - t0
    return sample_walkers * sample_steps / dt, dt


def cpu_baseline(wl, inp, sample_walkers, sample_steps):
    """The FP64 numpy oracle (not tuned) on a bounded sample of the workload:
    once with the BLAS threads the host gives it (`cores`), once on one
    thread over a quarter of the steps."""
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads, threadpool_limits = os.cpu_count() or 1, None
    rate, dt = _oracle_rate(wl, inp, sample_walkers, sample_steps)
    one = None
    if threadpool_limits is not None:
        n1 = max(sample_steps // 4, 1)
        with threadpool_limits(limits=1):
            r1, d1 = _oracle_rate(wl, inp, sample_walkers, n1)
        one = {"value": r1, "cores": 1,
               "sample": f"{sample_walkers} walkers x {n1} steps, one BLAS thread, {d1:.1f} s"}
    return {"value": rate, "unit": "walker-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{sample_walkers} walkers x {sample_steps} steps of {wl.name} "
                      f"(FP64 numpy oracle, comb off), {dt:.1f} s",
            "single_thread": one}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="hchain-M50")
    ap.add_argument("--walkers", type=int, default=0)
    ap.add_argument("--prec", default="",
                    help="override precisions: 'chol' or 'chol,taylor' from fp64/fp32/bf16/bf16x3")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--weight-mode", choices=["local", "hybrid"], default="local",
                    help="local-energy weights every step (default) or the hybrid form")
    ap.add_argument("--meas-every", type=int, default=20,
                    help="hybrid form: steps between E_L measurements")
    ap.add_argument("--exchange-route", choices=["auto", "ltilde", "q"], default="auto",
                    help="exchange route of single-determinant trials (auto: the library's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-walkers", type=int, default=16)
    ap.add_argument("--cpu-steps", type=int, default=80)
    ap.add_argument("--tte-repeats", type=int, default=20,
                    help="time-to-energy repeats (field seeds 0 .. repeats - 1)")
    ap.add_argument("--tte-steps", type=int, default=0,
                    help="steps of each time-to-energy run (0: the workload's full run)")
    ap.add_argument("--precision-report", action="store_true",
                    help="E_L error and E_mix drift of the contraction precisions vs FP64")
    ap.add_argument("--sweep-precs", default="fp32,bf16,bf16x3,fp64,fp32+q")
    ap.add_argument("--serving", action="store_true",
                    help="run the mixed request stream through the serving loop instead")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--serve-steps", type=int, default=200)
    ap.add_argument("--serve-seed", type=int, default=0)
    ap.add_argument("--serve-budget-gb", type=int, default=64)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-chunk", type=int, default=10)
    ap.add_argument("--serve-check", type=int, default=16,
                    help="requests rerun alone and compared bitwise with their run in the mix")
    ap.add_argument("--cs", action="store_true",
                    help="correlated-sampling energy difference (neutral vs cation sharing the "
                         "fields) over repeats, and a reblocking analysis of a long run")
    ap.add_argument("--cs-repeats", type=int, default=16)
    ap.add_argument("--cs-walkers", type=int, default=256)
    ap.add_argument("--cs-steps", type=int, default=100)
    ap.add_argument("--cs-long-steps", type=int, default=1000)
    ap.add_argument("--path", choices=["chain", "resident"], default="chain",
                    help="per-kernel chain (afqmc_propagate) or the walker-resident group "
                         "kernel (afqmc_group_*, FP64, systems up to M = 64)")
    ap.add_argument("--batched", action="store_true",
                    help="a group of uneven systems in one resident launch per segment")
    ap.add_argument("--tune", action="store_true", help="autotune the group's launch shape first")
    ap.add_argument("--tune-cache", default="", help="JSON file of the autotuner's choices")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain elementwise copy of 256 MiB (reads 256 MiB, writes "
                         "256 MiB) so that HBM byte counters can be scaled")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(walker sharding across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    if args.serving:
        serving_bench(args)
        return
    if args.precision_report:
        precision_report(args)
        return
    if args.cs:
        cs_report(args)
        return
    if args.batched or args.path == "resident":
        group_bench(args)
        return

    import torch

    import afqmc_synth as syn
    import paper_1804_03310_amd as afq

    wl = syn.WORKLOADS[args.workload]
    W = args.walkers or wl.n_walkers
    chol_prec, taylor_prec = wl.chol_prec, wl.taylor_prec
    if args.prec:
        parts = args.prec.split(",")
        chol_prec = parts[0]
        taylor_prec = parts[1] if len(parts) > 1 else ("fp64" if parts[0] == "fp64" else taylor_prec)
    inp = syn.workload_system(wl)
    torch.cuda.set_device(0)
    ham = afq.Hamiltonian(inp.h, inp.L, inp.e_core)
    multi = inp.n_det > 1
    trial = afq.Trial(ham, inp.n_up, inp.n_dn, inp.C_up, inp.C_dn,
                      inp.coeff if multi else None, inp.exc if multi else None)
    if args.exchange_route != "auto":
        trial.exchange_route = args.exchange_route
    route = trial.exchange_route if chol_prec not in ("bf16", "bf16x3") else "ltilde"
    w = afq.Walkers(trial, W)
    afq.walkers_from_trial(ham, trial, w)
    et = afq.local_energy(ham, trial, w)
    opt_kw = dict(taylor_order=wl.taylor_order, ortho_every=wl.ortho_every,
                  chol_prec=chol_prec, taylor_prec=taylor_prec, weight_mode=args.weight_mode,
                  meas_every=args.meas_every)
    opt = afq.Options(pc_every=wl.pc_every, e_trial=et, **opt_kw)
    if args.tte_steps <= 0:
        args.tte_steps = wl.n_steps
    if args.weight_mode == "hybrid":  # the time-to-energy runs end on a measured step
        args.tte_steps = -(-args.tte_steps // args.meas_every) * args.meas_every
    emix = torch.empty(max(args.steps, args.warmup, args.tte_steps, 1), dtype=torch.float64,
                       device="cuda")
    # warmup
    if args.warmup:
        afq.propagate(ham, trial, w, args.warmup, wl.dt, 1, 0, opt, emix=emix)
    torch.cuda.synchronize()
    for k in afq._abi.KERNEL_CLASSES:
        afq.timing_read(ham, k)
    # timed region: exactly `steps` steps in one call; HIP events on the launch
    # stream bracket the launches of the roofline candidate classes only (the
    # exchange and the Taylor propagation), so that the timing itself adds
    # little to the step
    roof_classes = ["exchange", "taylor_b1"]
    afq.timing_enable(ham, roof_classes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    afq.propagate(ham, trial, w, args.steps, wl.dt, 1, args.warmup, opt, emix=emix)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    afq.timing_enable(ham, False)
    ktimes = {k: afq.timing_read(ham, k) for k in afq._abi.KERNEL_CLASSES}
    em_host = emix[:args.steps].cpu().numpy() if args.steps else np.zeros(0)
    finite = em_host[np.isfinite(em_host)]
    e_last = float(finite[-1]) if finite.size else float("nan")
    alive = int((w.weight > 0).sum().item())
    # profiling pass after the timed region: the same number of steps with
    # every kernel class timed, for the per-class breakdown
    afq.timing_enable(ham, True)
    afq.propagate(ham, trial, w, args.steps, wl.dt, 1, args.warmup + args.steps, opt, emix=emix)
    torch.cuda.synchronize()
    afq.timing_enable(ham, False)
    kprof = {k: afq.timing_read(ham, k) for k in afq._abi.KERNEL_CLASSES}

    # time to energy: propagate start -> final E_mix on the host
    tte = []
    for r in range(args.tte_repeats):
        afq.walkers_from_trial(ham, trial, w)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        e = afq.propagate(ham, trial, w, args.tte_steps, wl.dt, r, 0, opt, emix=emix)
        _ = float(e[args.tte_steps - 1].item())
        tte.append(time.perf_counter() - t1)

    # candidate kernels for the roofline line: the exchange contraction and,
    # where it runs as one fused launch, the Taylor propagation; the one with
    # the larger time per step is reported, the other under "roofline_other"
    if multi:
        md_rows = multidet_compact_rows(wl.M, wl.n_up, wl.n_dn, inp.exc, chol_prec)
        ex_flops = multidet_flops_per_walker(wl.M, wl.n_up, wl.n_dn, wl.n_chol, md_rows) * W
        ex_name = ("k_md_energy (P = (C^T L_g) Theta_0, X0^2, per-determinant corrections)"
                   if md_rows is None else
                   f"k_md_energy_rows (P = (C^T L_g) Theta_0 over {md_rows[0]} + {md_rows[1]} "
                   "compact rows, X0^2, per-determinant corrections)")
    elif route == "q":
        ex_flops = qform_flops_per_walker(wl.M, wl.n_up, wl.n_dn) * W
        ex_name = "k_qform (theta^T Q theta, upper-triangular tile pairs)"
    else:
        ex_flops = exchange_flops_per_walker(wl.M, wl.n_up, wl.n_dn, wl.n_chol) * W
        if chol_prec in ("bf16", "bf16x3"):
            ex_name = "k_exchange_bf16_rf (fused Ltil*Theta with X^T tiles, Tr X, Tr XX)"
        else:
            ex_name = ("k_exchange_full (fused Ltil*Theta, Tr X, Tr XX)"
                       if max(wl.n_up, wl.n_dn) <= 32 else "k_exchange (fused Ltil*Theta, Tr X, Tr XX)")
    # the Q route's contractions are FP32 only under FP32 and while
    # M max(N) <= AFQMC_QROUTE_FP32_MAX_K, FP64 otherwise
    q32 = chol_prec == "fp32" and wl.M * max(wl.n_up, wl.n_dn) <= afq._abi.QROUTE_FP32_MAX_K
    ex_prec = ("fp32" if q32 else "fp64") if (route == "q" and not multi) else chol_prec
    # BF16X3 takes three bf16 MFMA products per algorithmic product: its
    # fraction is against the bf16 peak (so at most 1/3)
    ex_peak = {"fp32": FP32_PEAK_TFLOPS, "fp64": FP64_PEAK_TFLOPS, "bf16": BF16_PEAK_TFLOPS,
               "bf16x3": BF16_PEAK_TFLOPS}[ex_prec]
    # per step: the exchange class is one launch; the Taylor class is one
    # fused launch, or a chain of GEMM launches (B1, each term, B1) whose
    # algorithmic flops are shared out over the chain's launches
    cands = [("exchange", ex_name, ex_flops, ex_peak)]
    tay_flops = taylor_flops_per_walker(wl.M, wl.n_up + wl.n_dn, wl.taylor_order) * W
    tay_peak = {"fp32": FP32_PEAK_TFLOPS, "fp64": FP64_PEAK_TFLOPS}[taylor_prec]
    if taylor_fused(wl.M, wl.n_up + wl.n_dn, taylor_prec):
        cands.append(("taylor_b1",
                      "k_propagate_fused (B1 exp(A) B1 phi, Taylor order %d)" % wl.taylor_order,
                      tay_flops, tay_peak))
    else:
        cands.append(("taylor_b1",
                      "k_cgemm_walkers chain (B1, %d Taylor terms, B1; walker-batched complex "
                      "GEMMs; the chain timed as one bracket per step)" % wl.taylor_order, tay_flops,
                      tay_peak))
    lines = []
    for cls, nm, fl_step, pk in cands:
        n_l, ms_l = ktimes[cls]
        per_step = n_l / max(args.steps, 1)
        fl = fl_step / per_step if n_l else float("nan")  # flops per launch
        a_s = (ms_l / n_l) / 1e3 if n_l else float("nan")
        ach = fl / a_s / 1e12 if n_l else float("nan")
        lines.append({"class": cls, "bound": "mfma", "kernel": nm, "achieved": ach, "peak": pk,
                      "unit": "TFLOP/s", "frac": ach / pk,
                      "traffic": measured_traffic(wl.name, cls, ex_prec, taylor_prec),
                      "flops_per_launch": fl, "flops_per_step": fl_step,
                      "avg_launch_ms": a_s * 1e3, "launches": n_l,
                      "launches_per_step": per_step, "ms_per_step": ms_l / max(args.steps, 1)})
    lines.sort(key=lambda d: -(d["ms_per_step"] if d["launches"] else 0.0))
    roof, roof_other = lines[0], lines[1:]
    fbias_report = None
    n_fb, ms_fb = kprof["force_bias"]
    if route == "q" and n_fb and not multi:
        # the force-bias class: the k_fbias_mm launch
        fb_flops = fbias_flops_per_walker(wl.M, wl.n_up, wl.n_dn, wl.n_chol) * W
        fb_s = (ms_fb / n_fb) / 1e3
        fbias_report = {"flops_per_launch": fb_flops, "avg_launch_ms": fb_s * 1e3,
                        "achieved_tflops": fb_flops / fb_s / 1e12, "launches": n_fb}
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
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16": "bf16", "bf16x3": "bf16x3"}[chol_prec],
        "data": "synthetic",
        "config": {"workload": wl.name, "M": wl.M, "n_up": wl.n_up, "n_dn": wl.n_dn,
                   "n_chol": wl.n_chol, "n_walkers": W, "dt": wl.dt,
                   "taylor_order": wl.taylor_order, "ortho_every": wl.ortho_every,
                   "pc_every": wl.pc_every, "n_det": inp.n_det, "l_scale": wl.l_scale,
                   "weight_mode": args.weight_mode, "exchange_route": route,
                   "meas_every": args.meas_every if args.weight_mode == "hybrid" else 1,
                   "precision": f"contractions {chol_prec}, Taylor/B1 {taylor_prec}, "
                                "overlap/inverse/det/MGS/sums fp64"
                                + (", Q-route exchange and force bias fp64"
                                   if route == "q" and ex_prec == "fp64" else ""),
                   "e_trial": et, "e_mix_last": e_last, "alive_walkers": alive},
        "roofline": roof,
        "roofline_other": roof_other,
        "kernel_ms_per_step": {k: (v[1] / max(args.steps, 1)) for k, v in kprof.items() if v[0]},
        "kernel_ms_per_step_source": "a pass of the same number of steps after the timed region "
                                     "with every kernel class timed",
        "force_bias_class": fbias_report,
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
    if not args.no_accuracy and wl.name in GOLDEN and args.weight_mode == "local":
        out["accuracy"] = accuracy_check(afq, torch, wl, inp, ham, trial, opt_kw)
    elif not args.no_accuracy:
        out["accuracy"] = kernel_error_check(afq, torch, wl, inp, ham, trial, opt_kw,
                                             min(W, 256))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, inp, args.cpu_walkers, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
