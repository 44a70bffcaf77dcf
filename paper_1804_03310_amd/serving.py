"""Continuous-batching request loop for AFQMC runs on one GPU.

Requests (a system, a walker count, a number of steps, a seed) arrive over
time.  The server admits a request as soon as its device footprint (from
`afqmc_footprint_bytes`, computed before anything is allocated) fits in the
remaining HBM budget and an active slot is free, gives each admitted run its
own HIP stream, and keeps enqueuing chunks of steps on every active stream, so
the kernels of different runs overlap on the device while new requests are
admitted.  A run's result (the mixed energy after every step) is the same
whether it runs alone or in a mix: each run has its own buffers and the
kernels are deterministic.  Correlated-sampling pairs (a neutral and a cation
system) share a field stream by using the same seed and system id.

The scheduling logic is independent of the device: it talks to an executor
with start / enqueue / done / finish; `GpuExecutor` drives the HIP library,
and a host-only executor can stand in for tests of the policy.
"""
from __future__ import annotations

import ctypes
import dataclasses
import time
from typing import Any, Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    h: np.ndarray
    L: np.ndarray
    e_core: float
    C_up: np.ndarray
    C_dn: np.ndarray
    n_up: int
    n_dn: int
    n_walkers: int
    n_steps: int
    dt: float = 0.005
    seed: int = 0
    system_id: int = 0
    coeff: Optional[np.ndarray] = None
    exc: Optional[np.ndarray] = None
    taylor_order: int = 6
    ortho_every: int = 2
    pc_every: int = 20
    chol_prec: str = "fp32"
    taylor_prec: str = "fp32"
    arrival: float = 0.0
    tag: Any = None

    @property
    def M(self) -> int:
        return int(self.h.shape[0])

    @property
    def n_chol(self) -> int:
        return int(self.L.shape[0])

    @property
    def n_det(self) -> int:
        return 1 if self.coeff is None else int(np.asarray(self.coeff).size)


@dataclasses.dataclass
class Result:
    req_id: int
    emix: Optional[np.ndarray]
    e_trial: float
    t_arrival: float
    t_admit: float
    t_done: float
    footprint: int
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


def footprint_bytes(req: Request) -> int:
    from . import _abi
    lib = _abi.load()
    b = ctypes.c_size_t()
    _abi.check(lib.afqmc_footprint_bytes(req.M, req.n_chol, req.n_up, req.n_dn, req.n_det,
                                         req.n_walkers, ctypes.byref(b)))
    return int(b.value)


class GpuExecutor:
    """Runs requests through the HIP library, one torch stream per run.

    Requests that carry the same h and L arrays (the same Python objects, e.g.
    the neutral and cation of a correlated-sampling pair) share one device
    Hamiltonian, which is read-only once built; it is freed when its last run
    finishes.
    """

    def __init__(self, device: int = 0):
        self.device = device
        self._hams = {}

    def footprint(self, req: Request) -> int:
        return footprint_bytes(req)

    def _hamiltonian(self, req: Request):
        import torch

        from . import Hamiltonian
        key = (id(req.h), id(req.L), float(req.e_core))
        ent = self._hams.get(key)
        if ent is None:
            # set-up work (this Hamiltonian's and its trials' initialisation) goes
            # to a stream of its own, not behind a running request's steps
            if getattr(self, "_init_stream", None) is None:
                self._init_stream = torch.cuda.Stream(device=self.device)
            ham = Hamiltonian(req.h, req.L, req.e_core, device=self.device, stream=self._init_stream)
            self._init_stream.synchronize()
            ent = self._hams[key] = [ham, 0, req.h, req.L]  # keep the arrays alive with the key
        ent[1] += 1
        return key, ent[0]

    def start(self, req: Request):
        import torch

        from . import (Options, Trial, Walkers, local_energy, walkers_from_trial)
        stream = torch.cuda.Stream(device=self.device)
        ham_key, ham = self._hamiltonian(req)
        trial = Trial(ham, req.n_up, req.n_dn, req.C_up, req.C_dn, req.coeff, req.exc)
        w = Walkers(trial, req.n_walkers, system_id=req.system_id)
        emix = torch.empty(max(req.n_steps, 1), dtype=torch.float64,
                           device=torch.device("cuda", self.device))
        torch.cuda.current_stream(self.device).synchronize()
        walkers_from_trial(ham, trial, w, stream=stream)
        et = local_energy(ham, trial, w, stream=stream)
        opt = Options(taylor_order=req.taylor_order, ortho_every=req.ortho_every,
                      pc_every=req.pc_every, e_trial=et, chol_prec=req.chol_prec,
                      taylor_prec=req.taylor_prec)
        return {"ham": ham, "ham_key": ham_key, "trial": trial, "w": w, "stream": stream,
                "emix": emix, "opt": opt, "e_trial": et, "done_steps": 0, "event": None}

    def enqueue(self, h, req: Request, n: int) -> None:
        import torch

        from . import propagate
        s0 = h["done_steps"]
        propagate(h["ham"], h["trial"], h["w"], n, req.dt, req.seed, s0, h["opt"],
                  emix=h["emix"][s0:], stream=h["stream"])
        ev = torch.cuda.Event()
        ev.record(h["stream"])
        h["event"] = ev
        h["done_steps"] = s0 + n

    def done(self, h) -> bool:
        return h["event"] is None or h["event"].query()

    def finish(self, h):
        h["stream"].synchronize()
        out = h["emix"].cpu().numpy().copy()
        et = h["e_trial"]
        for k in ("w", "trial", "ham", "emix"):
            h[k] = None
        ent = self._hams.get(h["ham_key"])
        if ent is not None:
            ent[1] -= 1
            if ent[1] == 0:
                del self._hams[h["ham_key"]]
        return out, et


class Server:
    """Admission by HBM footprint, one slot per active run, chunked enqueue."""

    def __init__(self, budget_bytes: int, executor=None, max_active: int = 16,
                 chunk_steps: int = 20, clock: Callable[[], float] = time.perf_counter):
        self.budget = int(budget_bytes)
        self.ex = executor if executor is not None else GpuExecutor()
        self.max_active = max_active
        self.chunk = max(1, chunk_steps)
        self.clock = clock
        self.t0 = clock()
        self.pending: List[int] = []
        self.requests: Dict[int, Request] = {}
        self.fp: Dict[int, int] = {}
        self.active: Dict[int, Any] = {}
        self.admit_time: Dict[int, float] = {}
        self.results: Dict[int, Result] = {}
        self.used = 0
        self.peak_used = 0
        self._next = 0

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request) -> int:
        rid = self._next
        self._next += 1
        self.requests[rid] = req
        self.fp[rid] = self.ex.footprint(req)
        self.pending.append(rid)
        self.pending.sort(key=lambda r: (self.requests[r].arrival, r))
        return rid

    def poll(self, rid: int) -> Optional[Result]:
        return self.results.get(rid)

    def _admit(self, now: float) -> None:
        for rid in list(self.pending):
            req = self.requests[rid]
            if req.arrival > now:
                break
            fp = self.fp[rid]
            if fp > self.budget:
                self.pending.remove(rid)
                self.results[rid] = Result(rid, None, float("nan"), req.arrival, now, now, fp,
                                           error="footprint exceeds the HBM budget")
                continue
            if len(self.active) >= self.max_active or self.used + fp > self.budget:
                continue  # first fit: a later, smaller request may still be admitted
            self.pending.remove(rid)
            self.used += fp
            self.peak_used = max(self.peak_used, self.used)
            self.admit_time[rid] = now
            self.active[rid] = self.ex.start(req)

    def step(self) -> bool:
        """One scheduler pass; returns True if anything is left to do."""
        self._admit(self.now())
        for rid in list(self.active):
            h = self.active[rid]
            req = self.requests[rid]
            if not self.ex.done(h):
                continue
            left = req.n_steps - h["done_steps"]
            if left > 0:
                self.ex.enqueue(h, req, min(self.chunk, left))
                continue
            emix, et = self.ex.finish(h)
            t = self.now()
            self.results[rid] = Result(rid, emix, et, req.arrival, self.admit_time[rid], t,
                                       self.fp[rid])
            del self.active[rid]
            self.used -= self.fp[rid]
        return bool(self.pending or self.active)

    def run(self, idle_sleep: float = 0.0005) -> None:
        while self.step():
            if not self.active and self.pending:
                nxt = self.requests[self.pending[0]].arrival
                wait = nxt - self.now()
                if wait > 0:
                    self._sleep(min(wait, 0.05))
            elif idle_sleep:
                self._sleep(idle_sleep)

    def _sleep(self, dt: float) -> None:
        sleeper = getattr(self.ex, "sleep", None)
        if sleeper is not None:
            sleeper(dt)
        else:
            time.sleep(dt)

    def stats(self) -> dict:
        done = [r for r in self.results.values() if r.error is None]
        lat = np.array([r.latency for r in done]) if done else np.zeros(0)
        if not done:
            return {"completed": 0}
        span = max(r.t_done for r in done) - min(r.t_arrival for r in done)
        ws = sum(self.requests[r.req_id].n_walkers * self.requests[r.req_id].n_steps for r in done)
        return {"completed": len(done), "rejected": len(self.results) - len(done),
                "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "walker_steps_per_s": ws / span if span > 0 else float("nan"),
                "makespan_s": span, "peak_bytes": self.peak_used}
