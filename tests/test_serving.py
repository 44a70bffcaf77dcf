"""Serving loop: admission policy (host only, simulated executor) and, on the
GPU, results that are bitwise the same alone and in a mix."""
import numpy as np
import pytest

import afqmc_synth as syn


def _serving():
    # imported inside the tests: the package loads (and if needed builds) the
    # HIP library, and a failure there must not stop collection of the others
    from paper_1804_03310_amd import serving
    return serving


def _req(M, W, steps, arrival, seed=0, system_id=0, n_dn=None, prec="fp64"):
    inp = syn.make_system(M, M // 4, M // 4 if n_dn is None else n_dn, 2 * M, 8.0, seed=M)
    return _serving().Request(h=inp.h, L=inp.L, e_core=0.0, C_up=inp.C_up, C_dn=inp.C_dn, n_up=inp.n_up,
                   n_dn=inp.n_dn, n_walkers=W, n_steps=steps, dt=0.005, seed=seed,
                   system_id=system_id, arrival=arrival, chol_prec=prec, taylor_prec=prec,
                   ortho_every=2, pc_every=5)


class SimExecutor:
    """Host-only stand-in: cost proportional to walkers x steps x M^2."""

    def __init__(self):
        self.t = 0.0
        self.started = []

    def clock(self):
        return self.t

    def sleep(self, dt):
        self.t += dt

    def footprint(self, req):
        # host-side stand-in for the library's footprint query: L, one A and a
        # few orbital-sized arrays per walker, in bytes
        M, nt = req.M, req.n_up + req.n_dn
        return 8 * (req.n_chol * M * M + req.n_walkers * (2 * M * M + 8 * M * nt))

    def start(self, req):
        self.started.append(req.tag)
        return {"done_steps": 0, "until": self.t}

    def enqueue(self, h, req, n):
        h["until"] = max(h["until"], self.t) + 1e-7 * req.n_walkers * n * req.M ** 2
        h["done_steps"] += n

    def done(self, h):
        return self.t >= h["until"]

    def finish(self, h):
        return np.arange(3.0), -1.0


def test_footprint_grows_with_size():
    footprint_bytes = _serving().footprint_bytes
    a = footprint_bytes(_req(16, 32, 10, 0))
    b = footprint_bytes(_req(32, 32, 10, 0))
    c = footprint_bytes(_req(32, 128, 10, 0))
    assert 0 < a < b < c


def test_admission_respects_budget_and_first_fit():
    Server = _serving().Server
    ex = SimExecutor()
    big = _req(40, 256, 50, 0.0)
    small = [_req(12, 32, 20, 0.001 * i) for i in range(6)]
    budget = ex.footprint(big) + ex.footprint(small[0])
    srv = Server(budget, executor=ex, max_active=4, chunk_steps=10, clock=ex.clock)
    big.tag = "big"
    ids = [srv.submit(big)]
    for i, r in enumerate(small):
        r.tag = f"s{i}"
        ids.append(srv.submit(r))
    huge = _req(64, 4096, 10, 0.0)
    huge.tag = "huge"
    hid = srv.submit(huge)
    srv.run(idle_sleep=1e-4)
    assert srv.peak_used <= budget
    for i in ids:
        res = srv.poll(i)
        assert res is not None and res.error is None
        assert res.t_done >= res.t_admit >= res.t_arrival
    assert srv.poll(hid).error is not None
    # small requests were admitted while the big one was still running
    assert ex.started[:2] == ["big", "s0"]
    st = srv.stats()
    assert st["completed"] == 7 and st["rejected"] == 1
    assert st["p99_s"] >= st["p50_s"] > 0


def test_slots_limit_concurrency():
    Server = _serving().Server
    ex = SimExecutor()
    reqs = [_req(8, 16, 10, 0.0) for _ in range(5)]
    srv = Server(10 ** 12, executor=ex, max_active=2, chunk_steps=5, clock=ex.clock)
    for r in reqs:
        srv.submit(r)
    max_seen = 0
    while srv.step():
        max_seen = max(max_seen, len(srv.active))
        ex.sleep(1e-5)
    assert max_seen == 2
    assert srv.stats()["completed"] == 5


@pytest.mark.gpu
def test_results_identical_alone_and_in_mix():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu-case] serving alone vs mix", flush=True)
    Server = _serving().Server
    mk = lambda: [_req(8, 16, 12, 0.0, seed=3, system_id=1),
                  _req(8, 16, 12, 0.0, seed=3, system_id=1, n_dn=1),   # cation of the pair
                  _req(12, 32, 12, 0.0, seed=5),
                  _req(16, 24, 12, 0.01, seed=7, prec="fp32"),
                  _req(12, 8, 12, 0.02, seed=9)]
    srv = Server(8 << 30, max_active=8, chunk_steps=4)
    ids = [srv.submit(r) for r in mk()]
    srv.run()
    mixed = [srv.poll(i) for i in ids]
    assert all(r is not None and r.error is None for r in mixed)
    for i, r in enumerate(mk()):
        r.arrival = 0.0
        s1 = Server(8 << 30, max_active=1, chunk_steps=4)
        rid = s1.submit(r)
        s1.run()
        alone = s1.poll(rid)
        assert np.array_equal(alone.emix, mixed[i].emix), i
    st = srv.stats()
    print("serving stats", st)
    assert st["completed"] == 5
