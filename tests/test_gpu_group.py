"""Groups (afqmc_group_*): the walker-resident kernel over several systems in
one launch per segment, replayed as a HIP graph.  Parity with the FP64
oracle, bitwise identity of each member's results alone and in a group of
uneven systems, independence of the launch shape, and the autotuner's cache.
"""
import json
import os
import sys

import numpy as np
import pytest

import afqmc_synth as syn
from oracle import Oracle, Options as OOptions

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def afq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_03310_amd as afq
    return afq


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _member(afq, inp, W, dt, seed, system_id=0, **opt_kw):
    ham = afq.Hamiltonian(inp.h, inp.L, inp.e_core)
    trial = afq.Trial(ham, inp.n_up, inp.n_dn, inp.C_up, inp.C_dn)
    w = afq.Walkers(trial, W, system_id=system_id)
    afq.walkers_from_trial(ham, trial, w)
    et = afq.local_energy(ham, trial, w)
    opt = afq.Options(e_trial=et, chol_prec="fp64", taylor_prec="fp64", **opt_kw)
    return afq.GroupMember(ham, trial, w, dt, seed, opt)


def _state(m):
    w = m.walkers
    return [_np(x).copy() for x in (w.phi_re, w.phi_im, w.weight, w.logovlp, w.eloc)]


def test_group_plain_fp64_parity_100_steps(afq):
    """The 10-orbital FP64 workload (64 walkers, 100 steps, MGS every 2) as a
    group of one: E_mix within 1e-9 Ha of the oracle at every step."""
    _say("group plain-M10 fp64 100 steps")
    wl = syn.WORKLOADS["plain-M10"]
    inp = syn.workload_system(wl)
    m = _member(afq, inp, wl.n_walkers, wl.dt, 0, taylor_order=6, ortho_every=wl.ortho_every)
    g = afq.Group([m])
    em = _np(g.propagate(wl.n_steps, 0)[0])
    o = Oracle.from_inputs(inp)
    st = o.init_walkers(wl.n_walkers)
    oe = o.propagate(st, wl.n_steps, wl.dt, 0, 0,
                     OOptions(taylor_order=6, ortho_every=wl.ortho_every, e_trial=m.opt.e_trial))
    print("max |dE_mix| =", np.max(np.abs(em - oe)))
    assert np.max(np.abs(em - oe)) <= 1e-9
    assert np.allclose(_np(m.walkers.weight), st.weight, rtol=1e-9, atol=1e-12)
    el = _np(m.walkers.eloc[0])
    alive = st.weight > 0
    assert np.allclose(el[alive], st.eloc.real[alive], rtol=1e-9)
    phi = _np(m.walkers.phi_re) + 1j * _np(m.walkers.phi_im)
    assert np.allclose(phi, st.phi, rtol=0, atol=1e-9)


@pytest.mark.parametrize("W,pc,steps,step0", [(64, 5, 30, 0), (37, 4, 13, 3)])
def test_group_with_comb_fp64_parity(afq, W, pc, steps, step0):
    """Combs every pc steps at segment ends (including a first segment that
    starts off the comb grid): E_mix within 1e-9 Ha of the oracle."""
    _say(f"group plain-M10 fp64 comb every {pc}, W={W}, {steps} steps from {step0}")
    wl = syn.WORKLOADS["plain-M10"]
    inp = syn.workload_system(wl)
    m = _member(afq, inp, W, wl.dt, 4, taylor_order=6, ortho_every=2, pc_every=pc)
    g = afq.Group([m])
    em = _np(g.propagate(steps, step0)[0])
    o = Oracle.from_inputs(inp)
    st = o.init_walkers(W)
    oe = o.propagate(st, steps, wl.dt, 4, step0,
                     OOptions(taylor_order=6, ortho_every=2, pc_every=pc, e_trial=m.opt.e_trial))
    assert np.max(np.abs(em - oe)) <= 1e-9
    assert np.allclose(_np(m.walkers.weight), st.weight, rtol=1e-9)


def test_group_matches_per_kernel_chain(afq):
    """A member's run equals afqmc_propagate's FP64 chain on the same system
    and fields (M = 12, 5/4 electrons, 36 vectors, 96 walkers, 12 steps with
    MGS and a comb): E_mix within 1e-10 relative."""
    _say("group vs chain M=12")
    inp = syn.make_system(12, 5, 4, 36, 8.0, seed=31)
    kw = dict(taylor_order=6, ortho_every=3, pc_every=6)
    m = _member(afq, inp, 96, 0.005, 2, **kw)
    em = _np(afq.Group([m]).propagate(12, 0)[0])
    c = _member(afq, inp, 96, 0.005, 2, **kw)
    ec = _np(afq.propagate(c.ham, c.trial, c.walkers, 12, 0.005, 2, 0, c.opt))
    assert np.all(np.isfinite(em))
    assert np.max(np.abs(em - ec)) <= 1e-10 * np.max(np.abs(ec))


def _uneven_systems():
    """Three systems of uneven M, N, n_chol and walker count, one with a comb."""
    return [
        (syn.make_system(10, 5, 5, 40, 8.0, seed=0), 64, dict(taylor_order=6, ortho_every=2), 0, 0),
        (syn.make_system(12, 5, 4, 36, 8.0, seed=3), 128, dict(taylor_order=6, ortho_every=2), 5, 7),
        (syn.make_system(14, 4, 3, 30, 8.0, seed=9), 33,
         dict(taylor_order=4, ortho_every=3, pc_every=4), 11, 0),
    ]


def test_group_results_same_alone_and_in_group(afq):
    """Each system's E_mix and final walkers are bitwise the same when it
    runs alone and when it runs in a group with two others of other sizes."""
    _say("group alone vs in group")
    specs = _uneven_systems()
    n = 14
    alone = []
    for inp, W, kw, seed, sid in specs:
        m = _member(afq, inp, W, 0.005, seed, system_id=sid, **kw)
        e = _np(afq.Group([m]).propagate(n, 0)[0])
        alone.append((e, _state(m)))
    members = [_member(afq, inp, W, 0.005, seed, system_id=sid, **kw)
               for inp, W, kw, seed, sid in specs]
    g = afq.Group(members)
    assert g.config[1] == 4  # segments end at the combs of the third member
    em = [_np(e) for e in g.propagate(n, 0)]
    for k, m in enumerate(members):
        assert np.all(np.isfinite(em[k]))
        assert np.array_equal(em[k], alone[k][0])
        for x, y in zip(_state(m), alone[k][1]):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("threads", [64, 128, 512])
def test_group_launch_shape_does_not_change_results(afq, threads):
    """Threads per walker block change the work split, not one rounding."""
    _say(f"group launch shape threads={threads}")
    specs = _uneven_systems()
    ref, other = [], []
    for shape, out in (((256, 4), ref), ((threads, 4), other)):
        members = [_member(afq, inp, W, 0.005, seed, system_id=sid, **kw)
                   for inp, W, kw, seed, sid in specs]
        g = afq.Group(members)
        g.set_config(*shape)
        out.append([_np(e) for e in g.propagate(9, 2)])
        out.append([_state(m) for m in members])
    for a, b in zip(ref[0], other[0]):
        assert np.array_equal(a, b)
    for sa, sb in zip(ref[1], other[1]):
        for x, y in zip(sa, sb):
            assert np.array_equal(x, y)


def test_group_segment_length_does_not_change_results(afq):
    """Without combs the segment length is free: 7 and 20 give the same bits."""
    _say("group segment length")
    inp = syn.make_system(12, 3, 3, 24, 8.0, seed=5)
    outs = []
    for K in (7, 20):
        m = _member(afq, inp, 50, 0.005, 1, taylor_order=6, ortho_every=2)
        g = afq.Group([m])
        g.set_config(128, K)
        outs.append((_np(g.propagate(23, 0)[0]), _state(m)))
    assert np.array_equal(outs[0][0], outs[1][0])
    for x, y in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(x, y)


def test_group_tuner_keeps_state_and_caches(afq, tmp_path):
    """The autotuner restores the walkers it timed on, writes its choice to
    the JSON cache, and a new group of the same shapes takes it from there."""
    _say("group tuner")
    path = str(tmp_path / "tune.json")
    afq.tune_cache_path(path)
    try:
        inp = syn.make_system(10, 5, 5, 40, 8.0, seed=0)
        ref = _member(afq, inp, 64, 0.005, 0, taylor_order=6, ortho_every=2)
        e_ref = _np(afq.Group([ref]).propagate(10, 0)[0])
        m = _member(afq, inp, 64, 0.005, 0, taylor_order=6, ortho_every=2)
        g = afq.Group([m])
        assert g.config[2] == 0
        us = g.tune(steps=20)
        assert us > 0 and g.config[2] == 1
        e = _np(g.propagate(10, 0)[0])
        assert np.array_equal(e, e_ref)
        with open(path) as f:
            data = json.load(f)
        (entry,) = data["entries"].values()
        assert entry["threads"] == g.config[0] and entry["segment"] == g.config[1]
        m2 = _member(afq, inp, 64, 0.005, 0, taylor_order=6, ortho_every=2)
        g2 = afq.Group([m2])
        assert g2.config == (g.config[0], g.config[1], 2)
    finally:
        afq.tune_cache_path(None)
        os.environ.pop("AFQMC_TUNE_CACHE", None)


def test_group_rejects_unsupported_members(afq):
    """Multi-determinant trials, the hybrid weights and systems beyond the
    resident kernel's limits are refused before any work."""
    _say("group rejects")
    for M, n, G in ((70, 10, 20), (20, 5, 100)):  # M > 64; operators beyond one CU's LDS
        inp = syn.make_system(M, n, n, G, 8.0, seed=2)
        m = _member(afq, inp, 4, 0.005, 0)
        assert not afq.resident_supported(m.trial)
        with pytest.raises(afq.AfqmcError) as e:
            afq.Group([m])
        assert e.value.status == -7
    small = syn.make_system(10, 5, 5, 40, 8.0, seed=0)
    h = _member(afq, small, 4, 0.005, 0, weight_mode="hybrid", meas_every=2)
    with pytest.raises(afq.AfqmcError):
        afq.Group([h])
