"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Every case prints its name before running so that a failing GPU step can be
identified from the log.  FP64 bar: mixed energy within 1e-9 Ha over 100
steps; per-walker E_L within 1e-11 relative.  FP32 contractions: stated
per-case tolerances in Ha.
"""
import math
import sys

import numpy as np
import pytest

import afqmc_synth as syn
from oracle import Oracle, Options as OOptions, gaussian_fields

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


def _make(afq, inp, W, mf=True):
    ham = afq.Hamiltonian(inp.h, inp.L, inp.e_core)
    coeff = inp.coeff if inp.n_det > 1 else None
    exc = inp.exc if inp.n_det > 1 else None
    trial = afq.Trial(ham, inp.n_up, inp.n_dn, inp.C_up, inp.C_dn, coeff, exc, mf_subtract=mf)
    w = afq.Walkers(trial, W)
    return ham, trial, w


def _routes(trial):
    """Exchange routes the trial offers: the Ltil route always, Q where built."""
    return ["ltilde", "q"] if trial.exchange_route == "q" else ["ltilde"]


def _set_phi(w, phi):
    w.phi_re.copy_(torch.from_numpy(np.ascontiguousarray(phi.real)))
    w.phi_im.copy_(torch.from_numpy(np.ascontiguousarray(phi.imag)))


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _wrap(a):
    return (a + np.pi) % (2 * np.pi) - np.pi


# --------------------------------------------------------------------------

@pytest.mark.parametrize("W,G,t,sys_id", [(37, 41, 0, 0), (5, 250, 17, 3), (64, 1, 99, 0)])
def test_fields_match_oracle(afq, W, G, t, sys_id):
    _say(f"fields W={W} G={G} t={t} sys={sys_id}")
    x = _np(afq.fields(11, t, W, G, sys_id))
    ref = gaussian_fields(11, t, np.arange(W), G, sys_id)
    assert np.max(np.abs(x - ref)) < 1e-13


def test_local_energy_at_trial_equals_oracle(afq):
    _say("local energy at trial, plain-M10")
    inp = syn.workload_system(syn.WORKLOADS["plain-M10"])
    ham, trial, w = _make(afq, inp, 8)
    afq.walkers_from_trial(ham, trial, w)
    e = afq.local_energy(ham, trial, w)
    o = Oracle.from_inputs(inp)
    ref = o.init_walkers(1).eloc[0].real
    assert abs(e - ref) < 1e-11 * abs(ref)
    assert np.allclose(_np(w.eloc[0]), ref, rtol=1e-11, atol=0)


@pytest.mark.parametrize("M,n_up,n_dn,G,W", [(10, 5, 5, 40, 16), (23, 7, 4, 37, 9),
                                               (50, 25, 25, 250, 6), (40, 17, 0, 30, 5),
                                               (29, 20, 9, 33, 7), (70, 31, 32, 41, 3),
                                               (70, 40, 33, 23, 3), (12, 5, 0, 30, 130),
                                               (16, 7, 6, 40, 65)])
def test_local_energy_random_walkers_fp64(afq, M, n_up, n_dn, G, W):
    _say(f"local energy random walkers M={M} N={n_up}/{n_dn} G={G} W={W}")
    inp = syn.make_system(M, n_up, n_dn, G, 8.0, seed=M + G, e_core=0.75)
    ham, trial, w = _make(afq, inp, W)
    re, im = syn.random_walkers(M, n_up, n_dn, W, seed=3, scale=0.3)
    D0 = np.concatenate([inp.C_up[:, :n_up], inp.C_dn[:, :n_dn]], axis=1)
    phi = D0[None] + re + 1j * im
    o = Oracle.from_inputs(inp)
    m = o.measure(phi)
    for route in _routes(trial):
        trial.exchange_route = route
        _set_phi(w, phi)
        afq.local_energy(ham, trial, w)
        el = _np(w.eloc[0]) + 1j * _np(w.eloc[1])
        ls = _np(w.logovlp[0]) + 1j * _np(w.logovlp[1])
        assert np.allclose(el, m["eloc"], rtol=1e-10, atol=1e-10), route
        assert np.allclose(ls.real, m["logS"].real, atol=1e-10)
        assert np.allclose(_wrap(ls.imag - m["logS"].imag), 0.0, atol=1e-10)


@pytest.mark.parametrize("M,n_up,n_dn,G,W", [(23, 7, 4, 37, 9), (29, 20, 9, 33, 7),
                                               (50, 25, 25, 250, 6), (40, 17, 0, 30, 5),
                                               (70, 40, 33, 23, 3), (90, 50, 64, 19, 2),
                                               (80, 40, 20, 21, 3), (75, 49, 0, 17, 2),
                                               (12, 5, 0, 30, 130), (16, 7, 6, 40, 65)])
def test_local_energy_random_walkers_fp32(afq, M, n_up, n_dn, G, W):
    """FP32 contractions (reached through a zero-step propagate, which
    refreshes E_L with the step's precision): relative 1e-5.  The walkers
    are 0.1-scale perturbations of D_0 (overlap condition numbers below 10):
    the FP32 error of E_L grows with cond(S) since Theta carries S^-1."""
    _say(f"local energy random walkers fp32 M={M} N={n_up}/{n_dn} G={G} W={W}")
    inp = syn.make_system(M, n_up, n_dn, G, 8.0, seed=M + G, e_core=0.75)
    ham, trial, w = _make(afq, inp, W)
    re, im = syn.random_walkers(M, n_up, n_dn, W, seed=3, scale=0.1)
    D0 = np.concatenate([inp.C_up[:, :n_up], inp.C_dn[:, :n_dn]], axis=1)
    phi = D0[None] + re + 1j * im
    m = Oracle.from_inputs(inp).measure(phi)
    for route in _routes(trial):
        trial.exchange_route = route
        _set_phi(w, phi)
        afq.propagate(ham, trial, w, 0, 0.01, 0, 0, afq.Options(chol_prec="fp32", taylor_prec="fp32"))
        el = _np(w.eloc[0]) + 1j * _np(w.eloc[1])
        err = np.abs(el - m["eloc"]) / np.abs(m["eloc"])
        print(f"fp32 {route}: max rel dE_L = {err.max():.3e}")
        assert err.max() <= 1e-5


@pytest.mark.parametrize("M,n_up,n_dn,G,W", [(23, 7, 4, 37, 9), (50, 25, 25, 250, 6),
                                               (40, 17, 0, 30, 5), (80, 40, 20, 21, 3),
                                               (90, 50, 64, 19, 2), (75, 49, 0, 17, 2),
                                               (130, 64, 64, 9, 2), (12, 5, 0, 30, 130),
                                               (16, 7, 6, 40, 65)])
@pytest.mark.parametrize("prec,tol", [("bf16", 5e-3), ("bf16x3", 2e-5)])
def test_local_energy_random_walkers_bf16(afq, M, n_up, n_dn, G, W, prec, tol):
    """BF16 and split-BF16 exchange contraction (Ltil Theta with FP32
    accumulation; Sec. III single-precision contractions) on row-tile counts
    1 to 4 (the register-resident kernel, unequal and empty spins, G not a
    multiple of the four wavefronts, ragged k chunks, the largest spin of 64
    electrons): E_L against the FP64 oracle, relative bound 5e-3 for BF16
    (8 significant bits per operand) and 2e-5 for the split form (16)."""
    _say(f"local energy random walkers {prec} M={M} N={n_up}/{n_dn} G={G} W={W}")
    inp = syn.make_system(M, n_up, n_dn, G, 8.0, seed=M + G, e_core=0.75)
    ham, trial, w = _make(afq, inp, W)
    trial.exchange_route = "ltilde"
    re, im = syn.random_walkers(M, n_up, n_dn, W, seed=3, scale=0.1)
    D0 = np.concatenate([inp.C_up[:, :n_up], inp.C_dn[:, :n_dn]], axis=1)
    phi = D0[None] + re + 1j * im
    m = Oracle.from_inputs(inp).measure(phi)
    _set_phi(w, phi)
    afq.propagate(ham, trial, w, 0, 0.01, 0, 0, afq.Options(chol_prec=prec, taylor_prec="fp32"))
    el = _np(w.eloc[0]) + 1j * _np(w.eloc[1])
    err = np.abs(el - m["eloc"]) / np.abs(m["eloc"])
    print(f"{prec}: max rel dE_L = {err.max():.3e}")
    assert np.all(np.isfinite(el))
    assert err.max() <= tol


def _run_both(afq, inp, W, n_steps, dt, opt_kw, prec=("fp64", "fp64"), seed=0, oracle_walkers=None):
    ham, trial, w = _make(afq, inp, W)
    afq.walkers_from_trial(ham, trial, w)
    et = afq.local_energy(ham, trial, w)
    opt = afq.Options(e_trial=et, chol_prec=prec[0], taylor_prec=prec[1], **opt_kw)
    em = _np(afq.propagate(ham, trial, w, n_steps, dt, seed, 0, opt))
    o = Oracle.from_inputs(inp)
    st = o.init_walkers(W)
    oe = o.propagate(st, n_steps, dt, seed, 0, OOptions(e_trial=et, **opt_kw))
    return em, oe, w, st


def test_propagate_plain_fp64_parity_100_steps(afq):
    """Plain FP64 workload (M=10, 5/5, 40 vectors, 64 walkers, 100 steps)."""
    _say("propagate plain-M10 fp64 100 steps")
    wl = syn.WORKLOADS["plain-M10"]
    inp = syn.workload_system(wl)
    em, oe, w, st = _run_both(afq, inp, wl.n_walkers, wl.n_steps, wl.dt,
                              dict(taylor_order=6, ortho_every=wl.ortho_every, pc_every=0))
    print("max |dE_mix| =", np.max(np.abs(em - oe)), "alive", int(np.sum(st.weight > 0)))
    assert np.max(np.abs(em - oe)) <= 1e-9
    assert np.allclose(_np(w.weight), st.weight, rtol=1e-9, atol=1e-12)
    el = _np(w.eloc[0])
    assert np.allclose(el[st.weight > 0], st.eloc.real[st.weight > 0], rtol=1e-9)


def test_propagate_with_comb_fp64_parity(afq):
    _say("propagate plain-M10 fp64 with comb every 5")
    wl = syn.WORKLOADS["plain-M10"]
    inp = syn.workload_system(wl)
    em, oe, w, st = _run_both(afq, inp, 64, 30, wl.dt, dict(taylor_order=6, ortho_every=2, pc_every=5))
    assert np.max(np.abs(em - oe)) <= 1e-9
    assert np.allclose(_np(w.weight), st.weight, rtol=1e-9)


def test_propagate_is_deterministic(afq):
    _say("determinism")
    wl = syn.WORKLOADS["plain-M10"]
    inp = syn.workload_system(wl)
    outs = []
    for _ in range(2):
        ham, trial, w = _make(afq, inp, 32)
        afq.walkers_from_trial(ham, trial, w)
        opt = afq.Options(e_trial=-10.0, ortho_every=2, pc_every=4)
        outs.append((_np(afq.propagate(ham, trial, w, 12, 0.005, 7, 3, opt)), _np(w.phi_re)))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_split_calls_equal_one_call(afq):
    _say("split propagate calls")
    inp = syn.workload_system(syn.WORKLOADS["plain-M10"])
    ham, trial, w = _make(afq, inp, 16)
    afq.walkers_from_trial(ham, trial, w)
    opt = afq.Options(e_trial=-10.0, ortho_every=3, pc_every=0)
    e_all = _np(afq.propagate(ham, trial, w, 10, 0.005, 5, 0, opt))
    ham2, trial2, w2 = _make(afq, inp, 16)
    afq.walkers_from_trial(ham2, trial2, w2)
    e1 = _np(afq.propagate(ham2, trial2, w2, 4, 0.005, 5, 0, opt))
    e2 = _np(afq.propagate(ham2, trial2, w2, 6, 0.005, 5, 4, opt))
    assert np.allclose(np.concatenate([e1, e2]), e_all, rtol=0, atol=1e-11)


@pytest.mark.parametrize("M,nu,nd,W", [(30, 9, 6, 7), (64, 20, 0, 5), (80, 12, 11, 3)])
def test_orthonormalize_parity(afq, M, nu, nd, W):
    """MGS per walker and spin: one wavefront per matrix up to M = 64 (M = 64
    fills every lane), the block form above."""
    _say(f"orthonormalize M={M} N={nu}/{nd} W={W}")
    inp = syn.make_system(M, nu, nd, 20, 8.0, seed=4)
    ham, trial, w = _make(afq, inp, W)
    re, im = syn.random_walkers(M, nu, nd, W, seed=5, scale=0.4)
    phi = np.concatenate([inp.C_up[:, :nu], inp.C_dn[:, :nd]], axis=1)[None] + re + 1j * im
    _set_phi(w, phi)
    afq.local_energy(ham, trial, w)
    e0 = _np(w.eloc[0]).copy()
    afq.orthonormalize(ham, trial, w)
    o = Oracle.from_inputs(inp)
    st = o.init_walkers(W, phi=phi)
    o.orthonormalize(st)
    got = _np(w.phi_re) + 1j * _np(w.phi_im)
    assert np.allclose(got, st.phi, atol=1e-12)
    ls = _np(w.logovlp[0]) + 1j * _np(w.logovlp[1])
    assert np.allclose(ls.real, st.logS.real, atol=1e-10)
    assert np.allclose(_wrap(ls.imag - st.logS.imag), 0, atol=1e-10)
    afq.local_energy(ham, trial, w)
    assert np.allclose(_np(w.eloc[0]), e0, rtol=1e-11)


@pytest.mark.parametrize("W", [1, 7, 64, 1000])
def test_reconfigure_parity(afq, W):
    _say(f"reconfigure W={W}")
    inp = syn.make_system(6, 2, 2, 4, 8.0, seed=6)
    ham, trial, w = _make(afq, inp, W)
    rng = np.random.default_rng(W)
    re, im = syn.random_walkers(6, 2, 2, W, seed=W, scale=0.3)
    D0 = np.concatenate([inp.C_up[:, :2], inp.C_dn[:, :2]], axis=1)
    phi = D0[None] + re + 1j * im
    _set_phi(w, phi)
    wts = rng.exponential(size=W)
    wts[rng.random(W) < 0.25] = 0.0
    if not np.any(wts > 0):
        wts[0] = 1.0
    w.weight.copy_(torch.from_numpy(wts))
    afq.local_energy(ham, trial, w)
    el_before = _np(w.eloc[0]).copy()
    norm = afq.reconfigure(trial, w, 13, 4)
    o = Oracle.from_inputs(inp)
    st = o.init_walkers(W, phi=phi)
    st.weight = wts.copy()
    onorm = o.reconfigure(st, 13, 4)
    assert norm == pytest.approx(onorm, rel=1e-14)
    got = _np(w.phi_re) + 1j * _np(w.phi_im)
    assert np.array_equal(got, st.phi)   # bit-exact copies of the same parents
    assert np.array_equal(_np(w.weight), np.ones(W))
    # parents are unique: E_L were copied along
    assert np.all(np.isin(_np(w.eloc[0]), el_before))


def test_dead_walkers_reset_like_the_oracle(afq):
    """Walkers whose weight is zero or not finite die (Sec. II phaseless
    constraint): reset to D_0 with its reference log S, E_L and v, weight 0,
    still propagated, left out of E_mix.  Two of 16 walkers are killed before
    a 3-step FP64 run; every walker's state and E_mix match the oracle."""
    _say("dead-walker reset plain-M10 fp64")
    wl = syn.WORKLOADS["plain-M10"]
    inp = syn.workload_system(wl)
    W = 16
    ham, trial, w = _make(afq, inp, W)
    afq.walkers_from_trial(ham, trial, w)
    et = afq.local_energy(ham, trial, w)
    kw = dict(taylor_order=6, ortho_every=2, pc_every=0, e_trial=et)
    afq.propagate(ham, trial, w, 2, wl.dt, 9, 0, afq.Options(**kw))
    o = Oracle.from_inputs(inp)
    st = o.init_walkers(W)
    o.propagate(st, 2, wl.dt, 9, 0, OOptions(**kw))
    wt = _np(w.weight).copy()
    wt[3], wt[11] = 0.0, np.nan
    w.weight.copy_(torch.from_numpy(wt))
    st.weight[3], st.weight[11] = 0.0, np.nan
    em = _np(afq.propagate(ham, trial, w, 3, wl.dt, 9, 2, afq.Options(**kw)))
    oe = o.propagate(st, 3, wl.dt, 9, 2, OOptions(**kw))
    assert np.max(np.abs(em - oe)) <= 1e-9
    got_w = _np(w.weight)
    assert got_w[3] == 0.0 and got_w[11] == 0.0
    assert np.allclose(got_w, st.weight, rtol=1e-9, atol=0)
    phi = _np(w.phi_re) + 1j * _np(w.phi_im)
    assert np.allclose(phi, st.phi, rtol=0, atol=1e-10)
    D0 = np.concatenate([inp.C_up[:, :inp.n_up], inp.C_dn[:, :inp.n_dn]], axis=1)
    for k in (3, 11):
        assert np.allclose(phi[k], D0, atol=1e-14)
    ls = _np(w.logovlp[0]) + 1j * _np(w.logovlp[1])
    el = _np(w.eloc[0]) + 1j * _np(w.eloc[1])
    assert np.allclose(ls.real, st.logS.real, atol=1e-9)
    assert np.allclose(_wrap(ls.imag - st.logS.imag), 0, atol=1e-9)
    assert np.allclose(el, st.eloc, rtol=1e-10)


def test_reconfigure_all_dead_reports_nonfinite(afq):
    """A comb over an all-dead population: AFQMC_ERR_NONFINITE, walkers left
    as they are (weights stay 0)."""
    _say("reconfigure all dead")
    inp = syn.make_system(6, 2, 2, 4, 8.0, seed=6)
    ham, trial, w = _make(afq, inp, 9)
    afq.walkers_from_trial(ham, trial, w)
    re, im = syn.random_walkers(6, 2, 2, 9, seed=3, scale=0.3)
    D0 = np.concatenate([inp.C_up[:, :2], inp.C_dn[:, :2]], axis=1)
    _set_phi(w, D0[None] + re + 1j * im)
    w.weight.zero_()
    before = _np(w.phi_re).copy()
    with pytest.raises(afq.AfqmcError) as e:
        afq.reconfigure(trial, w, 13, 4)
    assert e.value.status == -6
    assert np.array_equal(_np(w.weight), np.zeros(9))
    assert np.array_equal(_np(w.phi_re), before)


def _one_step_sampled(afq, inp, W, sample, dt, prec, taylor_order=6, route=None):
    """One step of all W walkers from the reference on the GPU; the oracle
    repeats the step for the sampled walkers alone (counter-based fields)."""
    ham, trial, w = _make(afq, inp, W)
    if route is not None:
        trial.exchange_route = route
    afq.walkers_from_trial(ham, trial, w)
    et = afq.local_energy(ham, trial, w)
    opt = afq.Options(taylor_order=taylor_order, e_trial=et, chol_prec=prec[0], taylor_prec=prec[1])
    afq.propagate(ham, trial, w, 1, dt, 3, 0, opt)
    el = _np(w.eloc[0]) + 1j * _np(w.eloc[1])
    wt = _np(w.weight)
    o = Oracle.from_inputs(inp)
    st = o.init_walkers(len(sample), index=np.asarray(sample))
    o.propagate(st, 1, dt, 3, 0, OOptions(taylor_order=taylor_order, e_trial=et))
    return el[sample], wt[sample], st


@pytest.mark.parametrize("name,prec,rel_tol,abs_tol,route", [
    ("hchain-M50", ("fp64", "fp64"), 1e-12, 1e-9, "q"),
    ("hchain-M50", ("fp64", "fp64"), 1e-12, 1e-9, "ltilde"),
    ("hchain-M50", ("fp32", "fp32"), None, 1e-4, "q"),
    ("hchain-M50", ("fp32", "fp32"), None, 1e-4, "ltilde"),
    ("hchain-M50-literal", ("fp64", "fp64"), 1e-9, None, "q"),
    ("hchain-M50-literal", ("fp32", "fp32"), 2e-6, None, "q"),
    ("hchain-M50-literal", ("fp32", "fp32"), 2e-6, None, "ltilde")])
def test_hchain_full_size_one_step_sampled(afq, name, prec, rel_tol, abs_tol, route):
    """Hydrogen-chain shapes at full size (1024 walkers, the benchmark's
    launch configuration): per-walker E_L and weight after one step on 8
    sampled walkers vs the oracle.  With the health-scaled vectors the FP32
    bound is the 0.1 mHa gate per walker; with the unscaled recipe
    (|E_L| ~ 1e4 Ha) FP32 is bounded relative, 2e-6."""
    wl = syn.WORKLOADS[name]
    inp = syn.workload_system(wl)
    sample = [0, 1, 255, 256, 511, 700, 1022, 1023]
    _say(f"{name} full size one step {prec} route {route}")
    el, wt, st = _one_step_sampled(afq, inp, wl.n_walkers, sample, wl.dt, prec, route=route)
    alive = st.weight > 0
    err = np.abs(el - st.eloc)[alive]
    rel = err / np.abs(st.eloc[alive])
    print(f"{name} {prec}: alive {int(alive.sum())}/8, max |dE_L| = {np.max(err):.3e} Ha,"
          f" max rel {np.max(rel):.3e}")
    assert np.array_equal(wt > 0, alive)
    if rel_tol is not None:
        assert np.max(rel) <= rel_tol
    if abs_tol is not None:
        assert np.max(err) <= abs_tol
    wrel = 50 * (rel_tol if rel_tol is not None else abs_tol / np.min(np.abs(st.eloc[alive])))
    assert np.allclose(wt[alive], st.weight[alive], rtol=wrel)


def test_fp32_trajectory_hchain(afq):
    """Hydrogen-chain workload, 32 walkers, 20 steps, FP32 contractions and
    Taylor vs the FP64 oracle's mixed energy: within the 0.1 mHa gate."""
    _say("fp32 hchain 32 walkers 20 steps")
    wl = syn.WORKLOADS["hchain-M50"]
    inp = syn.workload_system(wl)
    em, oe, w, st = _run_both(afq, inp, 32, 20, wl.dt,
                              dict(taylor_order=6, ortho_every=10, pc_every=0), prec=("fp32", "fp32"))
    err = np.max(np.abs(em - oe))
    print("fp32 hchain: max |dE_mix| (Ha) =", err, " |E| ~", abs(oe[-1]), "alive", int(np.sum(st.weight > 0)))
    assert np.all(np.isfinite(oe))
    assert err <= 1e-4


def test_fp64_trajectory_hchain(afq):
    _say("fp64 hchain 32 walkers 20 steps")
    wl = syn.WORKLOADS["hchain-M50"]
    inp = syn.workload_system(wl)
    em, oe, w, st = _run_both(afq, inp, 32, 20, wl.dt, dict(taylor_order=6, ortho_every=10, pc_every=0))
    err = np.max(np.abs(em - oe))
    print("fp64 hchain: max |dE_mix| (Ha) =", err)
    assert err <= 1e-9 * abs(oe[-1])


def _golden_hchain(fname):
    """Stored FP64 oracle sums (see tests/golden/make_hchain_reference.py)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", fname)
    et, num, den, walkers = None, [], [], []
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                continue
            p = line.split()
            if p[0] == "e_trial":
                et = float(p[1])
            elif p[0] == "step":
                num.append(float(p[2]))
                den.append(float(p[3]))
            elif p[0] == "walker":
                walkers.append([float(v) for v in p[2:]])
    return et, np.array(num), np.array(den), np.array(walkers)


def _gpu_hchain(afq, W, n_steps, et, prec, pc=False):
    wl = syn.WORKLOADS["hchain-M50"]
    inp = syn.workload_system(wl)
    ham, trial, w = _make(afq, inp, W)
    afq.walkers_from_trial(ham, trial, w)
    opt = afq.Options(taylor_order=wl.taylor_order, ortho_every=wl.ortho_every,
                      pc_every=wl.pc_every if pc else 0,
                      e_trial=et, chol_prec=prec[0], taylor_prec=prec[1])
    em = _np(afq.propagate(ham, trial, w, n_steps, wl.dt, 1, 0, opt))
    return em, w


@pytest.mark.parametrize("prec,tol", [(("fp64", "fp64"), 1e-6), (("fp32", "fp32"), 1e-4)])
def test_hchain_gate_all_walkers_100_steps(afq, prec, tol):
    """The 0.1 mHa gate at the benchmark's size: all 1024 walkers, 100 steps,
    population control off, E_mix per step vs the stored FP64 oracle run.
    FP64 is held to 1e-6 Ha: differences in rounding order (1e-16 relative)
    grow along each trajectory, and without population control the weights
    spread over many orders of magnitude, so E_mix follows a few walkers."""
    _say(f"hchain gate 1024 walkers 100 steps {prec}")
    et, num, den, _ = _golden_hchain("hchain-M50_W1024_T100.txt")
    em, w = _gpu_hchain(afq, 1024, 100, et, prec)
    ref = num / den
    err = np.abs(em - ref)
    print(f"{prec}: max |dE_mix| over 100 steps = {err.max():.3e} Ha (|E| ~ {abs(ref[-1]):.1f}),"
          f" alive {int((_np(w.weight) > 0).sum())}/1024;"
          f" |dE_mix| at steps 1, 10, 50, 100: {err[0]:.1e} {err[9]:.1e} {err[49]:.1e} {err[99]:.1e}")
    assert np.all(np.isfinite(ref))
    assert err.max() <= tol


# --------------------------------------------------------------------------
# Multi-determinant trial (SMW route on the GPU, direct per-determinant
# matrix elements in the oracle)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-5)])
def test_multidet_local_energy_random_walkers(afq, prec, tol):
    _say(f"multidet local energy random walkers {prec}")
    M, nu, nd, G = 14, 4, 3, 9
    inp = syn.make_system(M, nu, nd, G, 4.0, n_det=40, seed=8, e_core=0.3)
    ham, trial, w = _make(afq, inp, 6)
    D0 = np.concatenate([inp.C_up[:, :nu], inp.C_dn[:, :nd]], axis=1)
    re, im = syn.random_walkers(M, nu, nd, 6, seed=2, scale=0.3)
    phi = D0[None] + re + 1j * im
    phi[5] = D0          # on the reference: every excited overlap is zero
    _set_phi(w, phi)
    if prec == "fp64":
        afq.local_energy(ham, trial, w)
    else:  # the FP32 contraction path is reached through a zero-step propagate
        afq.propagate(ham, trial, w, 0, 0.01, 0, 0, afq.Options(chol_prec="fp32"))
    o = Oracle.from_inputs(inp)
    m = o.measure(phi)
    el = _np(w.eloc[0]) + 1j * _np(w.eloc[1])
    ls = _np(w.logovlp[0]) + 1j * _np(w.logovlp[1])
    print(prec, "max rel dE_L", np.max(np.abs(el - m["eloc"]) / np.abs(m["eloc"])))
    assert np.allclose(el, m["eloc"], rtol=tol, atol=0)
    assert np.allclose(ls.real, m["logS"].real, atol=1e-10)
    assert np.allclose(_wrap(ls.imag - m["logS"].imag), 0.0, atol=1e-10)


def test_multidet_exact_fci_trial_zero_variance(afq):
    """Exact ground state as a multi-determinant trial in a rotated orbital
    basis (M=4, 2+2): every live walker's E_L equals the exact eigenvalue at
    every step of a real run with MGS and comb."""
    import fock
    _say("multidet exact FCI trial zero variance")
    M, nu, nd = 4, 2, 2
    inp = syn.make_system(M, nu, nd, 5, 3.0, seed=13, e_core=0.2)
    rng = np.random.default_rng(17)
    C = np.linalg.qr(rng.standard_normal((M, M)))[0]
    exc, coeff, efci = fock.fci_trial(inp.h, inp.L, inp.e_core, C, nu, nd)
    ham = afq.Hamiltonian(inp.h, inp.L, inp.e_core)
    trial = afq.Trial(ham, nu, nd, C, C, coeff, exc)
    w = afq.Walkers(trial, 16)
    afq.walkers_from_trial(ham, trial, w)
    e0 = afq.local_energy(ham, trial, w)
    assert abs(e0 - efci) < 1e-10
    opt = afq.Options(ortho_every=2, pc_every=3, e_trial=efci)
    em = _np(afq.propagate(ham, trial, w, 12, 0.02, 2, 0, opt))
    wt = _np(w.weight)
    el = _np(w.eloc[0])
    assert np.all(np.abs(em - efci) < 1e-9)
    assert np.allclose(el[wt > 0], efci, atol=1e-9)


def test_multidet_propagate_fp64_parity(afq):
    _say("multidet propagate fp64 parity")
    M, nu, nd, G = 24, 7, 5, 30
    inp = syn.make_system(M, nu, nd, G, 8.0, n_det=25, seed=31)
    em, oe, w, st = _run_both(afq, inp, 12, 10, 0.005, dict(taylor_order=6, ortho_every=2, pc_every=5))
    print("multidet max |dE_mix| =", np.max(np.abs(em - oe)), "alive", int(np.sum(st.weight > 0)))
    assert np.max(np.abs(em - oe)) <= 1e-9 * max(1.0, np.max(np.abs(oe)))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-5)])
def test_tm_multidet_full_size_sampled(afq, prec, tol):
    """tm-multidet-M120 at full size (2048 walkers, 100 determinants, 600
    vectors): E_L and log S of walkers perturbed from the reference, from the
    multi-determinant kernels in the launch shape the step uses; the oracle
    evaluates 3 sampled walkers directly."""
    wl = syn.WORKLOADS["tm-multidet-M120"]
    inp = syn.workload_system(wl)
    _say(f"tm-multidet full size sampled {prec}")
    W = wl.n_walkers
    ham, trial, w = _make(afq, inp, W)
    D0 = np.concatenate([inp.C_up[:, :wl.n_up], inp.C_dn[:, :wl.n_dn]], axis=1)
    re, im = syn.random_walkers(wl.M, wl.n_up, wl.n_dn, W, seed=4, scale=0.05)
    phi = D0[None] + re + 1j * im
    _set_phi(w, phi)
    if prec == "fp64":
        afq.local_energy(ham, trial, w)
    else:
        afq.propagate(ham, trial, w, 0, wl.dt, 0, 0, afq.Options(chol_prec="fp32"))
    el = _np(w.eloc[0]) + 1j * _np(w.eloc[1])
    ls = _np(w.logovlp[0]) + 1j * _np(w.logovlp[1])
    sample = [0, 1000, 2047]
    o = Oracle.from_inputs(inp)
    m = o.measure(phi[sample])
    rel = np.abs(el[sample] - m["eloc"]) / np.abs(m["eloc"])
    print(f"{prec}: max rel dE_L {np.max(rel):.3e}")
    assert np.max(rel) <= tol
    assert np.allclose(ls.real[sample], m["logS"].real, atol=1e-9)
    assert np.allclose(_wrap(ls.imag[sample] - m["logS"].imag), 0.0, atol=1e-9)


# --------------------------------------------------------------------------
# Precision sweep at the 200-orbital size
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def sweep_case():
    wl = syn.WORKLOADS["sweep-M200"]
    inp = syn.workload_system(wl)
    D0 = np.concatenate([inp.C_up[:, :wl.n_up], inp.C_dn[:, :wl.n_dn]], axis=1)
    re, im = syn.random_walkers(wl.M, wl.n_up, wl.n_dn, wl.n_walkers, seed=6, scale=0.03)
    phi = D0[None] + re + 1j * im
    sample = [0, 1023]
    o = Oracle.from_inputs(inp)
    ref = o.measure(phi[sample])
    return wl, inp, phi, sample, ref


@pytest.mark.parametrize("prec,tol,route", [("fp64", 1e-9, "q"), ("fp64", 1e-9, "ltilde"),
                                            ("fp32", 5e-5, "q"), ("fp32", 5e-5, "ltilde"),
                                            ("bf16", 1e-1, "ltilde"), ("bf16x3", 1e-4, "ltilde")])
def test_sweep_full_size_local_energy(afq, sweep_case, prec, tol, route):
    """sweep-M200 (M=200, 50/50, 1000 vectors, 1024 walkers): E_L of perturbed
    walkers with the exchange contraction in FP64 / FP32 / BF16 / split BF16
    (FP32 accumulation) against the FP64 oracle on 2 sampled walkers, bound
    in Ha (|E_L| is about 450 Ha): FP64 1e-9; FP32 5e-5 (five times the
    largest one-step error the precision report measures over all walkers);
    BF16 0.1 (three times its 3.4e-2); BF16X3 the 0.1 mHa gate."""
    wl, inp, phi, sample, ref = sweep_case
    _say(f"sweep full size local energy {prec} route {route}")
    ham, trial, w = _make(afq, inp, wl.n_walkers)
    trial.exchange_route = route
    _set_phi(w, phi)
    afq.propagate(ham, trial, w, 0, wl.dt, 0, 0, afq.Options(chol_prec=prec))
    el = (_np(w.eloc[0]) + 1j * _np(w.eloc[1]))[sample]
    err = np.abs(el - ref["eloc"])
    print(f"sweep {prec} {route}: |E_L| ~ {np.abs(ref['eloc']).max():.1f} Ha, max |dE_L| = {err.max():.3e} Ha,"
          f" rel {np.max(err / np.abs(ref['eloc'])):.3e}")
    assert np.max(err) <= tol


@pytest.mark.parametrize("prec,tol", [("bf16", 2e-2), ("bf16x3", 2e-4)])
def test_bf16_propagate_tracks_fp64(afq, prec, tol):
    """BF16 and split-BF16 contractions (propagator build and Ltil Theta; FP32
    Taylor) over 10 steps of the hydrogen-chain workload on 16 walkers: the
    mixed energy against the FP64 oracle, bound in Ha (|E| is about 190 Ha)
    at a few times the drift measured: BF16 2e-2, BF16X3 2e-4 (this includes
    the trajectories' own divergence, not the per-step error alone)."""
    _say(f"{prec} hchain 16 walkers 10 steps")
    wl = syn.WORKLOADS["hchain-M50"]
    inp = syn.workload_system(wl)
    em, oe, w, st = _run_both(afq, inp, 16, 10, wl.dt, dict(taylor_order=6, ortho_every=10, pc_every=0),
                              prec=(prec, "fp32"))
    err = np.max(np.abs(em - oe))
    print(f"{prec} hchain: max |dE_mix| (Ha) =", err, " |E| ~", abs(oe[-1]))
    assert np.all(np.isfinite(em))
    assert err <= tol


def test_sweep_fp64_trajectory_walker_subset(afq):
    """The precision-sweep system (M=200, 50/50, 1000 vectors) in FP64 over
    six steps with MGS every two, on a subset of three walkers (walkers are
    independent without population control and their fields are keyed by
    walker index, so the subset is the full workload's first three walkers):
    E_mix at every step within 1e-8 Ha of the oracle, weights and E_L per
    walker too."""
    _say("sweep-M200 fp64 6 steps, 3 walkers")
    wl = syn.WORKLOADS["sweep-M200"]
    inp = syn.workload_system(wl)
    em, oe, w, st = _run_both(afq, inp, 3, 6, wl.dt, dict(taylor_order=6, ortho_every=2, pc_every=0))
    print("sweep fp64 subset: max |dE_mix| =", np.max(np.abs(em - oe)), "E_mix", oe[-1])
    assert np.all(np.isfinite(oe))
    assert np.max(np.abs(em - oe)) <= 1e-8
    assert np.allclose(_np(w.weight), st.weight, rtol=1e-10, atol=0)
    assert np.allclose(_np(w.eloc[0]), st.eloc.real, rtol=0, atol=1e-8)


@pytest.mark.parametrize("dt_scale", [1.0, 0.1])
def test_literal_hchain_fp64_trajectory_walker_subset(afq, dt_scale):
    """The unscaled hydrogen-chain recipe (|E_L| ~ 4e3 Ha) in FP64 over six
    steps on 16 walkers, without population control.  At the workload's
    dt the phaseless constraint kills walkers step by step (all 16 by the
    sixth step in the oracle): the GPU must kill the same walkers at the same
    steps, and E_mix must agree at every step while any walker lives (NaN
    where none does).  At dt / 10 every walker survives: E_mix, weights and
    E_L per walker within FP64 rounding of the oracle."""
    wl = syn.WORKLOADS["hchain-M50-literal"]
    inp = syn.workload_system(wl)
    dt = wl.dt * dt_scale
    _say(f"hchain-M50-literal fp64 6 steps, 16 walkers, dt {dt}")
    em, oe, w, st = _run_both(afq, inp, 16, 6, dt, dict(taylor_order=6, ortho_every=10, pc_every=0))
    alive_gpu = _np(w.weight) > 0
    print(f"literal dt={dt}: E_mix gpu {em}, oracle {oe}, alive gpu {int(alive_gpu.sum())}"
          f" oracle {int((st.weight > 0).sum())}")
    assert np.array_equal(np.isnan(em), np.isnan(oe))
    fin = np.isfinite(oe)
    assert fin[0]
    assert np.max(np.abs(em[fin] - oe[fin]) / np.abs(oe[fin])) <= 1e-9
    assert np.array_equal(alive_gpu, st.weight > 0)
    if dt_scale < 1.0:
        assert alive_gpu.all()
        assert np.allclose(_np(w.weight), st.weight, rtol=1e-9, atol=0)
        assert np.allclose(_np(w.eloc[0]), st.eloc.real, rtol=1e-9, atol=0)


# --------------------------------------------------------------------------
# Edge cases
# --------------------------------------------------------------------------

def test_zero_variance_one_body_no_cholesky_vectors(afq):
    """No Cholesky vectors (G = 0) and a trial of eigenvectors of h: E_L is the
    sum of occupied eigenvalues for every walker at every step."""
    _say("zero variance one-body, G=0")
    M, nu, nd = 9, 3, 2
    inp = syn.make_system(M, nu, nd, 1, 4.0, seed=5, e_core=1.25)
    L0 = np.zeros((0, M, M))
    eps = np.linalg.eigvalsh(inp.h)
    exact = inp.e_core + eps[:nu].sum() + eps[:nd].sum()
    ham = afq.Hamiltonian(inp.h, L0, inp.e_core)
    trial = afq.Trial(ham, nu, nd, inp.C_up, inp.C_dn)
    w = afq.Walkers(trial, 8)
    afq.walkers_from_trial(ham, trial, w)
    assert abs(afq.local_energy(ham, trial, w) - exact) < 1e-12
    em = _np(afq.propagate(ham, trial, w, 10, 0.01, 1, 0, afq.Options(ortho_every=2, pc_every=5,
                                                                     e_trial=exact)))
    assert np.allclose(em, exact, atol=1e-12)


@pytest.mark.parametrize("W,nu,nd", [(1, 4, 3), (5, 6, 0)])
def test_propagate_edge_shapes_fp64(afq, W, nu, nd):
    _say(f"edge shapes W={W} N={nu}/{nd}")
    inp = syn.make_system(13, nu, nd, 11, 6.0, seed=W + nu)
    em, oe, w, st = _run_both(afq, inp, W, 8, 0.01, dict(taylor_order=6, ortho_every=3, pc_every=4))
    assert np.max(np.abs(em - oe)) <= 1e-9 * max(1.0, np.max(np.abs(oe)))


@pytest.mark.parametrize("M,nu,nd,G,n_det,W,seed", [
    (14, 4, 3, 9, 150, 7, 8),     # three determinants per lane
    (12, 4, 0, 7, 30, 5, 5),      # no electrons of one spin
    (70, 9, 8, 20, 60, 9, 21),    # M > 64: 32 k steps, several row tiles
    (40, 17, 3, 10, 30, 5, 3),    # N > 16: the full-row kernel
    (100, 13, 11, 12, 100, 6, 40),  # 67 rows up (a last row tile of 3), M = 100 of 128 k rows
    (118, 12, 9, 10, 120, 5, 41),   # 67 rows down (a last row tile of 3), M = 118
    (20, 2, 1, 6, 3, 3, 53),      # 4 and 2 rows: one partial row tile per spin
])
def test_multidet_fp32_compact_rows_vs_oracle(afq, M, nu, nd, G, n_det, W, seed):
    """FP32 multi-determinant E_L from the compact-row kernel (only the rows of
    C^T L_g Theta_0 that the determinants read; past its limits, the full-row
    kernel) against the oracle's direct per-determinant evaluation, on walkers
    perturbed from the reference; one walker sits on the reference, where
    every excited overlap is zero.  W is not a multiple of the kernel's four
    walkers per block; the shapes include nearly empty last row tiles and
    k rows past M within the last k block."""
    _say(f"multidet fp32 compact rows M={M} {nu}+{nd} G={G} n_det={n_det} W={W}")
    inp = syn.make_system(M, nu, nd, G, 4.0, n_det=n_det, seed=seed, e_core=0.3)
    ham, trial, w = _make(afq, inp, W)
    D0 = np.concatenate([inp.C_up[:, :nu], inp.C_dn[:, :nd]], axis=1)
    re, im = syn.random_walkers(M, nu, nd, W, seed=seed + 1, scale=0.3)
    phi = D0[None] + re + 1j * im
    phi[W - 1] = D0
    _set_phi(w, phi)
    afq.propagate(ham, trial, w, 0, 0.01, 0, 0, afq.Options(chol_prec="fp32"))
    el = _np(w.eloc[0]) + 1j * _np(w.eloc[1])
    m = Oracle.from_inputs(inp).measure(phi)
    rel = np.abs(el - m["eloc"]) / np.abs(m["eloc"])
    print(f"max rel dE_L {rel.max():.3e}")
    assert np.all(np.isfinite(el))
    assert rel.max() <= 2e-5


def test_multidet_fp32_propagate_tracks_fp64(afq):
    """The FP32 multi-determinant path (its force bias drives the fields'
    shift) against the FP64 path on the same walkers and fields: per-step
    E_mix over 12 steps with MGS and the comb."""
    _say("multidet fp32 propagate tracks fp64")
    M, nu, nd, G = 24, 7, 5, 30
    inp = syn.make_system(M, nu, nd, G, 8.0, n_det=25, seed=31)
    ems = []
    for prec in ("fp64", "fp32"):
        ham, trial, w = _make(afq, inp, 12)
        afq.walkers_from_trial(ham, trial, w)
        et = afq.local_energy(ham, trial, w)
        opt = afq.Options(e_trial=et, chol_prec=prec, taylor_prec=prec, taylor_order=6,
                          ortho_every=2, pc_every=5)
        ems.append(_np(afq.propagate(ham, trial, w, 12, 0.005, 0, 0, opt)))
    err = np.abs(ems[1] - ems[0])
    print(f"max |dE_mix| fp32 vs fp64 = {err.max():.3e} Ha")
    assert np.all(np.isfinite(ems[1]))
    assert err.max() <= 1e-4


def test_multidet_with_only_the_reference_matches_single_det(afq):
    """A two-determinant trial whose second coefficient is 0 gives the
    single-determinant energies (exercises the multi-det kernels' reference
    terms against the single-det kernels)."""
    _say("multidet degenerate to single det")
    M, nu, nd, G = 12, 4, 3, 9
    inp = syn.make_system(M, nu, nd, G, 6.0, n_det=2, seed=4)
    inp.coeff = np.array([1.0, 0.0])
    ham = afq.Hamiltonian(inp.h, inp.L, inp.e_core)
    t1 = afq.Trial(ham, nu, nd, inp.C_up, inp.C_dn)
    t2 = afq.Trial(ham, nu, nd, inp.C_up, inp.C_dn, inp.coeff, inp.exc)
    D0 = np.concatenate([inp.C_up[:, :nu], inp.C_dn[:, :nd]], axis=1)
    re, im = syn.random_walkers(M, nu, nd, 4, seed=1, scale=0.3)
    out = []
    for t in (t1, t2):
        w = afq.Walkers(t, 4)
        _set_phi(w, D0[None] + re + 1j * im)
        afq.local_energy(ham, t, w)
        out.append(_np(w.eloc[0]) + 1j * _np(w.eloc[1]))
    assert np.allclose(out[0], out[1], rtol=1e-11)


def test_propagate_large_m_unfused_chain_fp64(afq):
    """M=100, 20/20 electrons (the fused small-M propagation does not fit in
    LDS here, so the walker-batched GEMM chain runs): mixed-energy parity."""
    _say("propagate M=100 unfused chain fp64")
    inp = syn.make_system(100, 20, 20, 40, 20.0, seed=9)
    inp.L = 0.3 * inp.L
    em, oe, w, st = _run_both(afq, inp, 4, 4, 0.005, dict(taylor_order=6, ortho_every=2, pc_every=0))
    fin = np.isfinite(oe)
    print("large M: E_mix", oe, "alive", int(np.sum(st.weight > 0)))
    assert np.array_equal(fin, np.isfinite(em)) and fin[0]
    assert np.max(np.abs(em - oe)[fin]) <= 1e-10 * np.max(np.abs(oe[fin]))


@pytest.mark.parametrize("prec,rtol", [(("fp64", "fp64"), 1e-12), (("fp32", "fp32"), 1e-7)])
def test_propagate_unfused_chain_ragged_walkers(afq, prec, rtol):
    """The walker-batched GEMM chain on a ragged shape: M=100 (the last 64-row
    block holds 36 rows), 21/18 electrons (39 columns), 11 walkers (the
    blocks of eight consecutive walkers are interleaved across the XCDs, and
    the last group of eight is partly empty): E_mix over four steps against
    the oracle, relative bound 1e-12 in FP64 and 1e-7 (the FP32 unit
    roundoff) with FP32 contractions and Taylor products."""
    _say(f"propagate M=100 21/18 W=11 unfused chain {prec}")
    inp = syn.make_system(100, 21, 18, 30, 20.0, seed=19)
    inp.L = 0.3 * inp.L
    em, oe, w, st = _run_both(afq, inp, 11, 4, 0.005,
                              dict(taylor_order=6, ortho_every=2, pc_every=0), prec=prec)
    fin = np.isfinite(oe)
    err = np.max(np.abs(em - oe)[fin]) / np.max(np.abs(oe[fin]))
    print(f"ragged chain {prec}: E_mix {oe}, max rel dE_mix {err:.3e}")
    assert np.array_equal(fin, np.isfinite(em)) and fin[0]
    assert err <= rtol


@pytest.mark.parametrize("prec,n_pin,tol", [(("fp64", "fp64"), 150, 1e-8),
                                            (("fp32", "fp32"), 100, 1e-4)])
def test_hchain_subset_1000_steps(afq, prec, n_pin, tol):
    """All 1000 steps of the hydrogen-chain workload, with its comb every 20
    steps, on a population of 64 walkers vs the stored FP64 oracle run.
    The trajectories are chaotic: in FP64 the GPU and the oracle agree to
    1e-12 Ha for about 170 steps, after which a walker near a node amplifies
    the rounding difference by orders of magnitude within a few steps and
    the populations part at the next combs.  So E_mix is held to the bound
    over the first n_pin steps (FP64 1e-8 Ha over 7 combs and 15
    orthonormalisations; FP32 the 0.1 mHa gate over 100 steps), the whole
    run must stay finite, and the step where the two runs part is printed."""
    _say(f"hchain 64 walkers, 1000 steps with comb {prec}")
    et, num, den, wk = _golden_hchain("hchain-M50_W64_T1000.txt")
    em, w = _gpu_hchain(afq, 64, 1000, et, prec, pc=True)
    ref = num / den
    err = np.abs(em - ref)
    part = np.nonzero(err > 1e-6)[0]
    print(f"{prec}: max |dE_mix| over the first {n_pin} steps = {err[:n_pin].max():.3e} Ha;"
          f" runs part (|dE_mix| > 1e-6 Ha) at step {int(part[0]) if part.size else None}")
    assert np.all(np.isfinite(ref)) and np.all(np.isfinite(em))
    assert err[:n_pin].max() <= tol


# --------------------------------------------------------------------------
# Hybrid weight form (Sec. IV.A): E_L measured every meas_every steps
# --------------------------------------------------------------------------

def _run_both_hybrid(afq, inp, W, n_steps, dt, opt_kw, prec=("fp64", "fp64"), seed=0):
    ham, trial, w = _make(afq, inp, W)
    afq.walkers_from_trial(ham, trial, w)
    et = afq.local_energy(ham, trial, w)
    opt = afq.Options(e_trial=et, chol_prec=prec[0], taylor_prec=prec[1], weight_mode="hybrid",
                      **opt_kw)
    em = _np(afq.propagate(ham, trial, w, n_steps, dt, seed, 0, opt))
    o = Oracle.from_inputs(inp)
    st = o.init_walkers(W)
    oe = o.propagate(st, n_steps, dt, seed, 0, OOptions(e_trial=et, weight_mode=1, **opt_kw))
    return em, oe, w, st


def test_hybrid_plain_fp64_parity(afq):
    """10-orbital workload, 64 walkers, 40 steps, E_L every 5 steps, comb every
    10: E_mix at the measured steps and the final weights within 1e-9 of the
    oracle; the other steps report NaN on both sides."""
    _say("hybrid plain-M10 fp64 40 steps")
    wl = syn.WORKLOADS["plain-M10"]
    inp = syn.workload_system(wl)
    em, oe, w, st = _run_both_hybrid(afq, inp, 64, 40, wl.dt,
                                     dict(taylor_order=6, ortho_every=2, pc_every=10, meas_every=5))
    meas = np.arange(40) % 5 == 4
    assert np.all(np.isnan(em[~meas])) and np.all(np.isnan(oe[~meas]))
    print("hybrid fp64: max |dE_mix| =", np.max(np.abs(em[meas] - oe[meas])))
    assert np.max(np.abs(em[meas] - oe[meas])) <= 1e-9
    assert np.allclose(_np(w.weight), st.weight, rtol=1e-9, atol=1e-12)


def test_hybrid_hchain_fp32(afq):
    """Hydrogen-chain workload, 32 walkers, 40 steps, FP32 contractions and
    Taylor, E_L every 10 steps: E_mix at the measured steps within the
    0.1 mHa gate of the FP64 oracle."""
    _say("hybrid hchain fp32 32 walkers 40 steps")
    wl = syn.WORKLOADS["hchain-M50"]
    inp = syn.workload_system(wl)
    em, oe, w, st = _run_both_hybrid(afq, inp, 32, 40, wl.dt,
                                     dict(taylor_order=6, ortho_every=10, pc_every=0, meas_every=10),
                                     prec=("fp32", "fp32"))
    meas = np.arange(40) % 10 == 9
    err = np.max(np.abs(em[meas] - oe[meas]))
    print("hybrid fp32 hchain: max |dE_mix| =", err, "E_mix", oe[meas])
    assert np.all(np.isfinite(oe[meas]))
    assert err <= 1e-4


def test_hybrid_multidet_fp64_parity(afq):
    """Multi-determinant trial in the hybrid form (every step measured on the
    GPU's multi-determinant route, weights from the importance function)."""
    _say("hybrid multidet fp64")
    M, nu, nd, G = 10, 3, 2, 12
    inp = syn.make_system(M, nu, nd, G, 8.0, n_det=12, seed=41)
    em, oe, w, st = _run_both_hybrid(afq, inp, 16, 12, 0.01,
                                     dict(taylor_order=6, ortho_every=2, pc_every=0, meas_every=4))
    meas = np.arange(12) % 4 == 3
    print("hybrid multidet: max |dE_mix| =", np.max(np.abs(em[meas] - oe[meas])))
    assert np.max(np.abs(em[meas] - oe[meas])) <= 1e-9
    assert np.allclose(_np(w.weight), st.weight, rtol=1e-9, atol=1e-12)


def test_hybrid_zero_variance_one_body(afq):
    """L = 0, eigenvector trial: measured E_mix exact, hybrid weights equal
    the local-energy form's."""
    _say("hybrid zero variance one-body")
    M, nu, nd = 9, 3, 2
    inp = syn.make_system(M, nu, nd, 4, 4.0, seed=5, e_core=1.25)
    inp.L = np.zeros_like(inp.L)
    eps = np.linalg.eigvalsh(inp.h)
    exact = inp.e_core + eps[:nu].sum() + eps[:nd].sum()
    res = []
    for mode in ("local", "hybrid"):
        ham, trial, w = _make(afq, inp, 8)
        afq.walkers_from_trial(ham, trial, w)
        opt = afq.Options(e_trial=exact + 0.5, ortho_every=2, weight_mode=mode, meas_every=3)
        em = _np(afq.propagate(ham, trial, w, 9, 0.02, 1, 0, opt))
        res.append((em, _np(w.weight)))
    assert np.allclose(res[1][0][2::3], exact, atol=1e-12)
    assert np.allclose(res[0][1], res[1][1], rtol=1e-12)


def test_exchange_route_selection(afq):
    """The Q route is built for single-determinant trials with n_chol >= 2 M
    and can be switched off and on; asking for it where it was not built is
    an error and leaves the route unchanged."""
    _say("exchange route selection")
    inp = syn.make_system(10, 5, 5, 40, 8.0, seed=50, e_core=0.75)
    ham, trial, w = _make(afq, inp, 2)
    assert trial.exchange_route == "q"
    trial.exchange_route = "ltilde"
    assert trial.exchange_route == "ltilde"
    trial.exchange_route = "q"
    assert trial.exchange_route == "q"
    inp2 = syn.make_system(23, 7, 4, 37, 8.0, seed=60, e_core=0.75)
    ham2, trial2, w2 = _make(afq, inp2, 2)
    assert trial2.exchange_route == "ltilde"
    with pytest.raises(afq.AfqmcError):
        trial2.exchange_route = "q"
    assert trial2.exchange_route == "ltilde"
    with pytest.raises(ValueError):
        trial2.exchange_route = "other"
