"""afqmc_reconfigure_noalloc (scratch in a static device array) against
afqmc_reconfigure (scratch in the walker workspace), through the C ABI: two
calls in a row, the second with a smaller input; the orbitals, weights,
overlaps, local energies and the norm factor bitwise equal (the first call's
orbitals exceed the array, so its snapshot is taken in column ranges), and one
further propagation step of both populations gives the same E_mix."""
import ctypes
import sys

import numpy as np
import pytest

import afqmc_synth as syn

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _population(afq, inp, W, seed):
    ham = afq.Hamiltonian(inp.h, inp.L, inp.e_core)
    trial = afq.Trial(ham, inp.n_up, inp.n_dn, inp.C_up, inp.C_dn)
    re, im = syn.random_walkers(inp.h.shape[0], inp.n_up, inp.n_dn, W, seed=seed, scale=0.3)
    D0 = np.concatenate([inp.C_up[:, :inp.n_up], inp.C_dn[:, :inp.n_dn]], axis=1)
    rng = np.random.default_rng(seed)
    wts = rng.exponential(size=W)
    wts[rng.random(W) < 0.3] = 0.0
    wts[0] = 1.0
    pops = []
    for _ in range(2):
        w = afq.Walkers(trial, W)
        w.phi_re.copy_(torch.from_numpy(np.ascontiguousarray(D0[None] + re)))
        w.phi_im.copy_(torch.from_numpy(np.ascontiguousarray(im)))
        w.weight.copy_(torch.from_numpy(wts))
        afq.local_energy(ham, trial, w)
        pops.append(w)
    return ham, trial, pops


def _state(w):
    torch.cuda.synchronize()
    return [t.detach().cpu().numpy().copy()
            for t in (w.phi_re, w.phi_im, w.weight, w.logovlp[0], w.logovlp[1], w.eloc[0], w.eloc[1])]


@pytest.mark.parametrize("calls", [[(50, 25, 25, 12, 2048), (20, 5, 4, 30, 300)]])
def test_noalloc_comb_matches_workspace_comb(calls):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_03310_amd as afq
    from paper_1804_03310_amd import _abi
    lib = _abi.load()
    for k, (M, nu, nd, G, W) in enumerate(calls):
        _say(f"reconfigure_noalloc call {k}: M={M} N={nu}/{nd} G={G} W={W} "
             f"(row {M * (nu + nd)} doubles, W*row {W * M * (nu + nd)})")
        inp = syn.make_system(M, nu, nd, G, 8.0, seed=40 + k)
        ham, trial, (wa, wb) = _population(afq, inp, W, seed=7 + k)
        na, nb = ctypes.c_double(), ctypes.c_double()
        stream = torch.cuda.current_stream().cuda_stream
        _abi.check(lib.afqmc_reconfigure(trial._t, ctypes.byref(wa.struct), 21, 3 + k,
                                         ctypes.byref(na), stream))
        _abi.check(lib.afqmc_reconfigure_noalloc(trial._t, ctypes.byref(wb.struct), 21, 3 + k,
                                                 ctypes.byref(nb), stream))
        assert na.value == nb.value and na.value > 0
        for x, y in zip(_state(wa), _state(wb)):
            assert np.array_equal(x, y)
        assert np.array_equal(_state(wb)[2], np.ones(W))
        opt = afq.Options(taylor_order=6, e_trial=0.0, chol_prec="fp64", taylor_prec="fp64")
        ea = afq.propagate(ham, trial, wa, 1, 0.005, 5, 0, opt).cpu().numpy()
        eb = afq.propagate(ham, trial, wb, 1, 0.005, 5, 0, opt).cpu().numpy()
        assert np.array_equal(ea, eb) and np.all(np.isfinite(ea))
