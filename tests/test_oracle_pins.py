"""Pins of the FP64 oracle to things other than itself (CPU only).

Each test checks the oracle against a value the mathematics fixes
independently: a published known-answer vector, a library routine, brute
force in Fock space, a closed form, or an invariant.  A plausible slip in the
oracle (a dropped term, a wrong sign or factor of i, a transposed operand, a
wrong spin sum) fails at least one of them.
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

import afqmc_synth as syn
import fock
from oracle import (Options, Oracle, comb_parents, comb_uniform, gaussian_fields,
                    mgs_orthonormalize, modified_cholesky, philox4x64_10,
                    taylor_apply)
from oracle.afqmc import log_det

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------

def test_philox_known_answer_vector():
    """Philox4x64-10 known-answer vector (Salmon et al., SC'11)."""
    with open(os.path.join(GOLDEN, "philox4x64_10_kat.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert rows
    for r in rows:
        vals = [int(x, 16) for x in r]
        ctr, key, out = vals[0:4], vals[4:6], vals[6:10]
        got = philox4x64_10(np.array([ctr], dtype=np.uint64), np.array(key, dtype=np.uint64))
        assert [int(x) for x in got[0]] == out


def test_philox_matches_numpy_bit_generator():
    """Raw words equal numpy.random.Philox (which pre-increments its counter)."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        ctr = [int(x) for x in rng.integers(1, 2**63, size=4)]
        key = [int(x) for x in rng.integers(0, 2**63, size=2)]
        prev = list(ctr)
        prev[0] -= 1  # no borrow: ctr[0] >= 1
        ref = np.random.Philox(counter=prev, key=key).random_raw(4)
        got = philox4x64_10(np.array([ctr], dtype=np.uint64), np.array(key, dtype=np.uint64))[0]
        assert [int(x) for x in got] == [int(x) for x in ref]


def test_fields_are_standard_normal_and_counter_keyed():
    x = gaussian_fields(seed=3, t=5, walker_index=np.arange(400), n_chol=250)
    assert x.shape == (400, 250)
    ks = scipy.stats.kstest(x.ravel(), "norm")
    assert ks.pvalue > 1e-3
    assert abs(x.mean()) < 0.01 and abs(x.std() - 1) < 0.01
    # any walker can be regenerated alone (counter-based)
    y = gaussian_fields(seed=3, t=5, walker_index=[17, 301], n_chol=250)
    assert np.array_equal(y, x[[17, 301]])
    # different step / system / seed give different fields
    assert not np.allclose(gaussian_fields(3, 6, [17], 250), x[[17]])
    assert not np.allclose(gaussian_fields(3, 5, [17], 250, system_id=1), x[[17]])
    assert not np.allclose(gaussian_fields(4, 5, [17], 250), x[[17]])


# --------------------------------------------------------------------------
# Determinants, inverse, MGS, Taylor
# --------------------------------------------------------------------------

def _cofactor_det(A):
    n = A.shape[0]
    if n == 1:
        return A[0, 0]
    tot = 0
    for j in range(n):
        minor = np.delete(np.delete(A, 0, axis=0), j, axis=1)
        tot += (-1) ** j * A[0, j] * _cofactor_det(minor)
    return tot


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
def test_log_det_matches_cofactor_expansion(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((4, n, n)) + 1j * rng.standard_normal((4, n, n))
    ld = log_det(A)
    for w in range(4):
        d = _cofactor_det(A[w])
        assert abs(np.exp(ld[w]) - d) <= 1e-12 * abs(d)


def test_mgs_gives_unique_qr():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((3, 9, 4)) + 1j * rng.standard_normal((3, 9, 4))
    q = mgs_orthonormalize(a)
    for w in range(3):
        assert np.allclose(q[w].conj().T @ q[w], np.eye(4), atol=1e-13)
        R = q[w].conj().T @ a[w]
        assert np.allclose(np.tril(R, -1), 0, atol=1e-12)
        assert np.all(np.abs(np.diag(R).imag) < 1e-12) and np.all(np.diag(R).real > 0)
        # uniqueness: agrees with LAPACK QR after fixing the diagonal phase
        Q2, R2 = np.linalg.qr(a[w])
        ph = np.diag(R2) / np.abs(np.diag(R2))
        assert np.allclose(Q2 * ph[None, :], q[w], atol=1e-12)


def test_taylor_within_remainder_bound():
    rng = np.random.default_rng(2)
    for scale in (0.05, 0.4, 1.5):
        A = scale * (rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))) / 6
        phi = rng.standard_normal((6, 3)) + 1j * rng.standard_normal((6, 3))
        exact = scipy.linalg.expm(A) @ phi
        for order in (2, 6, 12):
            got = taylor_apply(A[None], phi[None], order)[0]
            a = np.linalg.norm(A, 2)
            bound = a ** (order + 1) / math.factorial(order + 1) * math.exp(a) * np.linalg.norm(phi, 2)
            assert np.linalg.norm(got - exact, 2) <= bound * (1 + 1e-9) + 1e-13
        assert np.allclose(taylor_apply(A[None], phi[None], 40)[0], exact, atol=1e-13)


# --------------------------------------------------------------------------
# Local energy, overlap, force bias against brute force
# --------------------------------------------------------------------------

def _small_system(M, n_up, n_dn, n_chol, seed, tau_d=4.0):
    inp = syn.make_system(M, n_up, n_dn, n_chol, tau_d, seed=seed, e_core=0.37)
    return inp


def _hf_energy(h, L, e_core, occ):
    """Hartree-Fock energy of the determinant with occupied orbitals occ[spin]
    from the 4-index V of Eq. 1 (Coulomb between all pairs, exchange within a
    spin)."""
    V = fock.eri_from_chol(L)
    E = e_core
    for s in range(2):
        E += np.trace(occ[s].T @ h @ occ[s])
    for s in range(2):
        for t in range(2):
            Vmo = np.einsum("ia,jb,kc,ld,ijkl->abcd", occ[s], occ[t], occ[s], occ[t], V)
            n1, n2 = occ[s].shape[1], occ[t].shape[1]
            for a in range(n1):
                for b in range(n2):
                    E += 0.5 * Vmo[a, b, a, b]
                    if s == t:
                        E -= 0.5 * Vmo[a, b, b, a]
    return E


@pytest.mark.parametrize("M,n_up,n_dn", [(6, 3, 3), (7, 3, 2), (5, 2, 0)])
def test_local_energy_at_trial_is_hartree_fock(M, n_up, n_dn):
    """E_L(phi = D_0) equals the HF energy written from the 4-index V (Eq. 1)."""
    inp = _small_system(M, n_up, n_dn, 9, seed=M + n_up)
    # an unrestricted trial: different orbitals per spin
    rng = np.random.default_rng(5)
    Cdn = np.linalg.qr(rng.standard_normal((M, M)))[0]
    o = Oracle(inp.h, inp.L, inp.e_core, inp.C_up, Cdn, n_up, n_dn)
    st = o.init_walkers(2)
    E = _hf_energy(inp.h, inp.L, inp.e_core, [inp.C_up[:, :n_up], Cdn[:, :n_dn]])
    assert np.allclose(st.eloc, E, rtol=0, atol=1e-11)
    assert np.allclose(st.logS, 0.0, atol=1e-12)
    # force-bias input at the trial is lbar
    assert np.allclose(st.v, o.lbar[None, :], atol=1e-12)


def _fci_check(o, inp, M, n_up, n_dn, phi, ctrial):
    V = fock.eri_from_chol(inp.L)
    H, states, index = fock.hamiltonian_matrix(inp.h, V, inp.e_core, M, n_up, n_dn)
    m = o.measure(phi)
    for w in range(phi.shape[0]):
        cphi = fock.det_amplitudes(phi[w, :, :n_up], phi[w, :, n_up:], M, states)
        ov = ctrial.conj() @ cphi
        eloc = (ctrial.conj() @ H @ cphi) / ov
        assert abs(np.exp(m["logS"][w]) - ov) <= 1e-11 * abs(ov)
        assert abs(m["eloc"][w] - eloc) <= 1e-10 * max(1.0, abs(eloc))
        # force-bias input v_gamma = <Psi_T| Lhat_gamma |phi> / <Psi_T|phi>
        for g in range(inp.n_chol):
            Lg = fock.one_body_matrix(inp.L[g], M, states, index)
            vg = (ctrial.conj() @ Lg @ cphi) / ov
            assert abs(m["v"][w, g] - vg) <= 1e-10 * max(1.0, abs(vg))


@pytest.mark.parametrize("M,n_up,n_dn", [(4, 2, 2), (5, 2, 1)])
def test_local_energy_single_det_matches_fock_space(M, n_up, n_dn):
    inp = _small_system(M, n_up, n_dn, 5, seed=11 + M)
    o = Oracle.from_inputs(inp)
    re, im = syn.random_walkers(M, n_up, n_dn, 3, seed=4)
    phi = re + 1j * im
    states, _ = fock.basis(M, n_up, n_dn)
    ctrial = fock.det_amplitudes(inp.C_up[:, :n_up], inp.C_dn[:, :n_dn], M, states)
    _fci_check(o, inp, M, n_up, n_dn, phi, ctrial)


def test_local_energy_multi_det_matches_fock_space():
    M, n_up, n_dn = 5, 2, 2
    inp = syn.make_system(M, n_up, n_dn, 4, 3.0, n_det=12, seed=21, e_core=-0.5)
    o = Oracle.from_inputs(inp)
    states, _ = fock.basis(M, n_up, n_dn)
    ctrial = np.zeros(len(states))
    for i in range(inp.n_det):
        Du, Dd = o.D[i]
        ctrial += inp.coeff[i] * fock.det_amplitudes(Du, Dd, M, states)
    re, im = syn.random_walkers(M, n_up, n_dn, 3, seed=8)
    _fci_check(o, inp, M, n_up, n_dn, re + 1j * im, ctrial)


def test_two_body_energy_matches_paper_Y_tensor_route():
    """Eq. Ys: same-spin E2 = 1/2 sum_ijab Y_ijab Theta_ia Theta_jb; plus the
    opposite-spin Coulomb term; compared with the oracle's E_L - E_1 - e_core."""
    M, n_up, n_dn = 6, 3, 2
    inp = _small_system(M, n_up, n_dn, 7, seed=31)
    o = Oracle.from_inputs(inp)
    re, im = syn.random_walkers(M, n_up, n_dn, 2, seed=9)
    phi = re + 1j * im
    m = o.measure(phi)
    for w in range(2):
        thetas, e1, trs = [], 0.0, []
        E2 = 0.0
        for s, (n, C) in enumerate(((n_up, inp.C_up), (n_dn, inp.C_dn))):
            psi = C[:, :n]
            ph = phi[w][:, :n_up] if s == 0 else phi[w][:, n_up:]
            theta = ph @ np.linalg.inv(psi.T @ ph)
            e1 += np.trace(inp.h @ theta @ psi.T)
            # Y_ijab = sum_kl sum_alpha L_ik L_jl [psi_ka psi_lb - psi_la psi_kb]
            Y = (np.einsum("gik,gjl,ka,lb->ijab", inp.L, inp.L, psi, psi)
                 - np.einsum("gik,gjl,la,kb->ijab", inp.L, inp.L, psi, psi))
            E2 += 0.5 * np.einsum("ijab,ia,jb->", Y, theta, theta)
            trs.append(np.einsum("gik,ki->g", inp.L, theta @ psi.T))
        E2 += np.sum(trs[0] * trs[1])
        assert abs(m["eloc"][w] - (inp.e_core + e1 + E2)) < 1e-10 * abs(m["eloc"][w])


# --------------------------------------------------------------------------
# Cholesky input
# --------------------------------------------------------------------------

def _model_eri(M, seed):
    """A PSD two-electron tensor from orbitals on a 1-D grid with the
    positive-definite kernel 1/sqrt((r-r')^2 + 1)."""
    rng = np.random.default_rng(seed)
    r = np.linspace(-4, 4, 60)
    orb = np.linalg.qr(rng.standard_normal((60, M)))[0]
    kern = 1.0 / np.sqrt((r[:, None] - r[None, :]) ** 2 + 1.0)
    dens = np.einsum("ri,rk->rik", orb, orb)
    # V_ijkl = sum_{r r'} phi_i(r) phi_k(r) v(r,r') phi_j(r') phi_l(r')
    return np.einsum("rik,rs,sjl->ijkl", dens, kern, dens)


@pytest.mark.parametrize("delta", [1e-4, 1e-6])
def test_cholesky_reconstructs_eri_within_threshold(delta):
    M = 6
    V = _model_eri(M, seed=3)
    L = modified_cholesky(V, delta)
    assert 0 < L.shape[0] < M * M
    err = np.max(np.abs(fock.eri_from_chol(L) - V))
    assert err <= delta
    # the decomposed vectors are symmetric like the pairs they come from
    assert np.allclose(L, L.transpose(0, 2, 1), atol=1e-12)
    # HF energy from the vectors vs from V: error bounded by the threshold
    h = -np.eye(M) + 0.05 * np.ones((M, M))
    C = syn.make_trial_orbitals(h)
    o = Oracle(h, L, 0.0, C, C, 2, 2)
    e_chol = o.init_walkers(1).eloc[0].real
    occ = C[:, :2]
    Vmo = np.einsum("ia,jb,kc,ld,ijkl->abcd", occ, occ, occ, occ, V)
    e_ref = 2 * np.trace(occ.T @ h @ occ)
    for a in range(2):
        for b in range(2):
            e_ref += 0.5 * 4 * Vmo[a, b, a, b] - 0.5 * 2 * Vmo[a, b, b, a]
    assert abs(e_chol - e_ref) <= 16 * 4 * delta


# --------------------------------------------------------------------------
# Hubbard-Stratonovich sign / factor i, and Thouless' theorem
# --------------------------------------------------------------------------

def test_hubbard_stratonovich_integral_reproduces_two_body_factor():
    """Eq. 2 with v = i(Lhat - lbar): the Gaussian average over x of the
    oracle's one-field propagator exp(i sqrt(dt) x (L - lbar)) acting on a
    determinant equals exp(-dt/2 (Lhat - lbar)^2) in Fock space."""
    M, n_up, n_dn = 4, 2, 1
    inp = _small_system(M, n_up, n_dn, 1, seed=41)
    o = Oracle.from_inputs(inp)
    lbar = o.lbar[0]
    states, index = fock.basis(M, n_up, n_dn)
    Lhat = fock.one_body_matrix(inp.L[0], M, states, index)
    dt = 0.3
    target_op = scipy.linalg.expm(-0.5 * dt * (Lhat - lbar * np.eye(len(states))) @
                                  (Lhat - lbar * np.eye(len(states))))
    re, im = syn.random_walkers(M, n_up, n_dn, 1, seed=2)
    phi = re[0] + 1j * im[0]
    c0 = fock.det_amplitudes(phi[:, :n_up], phi[:, n_up:], M, states)
    target = target_op @ c0
    xs, ws = np.polynomial.hermite_e.hermegauss(80)
    ws = ws / np.sqrt(2 * np.pi)
    acc = np.zeros(len(states), dtype=complex)
    for x, wgt in zip(xs, ws):
        A = o.propagator_matrix(np.array([[x]]), dt)[0]
        p = taylor_apply(A[None], phi[None], 60)[0]
        scal = np.exp(-1j * np.sqrt(dt) * x * lbar)
        acc += wgt * scal * fock.det_amplitudes(p[:, :n_up], p[:, n_up:], M, states)
    assert np.allclose(acc, target, atol=1e-11)


def test_thouless_one_body_exponential():
    M, n_up, n_dn = 4, 2, 2
    rng = np.random.default_rng(3)
    A = 0.3 * (rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M)))
    states, index = fock.basis(M, n_up, n_dn)
    Ahat = fock.one_body_matrix(A, M, states, index)
    phi = rng.standard_normal((M, n_up + n_dn)) + 1j * rng.standard_normal((M, n_up + n_dn))
    c0 = fock.det_amplitudes(phi[:, :n_up], phi[:, n_up:], M, states)
    p = taylor_apply(A[None], phi[None], 50)[0]
    c1 = fock.det_amplitudes(p[:, :n_up], p[:, n_up:], M, states)
    assert np.allclose(c1, scipy.linalg.expm(Ahat) @ c0, atol=1e-12)


# --------------------------------------------------------------------------
# Zero-variance special cases of the whole step
# --------------------------------------------------------------------------

def test_zero_variance_one_body_only():
    """L = 0 and the trial made of eigenvectors of h: E_L = sum of occupied
    eigenvalues for every walker at every step (ortho and comb on)."""
    M, n_up, n_dn = 8, 3, 2
    inp = syn.make_system(M, n_up, n_dn, 6, 4.0, seed=5, e_core=1.25)
    L0 = np.zeros_like(inp.L)
    o = Oracle(inp.h, L0, inp.e_core, inp.C_up, inp.C_dn, n_up, n_dn)
    eps = np.linalg.eigvalsh(inp.h)
    exact = inp.e_core + eps[:n_up].sum() + eps[:n_dn].sum()
    st = o.init_walkers(16)
    opt = Options(ortho_every=2, pc_every=5, e_trial=exact)
    emix = o.propagate(st, 12, 0.01, seed=1, step0=0, opt=opt)
    assert np.allclose(emix, exact, atol=1e-12)
    assert np.allclose(st.eloc, exact, atol=1e-12)


def test_zero_variance_exact_fci_trial_whole_step():
    """With the exact ground state as a multi-determinant trial, every
    walker's E_L equals E_FCI at every step of a real random-field run."""
    M, n_up, n_dn = 4, 2, 2
    inp = syn.make_system(M, n_up, n_dn, 5, 3.0, seed=13, e_core=0.2)
    rng = np.random.default_rng(17)
    C = np.linalg.qr(rng.standard_normal((M, M)))[0]   # rotated orbital basis
    exc, coeff, efci = fock.fci_trial(inp.h, inp.L, inp.e_core, C, n_up, n_dn)
    assert coeff.size > 10
    o = Oracle(inp.h, inp.L, inp.e_core, C, C, n_up, n_dn, coeff, exc)
    st = o.init_walkers(6)
    assert np.allclose(st.eloc, efci, atol=1e-10)
    opt = Options(ortho_every=2, pc_every=3, e_trial=efci)
    for t in range(8):
        em = o.step(st, t, seed=2, dt=0.02, opt=opt)
        assert abs(em - efci) < 1e-10
        assert np.allclose(st.eloc[st.weight > 0], efci, atol=1e-9)
        if (t + 1) % 2 == 0:
            o.orthonormalize(st)
        if (t + 1) % 3 == 0:
            o.reconfigure(st, 2, t)
    assert np.any(st.weight > 0)


# --------------------------------------------------------------------------
# Whole-step invariants
# --------------------------------------------------------------------------

def test_orthonormalization_leaves_estimates_unchanged():
    inp = _small_system(7, 3, 2, 6, seed=51)
    o = Oracle.from_inputs(inp)
    re, im = syn.random_walkers(7, 3, 2, 4, seed=1)
    st = o.init_walkers(4, phi=re + 1j * im)
    e0, v0 = st.eloc.copy(), st.v.copy()
    o.orthonormalize(st)
    m = o.measure(st.phi)
    assert np.allclose(m["eloc"], e0, rtol=1e-12)
    assert np.allclose(m["v"], v0, rtol=1e-11, atol=1e-12)
    for w in range(4):
        for a, b in ((0, 3), (3, 5)):
            blk = st.phi[w][:, a:b]
            assert np.allclose(blk.conj().T @ blk, np.eye(b - a), atol=1e-13)


def test_mixed_energy_invariant_under_trial_energy_shift():
    w = syn.WORKLOADS["plain-M10"]
    inp = syn.workload_system(w)
    o = Oracle.from_inputs(inp)
    out = []
    for et in (0.0, 3.0):
        st = o.init_walkers(16)
        opt = Options(ortho_every=2, pc_every=4, e_trial=et)
        out.append(o.propagate(st, 10, w.dt, seed=0, step0=0, opt=opt))
    assert np.allclose(out[0], out[1], rtol=1e-12, atol=0)


def test_comb_matches_brute_force_and_bounds():
    rng = np.random.default_rng(4)
    for K in (1, 7, 64, 301):
        w = rng.exponential(size=K)
        w[rng.random(K) < 0.2] = 0.0
        if not np.any(w > 0):
            w[0] = 1.0
        xi = comb_uniform(9, K)
        parents, norm = comb_parents(w, xi)
        tot = math.fsum(w)
        assert abs(norm - tot / K) < 1e-12 * tot
        counts = np.bincount(parents, minlength=K)
        assert counts.sum() == K
        assert np.all(counts[w == 0] == 0)
        exp_ = K * w / tot
        assert np.all(counts >= np.floor(exp_ - 1e-9)) and np.all(counts <= np.ceil(exp_ + 1e-9))
        # brute force: tooth j lands in the interval [C_{k-1}, C_k)
        C = np.cumsum(w)
        for j in range(K):
            z = (j + xi) * C[-1] / K
            k = [i for i in range(K) if (C[i - 1] if i else 0.0) <= z < C[i]]
            if k:
                assert parents[j] == k[0]
        assert np.all(np.diff(parents) >= 0)


def test_dead_walker_reset_to_reference_state():
    """Sec. II phaseless constraint: a walker whose weight becomes zero or
    non-finite dies.  It is reset to the reference determinant with weight 0,
    so its overlap is 1 (log S = 0), its E_L the Hartree-Fock energy of D_0
    from the 4-index V and its force-bias input v_g = sum_sigma Tr(D_0^T L_g
    D_0); it drops out of E_mix, the comb never picks it, and the other
    walkers are untouched."""
    M, n_up, n_dn = 6, 3, 2
    inp = _small_system(M, n_up, n_dn, 9, seed=21)
    o = Oracle.from_inputs(inp)
    opt = Options(taylor_order=6, e_trial=0.0)
    st = o.init_walkers(5)
    o.step(st, 0, 3, 0.01, opt)
    ref = st.copy()
    st.weight[1] = 0.0
    st.weight[3] = np.nan
    o.step(st, 1, 3, 0.01, opt)
    o.step(ref, 1, 3, 0.01, opt)
    dead, live = [1, 3], [0, 2, 4]
    occ = [inp.C_up[:, :n_up], inp.C_dn[:, :n_dn]]
    d0 = np.concatenate(occ, axis=1)
    vbar = np.array([sum(np.trace(c.T @ Lg @ c) for c in occ) for Lg in inp.L])
    e_hf = _hf_energy(inp.h, inp.L, inp.e_core, occ)
    for k in dead:
        assert st.weight[k] == 0.0
        assert np.array_equal(st.phi[k], d0.astype(complex))
        assert abs(st.logS[k]) < 1e-12
        assert abs(st.eloc[k] - e_hf) < 1e-11
        assert np.allclose(st.v[k], vbar, rtol=0, atol=1e-12)
    for k in live:
        assert st.weight[k] == ref.weight[k] and st.weight[k] > 0
        assert np.array_equal(st.phi[k], ref.phi[k])
        assert st.eloc[k] == ref.eloc[k]
    wl = st.weight[live]
    emix = math.fsum(wl * st.eloc[live].real) / math.fsum(wl)
    assert abs(Oracle.mixed_energy(st) - emix) < 1e-12 * abs(emix)
    for pc in range(20):
        parents, _ = comb_parents(st.weight, comb_uniform(3, pc))
        assert not set(parents.tolist()) & set(dead)


def test_comb_with_no_live_walker_leaves_population():
    """A comb over an all-dead population has no teeth to place (W_tot = 0):
    the population is left as it is and the norm factor is 0."""
    inp = _small_system(5, 2, 2, 6, seed=2)
    o = Oracle.from_inputs(inp)
    st = o.init_walkers(4)
    o.step(st, 0, 1, 0.01, Options(e_trial=0.0))
    st.weight[:] = 0.0
    before = st.copy()
    assert o.reconfigure(st, 1, 0) == 0.0
    assert np.array_equal(st.weight, before.weight)
    assert np.array_equal(st.phi, before.phi)


def test_comb_uniform_in_unit_interval():
    xs = [comb_uniform(s, p) for s in range(5) for p in range(50)]
    assert all(0.0 < x < 1.0 for x in xs)
    assert scipy.stats.kstest(xs, "uniform").pvalue > 1e-3


# --------------------------------------------------------------------------
# One-body split and weight update against Fock space
# --------------------------------------------------------------------------

def test_trotter_split_is_second_order_in_dt():
    """Gaussian average of the oracle's one-step propagator (B1, one field,
    mean-field phase) equals exp(dt (e_core - lbar^2/2)) exp(-dt H) up to
    O(dt^3): a wrong one-body term H1' would leave an O(dt^2) error."""
    M, n_up, n_dn = 4, 2, 1
    inp = _small_system(M, n_up, n_dn, 1, seed=61)
    o = Oracle.from_inputs(inp)
    lbar = o.lbar[0]
    V = fock.eri_from_chol(inp.L)
    H, states, _ = fock.hamiltonian_matrix(inp.h, V, inp.e_core, M, n_up, n_dn)
    re, im = syn.random_walkers(M, n_up, n_dn, 1, seed=3)
    phi = re[0] + 1j * im[0]
    c0 = fock.det_amplitudes(phi[:, :n_up], phi[:, n_up:], M, states)
    xs, ws = np.polynomial.hermite_e.hermegauss(60)
    ws = ws / np.sqrt(2 * np.pi)
    errs = []
    for dt in (0.2, 0.1, 0.05):
        acc = np.zeros(len(states), dtype=complex)
        for x, wgt in zip(xs, ws):
            p, mf = o.apply_propagator(phi[None], np.array([[x]]), dt, 60)
            acc += wgt * np.exp(mf[0]) * fock.det_amplitudes(p[0][:, :n_up], p[0][:, n_up:], M, states)
        ref = np.exp(dt * (inp.e_core - 0.5 * lbar ** 2)) * (scipy.linalg.expm(-dt * H) @ c0)
        errs.append(np.linalg.norm(acc - ref) / np.linalg.norm(ref))
    assert errs[0] / errs[1] > 6.0 and errs[1] / errs[2] > 6.5
    assert errs[2] < 1e-4


def test_hybrid_importance_function_average_matches_fock_space():
    """Hybrid weights (Sec. IV.A): the Gaussian average over x of the
    oracle's importance function I(x) for a walker away from the trial (so
    that the force bias is complex) equals <Psi_T|B1 e^{-dt/2 (L - lbar)^2}
    B1|phi>/<Psi_T|phi> from Fock space; restoring e^{-dt E_0} gives
    <Psi_T|e^{-dt H}|phi>/<Psi_T|phi> up to the O(dt^3) split error.  A wrong
    sign of x xbar or xbar^2/2, a dropped mean-field phase or a wrong E_0 fails."""
    M, n_up, n_dn = 4, 2, 1
    inp = _small_system(M, n_up, n_dn, 1, seed=91)
    o = Oracle.from_inputs(inp)
    V = fock.eri_from_chol(inp.L)
    H, states, index = fock.hamiltonian_matrix(inp.h, V, inp.e_core, M, n_up, n_dn)
    Lop = fock.one_body_matrix(inp.L[0], M, states, index)
    H1f = fock.one_body_matrix(o.H1p, M, states, index)
    dt = 0.01
    re, im = syn.random_walkers(M, n_up, n_dn, 1, seed=4, scale=0.4)
    D0 = np.concatenate([inp.C_up[:, :n_up], inp.C_dn[:, :n_dn]], axis=1)
    st = o.init_walkers(1, phi=D0[None] + re + 1j * im)
    assert abs((st.v[0, 0] - o.lbar[0]).imag) > 1e-3   # complex force bias
    cT = fock.det_amplitudes(inp.C_up[:, :n_up], inp.C_dn[:, :n_dn], M, states)
    c0 = fock.det_amplitudes(st.phi[0][:, :n_up], st.phi[0][:, n_up:], M, states)
    ovl0 = cT @ c0
    xs, ws = np.polynomial.hermite_e.hermegauss(80)
    ws = ws / np.sqrt(2 * np.pi)
    avg = 0.0
    for x, wgt in zip(xs, ws):
        _, _, _, logI = o.shifted_step(st, np.array([[x]]), dt, 40)
        avg += wgt * np.exp(logI[0])
    B1f = scipy.linalg.expm(-0.5 * dt * H1f)
    K = Lop - o.lbar[0] * np.eye(len(states))
    split = cT @ (B1f @ scipy.linalg.expm(-0.5 * dt * (K @ K)) @ B1f @ c0) / ovl0
    assert abs(avg - split) < 1e-10 * abs(split)
    full = cT @ (scipy.linalg.expm(-dt * H) @ c0) / ovl0
    assert abs(avg * np.exp(-dt * o.e0_shift) - full) < 1e-6 * abs(full)


def test_hybrid_weights_zero_variance_one_body():
    """L = 0 and a trial of eigenvectors of h: the hybrid importance function
    is exp(-dt E_1body) exactly, so hybrid and local-energy weights coincide
    and the measured E_mix is exact."""
    M, n_up, n_dn = 8, 3, 2
    inp = syn.make_system(M, n_up, n_dn, 6, 4.0, seed=5, e_core=1.25)
    L0 = np.zeros_like(inp.L)
    o = Oracle(inp.h, L0, inp.e_core, inp.C_up, inp.C_dn, n_up, n_dn)
    eps = np.linalg.eigvalsh(inp.h)
    exact = inp.e_core + eps[:n_up].sum() + eps[:n_dn].sum()
    re, im = syn.random_walkers(M, n_up, n_dn, 8, seed=2, scale=0.3)
    D0 = np.concatenate([inp.C_up[:, :n_up], inp.C_dn[:, :n_dn]], axis=1)
    sa = o.init_walkers(8, phi=D0[None] + re + 1j * im)
    sb = sa.copy()
    et = exact + 0.7
    ea = o.propagate(sa, 9, 0.02, seed=1, step0=0, opt=Options(ortho_every=2, e_trial=et))
    eb = o.propagate(sb, 9, 0.02, seed=1, step0=0,
                     opt=Options(ortho_every=2, e_trial=et, weight_mode=1, meas_every=3))
    assert np.allclose(sa.weight, sb.weight, rtol=1e-12)
    assert np.allclose(eb[2::3], ea[2::3], atol=1e-12)
    assert np.all(np.isnan(eb[0::3])) and np.all(np.isnan(eb[1::3]))


def test_weight_update_matches_fock_space():
    """One oracle step (exact exponential) against Fock space: new overlap
    ratio incl. the mean-field phase, E_L at the new walker, phaseless weight."""
    M, n_up, n_dn = 4, 2, 2
    inp = _small_system(M, n_up, n_dn, 3, seed=71)
    o = Oracle.from_inputs(inp)
    V = fock.eri_from_chol(inp.L)
    H, states, index = fock.hamiltonian_matrix(inp.h, V, inp.e_core, M, n_up, n_dn)
    Lops = [fock.one_body_matrix(inp.L[g], M, states, index) for g in range(3)]
    H1p = (inp.h - 0.5 * np.einsum("gik,gkj->ij", inp.L, inp.L)
           + np.einsum("g,gij->ij", o.lbar, inp.L))
    dt, et = 0.05, -3.0
    B1f = scipy.linalg.expm(-0.5 * dt * fock.one_body_matrix(H1p, M, states, index))
    cT = fock.det_amplitudes(inp.C_up[:, :n_up], inp.C_dn[:, :n_dn], M, states)
    re, im = syn.random_walkers(M, n_up, n_dn, 4, seed=12, scale=0.5)
    st = o.init_walkers(4, phi=re + 1j * im + np.concatenate(
        [inp.C_up[:, :n_up], inp.C_dn[:, :n_dn]], axis=1)[None])
    st.weight = np.array([1.0, 0.5, 2.0, 1.5])
    w0, phi0 = st.weight.copy(), st.phi.copy()
    o.step(st, t=3, seed=5, dt=dt, opt=Options(taylor_order=60, e_trial=et))
    x = gaussian_fields(5, 3, np.arange(4), 3)
    eye = np.eye(len(states))
    for w in range(4):
        c = fock.det_amplitudes(phi0[w][:, :n_up], phi0[w][:, n_up:], M, states)
        ov = cT @ c
        v = np.array([(cT @ Lg @ c) / ov for Lg in Lops])
        xbar = -1j * np.sqrt(dt) * (v - o.lbar)
        gen = sum((x[w, g] - xbar[g]) * (Lops[g] - o.lbar[g] * eye) for g in range(3))
        c1 = B1f @ scipy.linalg.expm(1j * np.sqrt(dt) * gen) @ B1f @ c
        ov1 = cT @ c1
        el = (cT @ H @ c1) / ov1
        wexp = w0[w] * np.exp(-dt * (el.real - et)) * max(0.0, np.cos(np.angle(ov1 / ov)))
        if wexp > 0:
            assert abs(st.eloc[w] - el) < 1e-10 * abs(el)
        assert abs(st.weight[w] - wexp) < 1e-10 * max(1.0, wexp)
