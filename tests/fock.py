"""Brute-force second quantisation on tiny systems (test helper).

Spin orbitals are numbered p = i (spin up) and p = M + i (spin down); a basis
state is the bit string of occupied spin orbitals, and |n> = c+_{p1} c+_{p2}
... |0> with p1 < p2 < ... .  Operators act with the Jordan-Wigner sign
(-1)^(number of occupied spin orbitals below p).

Nothing here is shared with the oracle or the HIP path: it is an independent
route to the same quantities, written from Eq. 1 of the paper.
"""
from __future__ import annotations

import itertools

import numpy as np

MAX_EXC = 4
EXC_ROW = 1 + 2 * MAX_EXC


def basis(M: int, n_up: int, n_dn: int):
    states = []
    for occ_up in itertools.combinations(range(M), n_up):
        for occ_dn in itertools.combinations(range(M), n_dn):
            bits = 0
            for i in occ_up:
                bits |= 1 << i
            for i in occ_dn:
                bits |= 1 << (M + i)
            states.append(bits)
    index = {b: k for k, b in enumerate(states)}
    return states, index


def _annihilate(bits, p):
    if not (bits >> p) & 1:
        return None, 0
    sign = -1 if bin(bits & ((1 << p) - 1)).count("1") % 2 else 1
    return bits ^ (1 << p), sign


def _create(bits, p):
    if (bits >> p) & 1:
        return None, 0
    sign = -1 if bin(bits & ((1 << p) - 1)).count("1") % 2 else 1
    return bits | (1 << p), sign


def apply_string(bits, ops):
    """Apply a product of operators, rightmost first.  ops: list of (p, 'c'|'a')."""
    sign = 1
    for p, kind in reversed(ops):
        if kind == "a":
            bits, s = _annihilate(bits, p)
        else:
            bits, s = _create(bits, p)
        if bits is None:
            return None, 0
        sign *= s
    return bits, sign


def one_body_matrix(T, M, states, index):
    """sum_ij T_ij sum_sigma c+_{i sigma} c_{j sigma} in the given basis."""
    n = len(states)
    H = np.zeros((n, n), dtype=np.result_type(T, np.float64))
    for col, b in enumerate(states):
        for s in range(2):
            for i in range(M):
                for j in range(M):
                    if T[i, j] == 0:
                        continue
                    nb, sg = apply_string(b, [(s * M + i, "c"), (s * M + j, "a")])
                    if nb is not None and nb in index:
                        H[index[nb], col] += sg * T[i, j]
    return H


def two_body_matrix(V, M, states, index):
    """1/2 sum_ijkl V_ijkl sum_{sigma,tau} c+_{i s} c+_{j t} c_{l t} c_{k s} (Eq. 1)."""
    n = len(states)
    H = np.zeros((n, n))
    nz = np.argwhere(np.abs(V) > 0)
    for col, b in enumerate(states):
        for (i, j, k, l) in nz:
            val = 0.5 * V[i, j, k, l]
            for s in range(2):
                for t in range(2):
                    nb, sg = apply_string(b, [(s * M + i, "c"), (t * M + j, "c"),
                                              (t * M + l, "a"), (s * M + k, "a")])
                    if nb is not None and nb in index:
                        H[index[nb], col] += sg * val
    return H


def hamiltonian_matrix(h, V, e_core, M, n_up, n_dn):
    states, index = basis(M, n_up, n_dn)
    H = one_body_matrix(h, M, states, index) + two_body_matrix(V, M, states, index)
    H = H + e_core * np.eye(len(states))
    return H, states, index


def det_amplitudes(phi_up, phi_dn, M, states):
    """<n|phi> for the determinant with up orbitals phi_up [M,N_up] and down phi_dn."""
    out = np.zeros(len(states), dtype=np.result_type(phi_up, phi_dn, np.float64))
    for k, b in enumerate(states):
        occ_up = [i for i in range(M) if (b >> i) & 1]
        occ_dn = [i for i in range(M) if (b >> (M + i)) & 1]
        a = np.linalg.det(phi_up[occ_up, :]) if occ_up else 1.0
        d = np.linalg.det(phi_dn[occ_dn, :]) if occ_dn else 1.0
        out[k] = a * d
    return out


def eri_from_chol(L):
    """V_ijkl = sum_g L_g,ik L_g,jl."""
    return np.einsum("gik,gjl->ijkl", L, L)


def permutation_sign(seq):
    """Sign of the permutation that sorts seq (distinct entries)."""
    seq = list(seq)
    sign = 1
    for i in range(len(seq)):
        for j in range(i + 1, len(seq)):
            if seq[i] > seq[j]:
                sign = -sign
    return sign


def fci_trial(h, L, e_core, C, n_up, n_dn):
    """Exact ground state of the Fock-space H, expressed as a multi-determinant
    trial over the orbitals C with the in-place hole->particle convention."""
    M = h.shape[0]
    hmo = C.T @ h @ C
    Lmo = np.einsum("ip,gij,jq->gpq", C, L, C)
    H, states, _ = hamiltonian_matrix(hmo, eri_from_chol(Lmo), e_core, M, n_up, n_dn)
    evals, evecs = np.linalg.eigh(H)
    # any eigenstate gives zero variance; take the lowest one with a sizeable
    # reference amplitude (walkers start at the reference determinant)
    ref_bits = sum(1 << i for i in range(n_up)) | sum(1 << (M + i) for i in range(n_dn))
    kref = states.index(ref_bits)
    pick = next(k for k in range(len(evals)) if abs(evecs[kref, k]) > 0.05)
    c = evecs[:, pick]
    exc_rows, coeff = [], []
    for k, b in enumerate(states):
        if abs(c[k]) < 1e-14:
            continue
        row = np.zeros((2, EXC_ROW), dtype=np.int32)
        sign = 1
        for s, n in enumerate((n_up, n_dn)):
            occ = [i for i in range(M) if (b >> (s * M + i)) & 1]
            holes = sorted(set(range(n)) - set(occ))
            parts = sorted(set(occ) - set(range(n)))
            inplace = list(range(n))
            for r, v in zip(holes, parts):
                inplace[inplace.index(r)] = v
            sign *= permutation_sign(inplace)
            row[s, 0] = len(holes)
            for e, (r, v) in enumerate(zip(holes, parts)):
                row[s, 1 + e] = r
                row[s, 1 + MAX_EXC + e] = v
        exc_rows.append(row)
        coeff.append(sign * c[k])
    # the reference (no excitations) first
    order = sorted(range(len(exc_rows)), key=lambda i: (exc_rows[i][0, 0] + exc_rows[i][1, 0]) != 0)
    exc = np.array([exc_rows[i] for i in order])
    coeff = np.array([coeff[i] for i in order])
    assert exc[0, 0, 0] == 0 and exc[0, 1, 0] == 0
    return exc, coeff, evals[pick]
