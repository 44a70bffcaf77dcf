"""Seeded synthetic inputs for the phaseless AFQMC walker update.

This module holds input generation only: one-body matrices, Cholesky-like
vectors, trial orbitals, excitation tables and CI coefficients.  It contains
none of the method's arithmetic (no propagation, overlaps, energies or
weights), so both the FP64 oracle and the HIP path can draw their inputs from
it without sharing any part of the method.

The shapes mirror the paper's workloads (Sec. IV: hydrogen chains in a
double-zeta basis, 5 orbitals per electron pair; Sec. III / V: transition
metal atoms with multi-determinant CASSCF trials).  Real molecular integrals
are not available, so entries are random with the distributions below:

* ``h``: symmetric; diagonal uniform in [-2, 0] Ha, off-diagonal N(0, 0.1)
  (0.1 read as the standard deviation).
* ``L[g]``: symmetric; upper triangle (diagonal included) drawn as
  ``0.5 * N(0,1) * exp(-g / tau_d)`` and mirrored.  ``V_ijkl = sum_g
  L[g,i,k] L[g,j,l]`` is then positive semidefinite as an (ik),(jl) matrix,
  like a Cholesky-decomposed two-electron integral (Sec. II, Eq. 1).
  The workloads with ``tau_d = 50`` then multiply every ``L[g]`` by
  ``l_scale = 1 / sqrt(M)`` (``health_scale``).  Unscaled, the spectral
  norm of the one-step propagator exponent ``sqrt(dt) sum_g x_g L[g]`` is
  about 2 to 5 at M = 50 to 200 (against 0.44 for the M = 10 workload), the
  exchange energy reaches 1e4 Ha and every walker of the M = 50 workload is
  dead within five steps.  The scale brings that norm to about 0.3; at the
  M = 50 size the walkers' Im E_L spread then stays near 3 Ha and no walker
  dies in 60 steps without population control, while at a norm of 0.44 the
  spread grows past 30 Ha by step 60.  The unscaled recipe stays available
  as ``hchain-M50-literal``.
* trial orbitals: all eigenvectors of ``h`` in ascending eigenvalue order,
  each column sign-fixed so that its largest-magnitude entry is positive
  (lowest index on ties).  The reference determinant occupies the first
  ``N_sigma`` columns.
* multi-determinant excitations: single/double excitations of the reference
  drawn as described in ``make_excitations``; coefficients ``0.1 * N(0,1)``
  with the reference coefficient 1.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

MAX_EXC = 4  # excitations per spin that the excitation table can hold
EXC_ROW = 1 + 2 * MAX_EXC  # (count, holes[MAX_EXC], particles[MAX_EXC])


@dataclasses.dataclass
class Workload:
    """A named synthetic workload (shapes and run parameters)."""

    name: str
    M: int
    n_up: int
    n_dn: int
    n_chol: int
    n_walkers: int
    n_steps: int
    dt: float
    tau_d: float
    n_det: int = 1
    chol_prec: str = "fp64"
    taylor_prec: str = "fp64"
    taylor_order: int = 6
    ortho_every: int = 2
    pc_every: int = 0
    ham_seed: int = 0
    field_seed: int = 0
    l_scale: float = 1.0


def health_scale(M: int) -> float:
    """Factor applied to the Cholesky-like vectors of the tau_d = 50
    workloads: brings ||sqrt(dt) sum_g x_g L[g]||_2 to about 0.3 at dt = 0.005."""
    return 1.0 / float(np.sqrt(M))


# The four single-system workloads of the measurement plan.  Run parameters
# the paper does not state (Taylor order, orthonormalisation and population
# control intervals for some sizes) follow the readings listed in the design
# notes: ortho every 2 steps (Sec. IV.A), population control every 0.1 Ha^-1
# = 20 steps at dt = 0.005 (Sec. IV.A).
WORKLOADS = {
    "plain-M10": Workload("plain-M10", M=10, n_up=5, n_dn=5, n_chol=40,
                          n_walkers=64, n_steps=100, dt=0.005, tau_d=8.0,
                          ortho_every=2, pc_every=0),
    "hchain-M50": Workload("hchain-M50", M=50, n_up=25, n_dn=25, n_chol=250,
                           n_walkers=1024, n_steps=1000, dt=0.005, tau_d=50.0,
                           chol_prec="fp32", taylor_prec="fp32",
                           ortho_every=10, pc_every=20, l_scale=health_scale(50)),
    "hchain-M50-literal": Workload("hchain-M50-literal", M=50, n_up=25, n_dn=25,
                                   n_chol=250, n_walkers=1024, n_steps=1000, dt=0.005,
                                   tau_d=50.0, chol_prec="fp32", taylor_prec="fp32",
                                   ortho_every=10, pc_every=20),
    "tm-multidet-M120": Workload("tm-multidet-M120", M=120, n_up=13, n_dn=11,
                                 n_chol=600, n_walkers=2048, n_steps=500,
                                 dt=0.005, tau_d=50.0, n_det=100,
                                 chol_prec="fp32", ortho_every=2, pc_every=20,
                                 l_scale=health_scale(120)),
    "sweep-M200": Workload("sweep-M200", M=200, n_up=50, n_dn=50, n_chol=1000,
                           n_walkers=1024, n_steps=200, dt=0.005, tau_d=50.0,
                           chol_prec="bf16", ortho_every=2, pc_every=20,
                           l_scale=health_scale(200)),
}


def make_hamiltonian(M: int, n_chol: int, tau_d: float, seed: int = 0,
                     l_scale: float = 1.0):
    """Return (h [M,M], L [n_chol,M,M]) as float64 arrays."""
    rng = np.random.default_rng(seed)
    h = np.zeros((M, M))
    iu = np.triu_indices(M, 1)
    h[iu] = rng.normal(0.0, 0.1, size=iu[0].size)
    h = h + h.T
    h[np.diag_indices(M)] = rng.uniform(-2.0, 0.0, size=M)
    L = np.zeros((n_chol, M, M))
    iu0 = np.triu_indices(M)
    for g in range(n_chol):
        vals = 0.5 * rng.standard_normal(iu0[0].size) * np.exp(-g / tau_d)
        Lg = np.zeros((M, M))
        Lg[iu0] = vals
        L[g] = Lg + Lg.T - np.diag(np.diag(Lg))
    if l_scale != 1.0:
        L *= l_scale
    return h, L


def sign_fix_columns(C: np.ndarray) -> np.ndarray:
    """Flip each column so its largest-|.| entry is positive (first on ties)."""
    C = np.array(C, dtype=np.float64, copy=True)
    for j in range(C.shape[1]):
        k = int(np.argmax(np.abs(C[:, j])))
        if C[k, j] < 0:
            C[:, j] = -C[:, j]
    return C


def make_trial_orbitals(h: np.ndarray) -> np.ndarray:
    """All eigenvectors of h (ascending), sign-fixed; columns are orbitals."""
    _, vecs = np.linalg.eigh(h)
    return sign_fix_columns(vecs)


def make_excitations(M: int, n_up: int, n_dn: int, n_det: int, seed: int):
    """Reference plus (n_det - 1) distinct single/double excitations.

    Each non-reference determinant: excitation level 1 or 2 with p = 1/2;
    a single picks the spin with p = 1/2; a double picks the channel
    (up-up, dn-dn, up-dn) uniformly.  Holes are drawn uniformly without
    replacement among the occupied orbitals of that spin, particles uniformly
    without replacement among its virtual orbitals; holes and particles are
    each sorted and paired in order.  Duplicates are rejected.

    Returns (exc [n_det, 2, EXC_ROW] int32, coeff [n_det] float64).
    """
    rng = np.random.default_rng(seed)
    exc = np.zeros((n_det, 2, EXC_ROW), dtype=np.int32)
    coeff = np.zeros(n_det)
    coeff[0] = 1.0
    seen = {((), (), (), ())}
    nocc = (n_up, n_dn)
    i = 1
    while i < n_det:
        level = 1 if rng.random() < 0.5 else 2
        if level == 1:
            per_spin = (1, 0) if rng.random() < 0.5 else (0, 1)
        else:
            ch = int(rng.integers(3))
            per_spin = [(2, 0), (0, 2), (1, 1)][ch]
        entry = []
        for s in range(2):
            k = per_spin[s]
            if k == 0:
                entry.append(((), ()))
                continue
            if k > nocc[s] or k > M - nocc[s]:
                entry = None
                break
            holes = tuple(sorted(rng.choice(nocc[s], size=k, replace=False).tolist()))
            parts = tuple(sorted((nocc[s] + rng.choice(M - nocc[s], size=k, replace=False)).tolist()))
            entry.append((holes, parts))
        if entry is None:
            continue
        key = (entry[0][0], entry[0][1], entry[1][0], entry[1][1])
        if key in seen:
            continue
        seen.add(key)
        for s in range(2):
            holes, parts = entry[s]
            exc[i, s, 0] = len(holes)
            for e, (r, v) in enumerate(zip(holes, parts)):
                exc[i, s, 1 + e] = r
                exc[i, s, 1 + MAX_EXC + e] = v
        coeff[i] = 0.1 * rng.standard_normal()
        i += 1
    return exc, coeff


@dataclasses.dataclass
class SystemInputs:
    h: np.ndarray
    L: np.ndarray
    e_core: float
    C_up: np.ndarray
    C_dn: np.ndarray
    n_up: int
    n_dn: int
    coeff: np.ndarray
    exc: np.ndarray

    @property
    def M(self) -> int:
        return self.h.shape[0]

    @property
    def n_chol(self) -> int:
        return self.L.shape[0]

    @property
    def n_det(self) -> int:
        return self.coeff.shape[0]


def make_system(M: int, n_up: int, n_dn: int, n_chol: int, tau_d: float,
                n_det: int = 1, seed: int = 0, e_core: float = 0.0,
                exc_seed: Optional[int] = None, l_scale: float = 1.0) -> SystemInputs:
    h, L = make_hamiltonian(M, n_chol, tau_d, seed, l_scale)
    C = make_trial_orbitals(h)
    if n_det > 1:
        exc, coeff = make_excitations(M, n_up, n_dn, n_det,
                                      seed + 1000 if exc_seed is None else exc_seed)
    else:
        exc = np.zeros((1, 2, EXC_ROW), dtype=np.int32)
        coeff = np.ones(1)
    return SystemInputs(h=h, L=L, e_core=e_core, C_up=C.copy(), C_dn=C.copy(),
                        n_up=n_up, n_dn=n_dn, coeff=coeff, exc=exc)


def workload_system(w: Workload) -> SystemInputs:
    return make_system(w.M, w.n_up, w.n_dn, w.n_chol, w.tau_d, n_det=w.n_det,
                       seed=w.ham_seed, l_scale=w.l_scale)


def random_walkers(M: int, n_up: int, n_dn: int, W: int, seed: int,
                   scale: float = 1.0):
    """Random complex orbital matrices [W, M, n_up + n_dn] (re, im), for
    tests that need walkers away from the trial."""
    rng = np.random.default_rng(seed)
    nt = n_up + n_dn
    re = scale * rng.standard_normal((W, M, nt))
    im = scale * rng.standard_normal((W, M, nt))
    return re, im


def trial_walkers(C_up: np.ndarray, C_dn: np.ndarray, n_up: int, n_dn: int, W: int):
    """W copies of the reference determinant [C_up[:, :n_up] | C_dn[:, :n_dn]]."""
    D0 = np.concatenate([C_up[:, :n_up], C_dn[:, :n_dn]], axis=1)
    re = np.broadcast_to(D0, (W,) + D0.shape).copy()
    im = np.zeros_like(re)
    return re, im
