"""FP64 oracle: phaseless AFQMC walker update, written from the paper.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing on the product
path may import this module.

Paper: Shee, Arthur, Zhang, Reichman, Friesner, "Phaseless Auxiliary-Field
Quantum Monte Carlo on Graphical Processing Units" (arXiv 1804.03310).

Notation follows Sec. II: M orbitals, N_sigma electrons per spin, Cholesky
vectors L_gamma with V_ijkl = sum_gamma L_gamma,ik L_gamma,jl (Eq. 1 and the
text after Eq. Ys), auxiliary fields x_gamma (Eq. 2), walker determinants phi
and weights W, trial Psi_T = sum_i c_i |D_i> (Sec. III).

Readings of points the paper leaves open (each is also listed in the design
notes):

* v_gamma = i (L_gamma - lbar_gamma): the two-body term of Eq. 1 is rewritten
  as +1/2 sum_gamma Lhat_gamma^2 minus the one-body normal-ordering term
  1/2 sum_gamma L_gamma L_gamma; Sec. II's form -1/2 sum v^2 then needs the
  factor i, so the propagator of Eq. 2 is exp(i sqrt(dt) sum (x - xbar)(L - lbar)).
  lbar_gamma is the reference determinant's expectation of L_gamma (mean-field
  subtraction, an exact rewrite).
* one-body propagator B1 = exp(-dt H1'/2) with
  H1' = h - 1/2 sum L L + sum lbar L, applied on both sides of the two-body
  factor (symmetric Trotter split).  Real constant scalars are dropped (they
  cancel in the mixed energy); the phase factor exp(-i sqrt(dt) sum (x-xbar) lbar)
  is kept in the overlap ratio.
* force bias xbar_gamma = -sqrt(dt) <v_gamma>_mix = -i sqrt(dt)(v_gamma - lbar_gamma)
  with v_gamma = <L_gamma>_mix (Sec. II: chosen to minimise weight fluctuations).
* weights in the local-energy form W <- W exp(-dt (Re E_L - E_T)) max(0, cos dtheta)
  (Sec. II), E_L evaluated at the propagated walker; dtheta = Im log of the
  overlap ratio.  Optionally the hybrid form the production runs use (Sec.
  IV.A, after Purwanto et al.): W <- W |I| exp(-dt (E_0 - E_T)) max(0, cos dtheta)
  with the importance function I = (<Psi_T|phi'>/<Psi_T|phi>) (mean-field phase
  included) exp(sum_gamma (x_gamma xbar_gamma - xbar_gamma^2 / 2)) and
  E_0 = e_core - 1/2 sum_gamma lbar_gamma^2, the constant the propagator drops;
  E_L is then only measured every meas_every steps.
* exp of the one-body operator by a Taylor series of fixed order.
* walkers that die (weight 0 or any non-finite quantity) are reset to the
  reference determinant with weight 0; they keep being propagated and are
  excluded from every sum by their zero weight.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

MAX_EXC = 4

# ---------------------------------------------------------------------------
# Counter-based random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw,
# "Parallel random numbers: as easy as 1, 2, 3", SC'11).  The fields of Eq. 2
# are standard normal draws; the generator is keyed so that any walker's
# fields can be regenerated alone.
# ---------------------------------------------------------------------------

_PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
_PHILOX_M1 = np.uint64(0xCA5A826395121157)
_PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
_PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo64(a, b):
    """Full 64x64 -> 128-bit product of uint64 arrays, as (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _MASK32, a >> _S32
    b_lo, b_hi = b & _MASK32, b >> _S32
    p_ll = a_lo * b_lo
    p_lh = a_lo * b_hi
    p_hl = a_hi * b_lo
    p_hh = a_hi * b_hi
    mid = (p_ll >> _S32) + (p_lh & _MASK32) + (p_hl & _MASK32)
    hi = p_hh + (p_lh >> _S32) + (p_hl >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox4x64_10(counter, key):
    """Philox4x64 with 10 rounds.

    counter: uint64 array [..., 4]; key: uint64 array [..., 2] (broadcast).
    Each round multiplies words 0 and 2 by the Philox constants, and the new
    words are (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key is bumped by
    the Weyl constants between rounds.
    """
    with np.errstate(over="ignore"):
        c = np.array(counter, dtype=np.uint64, copy=True)
        k = np.broadcast_to(np.asarray(key, dtype=np.uint64), c.shape[:-1] + (2,)).copy()
        for r in range(10):
            if r > 0:
                k[..., 0] = k[..., 0] + _PHILOX_W0
                k[..., 1] = k[..., 1] + _PHILOX_W1
            hi0, lo0 = _mulhilo64(_PHILOX_M0, c[..., 0])
            hi1, lo1 = _mulhilo64(_PHILOX_M1, c[..., 2])
            c = np.stack([hi1 ^ c[..., 1] ^ k[..., 0], lo1,
                          hi0 ^ c[..., 3] ^ k[..., 1], lo0], axis=-1)
        return c


def words_to_uniform(r):
    """Top 53 bits of a 64-bit word to a double in (0, 1): ((r >> 11) + 0.5) 2^-53."""
    r = np.asarray(r, dtype=np.uint64)
    return ((r >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)


FIELD_STREAM = 0
COMB_STREAM = 1


def gaussian_fields(seed: int, t: int, walker_index: Sequence[int], n_chol: int,
                    system_id: int = 0) -> np.ndarray:
    """Auxiliary fields x_{w,gamma} ~ N(0,1) (Eq. 2), shape [len(walker_index), n_chol].

    Key (seed, stream 0); counter (t, walker, gamma // 4, system_id).  The four
    words of one counter give four uniforms u0..u3, turned into four normals
    by the Box-Muller transform: sqrt(-2 ln u0) (cos, sin)(2 pi u1) and
    sqrt(-2 ln u2) (cos, sin)(2 pi u3), in that order for gamma = 4q .. 4q+3.
    """
    widx = np.asarray(walker_index, dtype=np.uint64)
    nq = (n_chol + 3) // 4
    ctr = np.zeros((widx.size, nq, 4), dtype=np.uint64)
    ctr[..., 0] = np.uint64(t)
    ctr[..., 1] = widx[:, None]
    ctr[..., 2] = np.arange(nq, dtype=np.uint64)[None, :]
    ctr[..., 3] = np.uint64(system_id)
    words = philox4x64_10(ctr, np.array([seed, FIELD_STREAM], dtype=np.uint64))
    u = words_to_uniform(words)
    r01 = np.sqrt(-2.0 * np.log(u[..., 0]))
    r23 = np.sqrt(-2.0 * np.log(u[..., 2]))
    z = np.stack([r01 * np.cos(2.0 * np.pi * u[..., 1]),
                  r01 * np.sin(2.0 * np.pi * u[..., 1]),
                  r23 * np.cos(2.0 * np.pi * u[..., 3]),
                  r23 * np.sin(2.0 * np.pi * u[..., 3])], axis=-1)
    return z.reshape(widx.size, nq * 4)[:, :n_chol]


def comb_uniform(seed: int, pc_index: int, system_id: int = 0) -> float:
    """The comb's single uniform xi: key (seed, stream 1), counter (pc_index, 0, 0, system_id), word 0."""
    ctr = np.array([[pc_index, 0, 0, system_id]], dtype=np.uint64)
    w = philox4x64_10(ctr, np.array([seed, COMB_STREAM], dtype=np.uint64))
    return float(words_to_uniform(w[0, 0]))


# ---------------------------------------------------------------------------
# Population control by combing (Sec. IV.A and Sec. V remarks: "simple
# combing"; fixed walker number).
# ---------------------------------------------------------------------------

def comb_parents(weights: np.ndarray, xi: float):
    """Systematic comb of K walkers with one uniform xi in (0,1).

    Inclusive prefix sums C_k are taken left to right; tooth j sits at
    z_j = ((j + xi) * W_tot) / K and picks the first k with C_k > z_j
    (half-open intervals [C_{k-1}, C_k), so zero-weight walkers are never
    picked).  If rounding pushes a tooth past C_{K-1}, the last walker with
    positive weight is taken.  Returns (parents [K] int64, W_tot / K).
    """
    w = np.asarray(weights, dtype=np.float64)
    K = w.size
    C = np.empty(K)
    acc = 0.0
    for k in range(K):  # explicit left-to-right sum
        acc = acc + w[k]
        C[k] = acc
    wtot = C[-1]
    live = np.nonzero(w > 0)[0]
    last = int(live[-1]) if live.size else K - 1
    parents = np.empty(K, dtype=np.int64)
    for j in range(K):
        z = ((j + xi) * wtot) / K
        k = int(np.searchsorted(C, z, side="right"))
        parents[j] = k if k < K else last
    return parents, wtot / K


# ---------------------------------------------------------------------------
# Linear algebra pieces.
# ---------------------------------------------------------------------------

def log_det(S: np.ndarray) -> np.ndarray:
    """Complex log det of a batch of square matrices: log|det| + i arg det."""
    sign, logabs = np.linalg.slogdet(S)
    return logabs + 1j * np.angle(sign)


def taylor_apply(A: np.ndarray, phi: np.ndarray, order: int) -> np.ndarray:
    """exp(A) phi by the Taylor series truncated after A^order / order!.

    T_0 = phi, T_n = A T_{n-1} / n, result = sum_{n=0..order} T_n, summed in
    increasing n.  (Thouless' theorem, Sec. II: the one-body propagator acts
    on a determinant by a matrix product on its orbitals.)
    """
    T = phi
    acc = phi.copy()
    for n in range(1, order + 1):
        T = (A @ T) / n
        acc = acc + T
    return acc


def mgs_orthonormalize(a: np.ndarray) -> np.ndarray:
    """Modified Gram-Schmidt on the columns of a batch [W, M, N] (complex).

    For j = 0..N-1: r_jj = ||q_j||, q_j /= r_jj, then for k > j:
    r_jk = q_j^dagger q_k, q_k -= r_jk q_j.  R has a positive real diagonal,
    so Q is unique (Sec. IV.A: walkers are orthonormalized periodically).
    """
    q = np.array(a, dtype=np.complex128, copy=True)
    N = q.shape[-1]
    for j in range(N):
        rjj = np.sqrt(np.sum(np.abs(q[:, :, j]) ** 2, axis=1))
        q[:, :, j] = q[:, :, j] / rjj[:, None]
        for k in range(j + 1, N):
            rjk = np.sum(np.conj(q[:, :, j]) * q[:, :, k], axis=1)
            q[:, :, k] = q[:, :, k] - rjk[:, None] * q[:, :, j]
    return q


def modified_cholesky(V: np.ndarray, delta: float, max_vectors: Optional[int] = None):
    """Pivoted (modified) Cholesky decomposition of a 4-index ERI (Sec. II).

    V[i,j,k,l] multiplies c+_i c+_j c_l c_k in Eq. 1; as a matrix over the
    pairs (ik),(jl) it is symmetric positive semidefinite.  Vectors are added
    at the pair with the largest remaining diagonal until that diagonal is
    below delta; returns L [n, M, M] with V_ijkl ~= sum_g L_g,ik L_g,jl.
    """
    M = V.shape[0]
    Vm = V.transpose(0, 2, 1, 3).reshape(M * M, M * M)  # rows (ik), cols (jl)
    diag = np.diag(Vm).copy()
    vecs = []
    nmax = M * M if max_vectors is None else max_vectors
    while len(vecs) < nmax:
        p = int(np.argmax(diag))
        if diag[p] < delta:
            break
        col = Vm[:, p].copy()
        for v in vecs:
            col = col - v * v[p]
        vec = col / np.sqrt(diag[p])
        vecs.append(vec)
        diag = diag - vec * vec
    L = np.array(vecs).reshape(len(vecs), M, M) if vecs else np.zeros((0, M, M))
    return L


# ---------------------------------------------------------------------------
# System, walkers, options.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Options:
    taylor_order: int = 6
    ortho_every: int = 0      # 0: never
    pc_every: int = 0         # 0: never
    e_trial: float = 0.0
    mf_subtract: bool = True
    system_id: int = 0
    weight_mode: int = 0      # 0: local-energy form; 1: hybrid form
    meas_every: int = 1       # hybrid: E_mix measured after steps t with (t+1) % meas_every == 0


@dataclasses.dataclass
class WalkerState:
    """Host walker batch.  phi is [W, M, N_up + N_dn] complex (both spins side by side)."""

    phi: np.ndarray
    weight: np.ndarray
    logS: np.ndarray
    eloc: np.ndarray
    v: np.ndarray            # [W, n_chol] mixed estimate <L_gamma> (force-bias input)
    index: np.ndarray        # walker ids used as the field counter

    def copy(self) -> "WalkerState":
        return WalkerState(self.phi.copy(), self.weight.copy(), self.logS.copy(),
                           self.eloc.copy(), self.v.copy(), self.index.copy())


def det_occupations(n_up: int, n_dn: int, exc: np.ndarray):
    """Orbital index lists per determinant and spin.

    Determinant i is the reference (orbitals 0..N_sigma-1) with each hole
    orbital r_e replaced in place by its particle orbital v_e, so the column
    order (and the sign convention) is the one the low-rank update of Sec. III
    produces.
    """
    out = []
    for i in range(exc.shape[0]):
        per_spin = []
        for s, n in enumerate((n_up, n_dn)):
            occ = list(range(n))
            cnt = int(exc[i, s, 0])
            for e in range(cnt):
                r = int(exc[i, s, 1 + e])
                v = int(exc[i, s, 1 + MAX_EXC + e])
                occ[occ.index(r)] = v
            per_spin.append(np.array(occ, dtype=np.int64))
        out.append(per_spin)
    return out


class Oracle:
    """One system: Hamiltonian (h, L, e_core) and trial (orbitals, dets, c_i)."""

    def __init__(self, h, L, e_core, C_up, C_dn, n_up, n_dn, coeff=None, exc=None,
                 mf_subtract: bool = True):
        self.h = np.asarray(h, dtype=np.float64)
        self.L = np.asarray(L, dtype=np.float64)
        self.e_core = float(e_core)
        self.M = self.h.shape[0]
        self.n_chol = self.L.shape[0]
        self.nel = (int(n_up), int(n_dn))
        self.C = (np.asarray(C_up, dtype=np.float64), np.asarray(C_dn, dtype=np.float64))
        if coeff is None:
            coeff = np.ones(1)
            exc = np.zeros((1, 2, 1 + 2 * MAX_EXC), dtype=np.int32)
        self.coeff = np.asarray(coeff, dtype=np.float64)
        self.exc = np.asarray(exc, dtype=np.int32)
        self.n_det = self.coeff.size
        self.occ = det_occupations(n_up, n_dn, self.exc)
        # D_i^sigma: trial determinant orbitals (columns), Sec. III.
        self.D = [[self.C[s][:, self.occ[i][s]] for s in range(2)] for i in range(self.n_det)]
        # Half-rotated tensors C^T L_gamma and C^T h for all M rows; a
        # determinant's rows are picked by its occupation list.
        self.Lfull = [np.einsum("mp,gmn->gpn", self.C[s], self.L, optimize=True) for s in range(2)]
        self.hfull = [self.C[s].T @ self.h for s in range(2)]
        # lbar_gamma = <D_0| L_gamma |D_0> = sum_sigma Tr(D_0^T L_gamma D_0).
        if mf_subtract:
            self.lbar = sum(np.einsum("ma,gmn,na->g", self.D[0][s], self.L, self.D[0][s], optimize=True)
                            for s in range(2) if self.nel[s] > 0)
            if np.isscalar(self.lbar):
                self.lbar = np.zeros(self.n_chol)
        else:
            self.lbar = np.zeros(self.n_chol)
        # H1' = h - 1/2 sum_gamma L_gamma L_gamma + sum_gamma lbar_gamma L_gamma.
        self.H1p = (self.h - 0.5 * np.einsum("gik,gkj->ij", self.L, self.L, optimize=True)
                    + np.einsum("g,gij->ij", self.lbar, self.L, optimize=True))
        # The scalar the propagator leaves out: with 1/2 sum L^2 = 1/2 sum (L - lbar)^2
        # + sum lbar L - 1/2 sum lbar^2, e^{-dt H} = B(x-integral) e^{-dt E_0}.
        self.e0_shift = self.e_core - 0.5 * float(np.dot(self.lbar, self.lbar))
        self._b1 = {}

    @classmethod
    def from_inputs(cls, inp, mf_subtract: bool = True) -> "Oracle":
        return cls(inp.h, inp.L, inp.e_core, inp.C_up, inp.C_dn, inp.n_up, inp.n_dn,
                   inp.coeff, inp.exc, mf_subtract=mf_subtract)

    # -- one-body propagator -------------------------------------------------
    def B1(self, dt: float) -> np.ndarray:
        """exp(-dt H1' / 2) from the eigendecomposition of the symmetric H1'."""
        if dt not in self._b1:
            lam, V = np.linalg.eigh(self.H1p)
            self._b1[dt] = (V * np.exp(-0.5 * dt * lam)) @ V.T
        return self._b1[dt]

    # -- walkers -------------------------------------------------------------
    def reference_phi(self) -> np.ndarray:
        return np.concatenate([self.D[0][0], self.D[0][1]], axis=1).astype(np.complex128)

    def split(self, phi: np.ndarray):
        nu = self.nel[0]
        return phi[:, :, :nu], phi[:, :, nu:]

    def init_walkers(self, W: int, phi: Optional[np.ndarray] = None,
                     index: Optional[np.ndarray] = None) -> WalkerState:
        if phi is None:
            phi = np.broadcast_to(self.reference_phi(), (W, self.M, sum(self.nel))).copy()
        phi = np.asarray(phi, dtype=np.complex128)
        if index is None:
            index = np.arange(phi.shape[0])
        m = self.measure(phi)
        return WalkerState(phi=phi.copy(), weight=np.ones(phi.shape[0]), logS=m["logS"],
                           eloc=m["eloc"], v=m["v"], index=np.asarray(index, dtype=np.int64))

    # -- mixed estimates -----------------------------------------------------
    @staticmethod
    def _det_poly_coeffs(S, Ys):
        """Taylor coefficients of t -> det(S + t Y) for each Y in Ys.

        With the SVD S = U diag(s) V^H and K = U^H Y V,
        det(S + tY) = det(U) det(V^H) det(diag(s) + tK), whose coefficients are
          c0 = prod_i s_i,
          c1 = sum_i K_ii prod_{j!=i} s_j,
          c2 = sum_{i<j} (K_ii K_jj - K_ij K_ji) prod_{k!=i,j} s_k
        times the unit phase det(U) det(V^H).  No inverse of S is taken, so
        the coefficients stay exact when S is singular.

        S: [W, N, N]; Ys: [W, G, N, N].  Returns c0 [W], c1 [W, G], c2 [W, G].
        """
        W, N, _ = S.shape
        U, sig, Vh = np.linalg.svd(S)
        ph = np.linalg.det(U) * np.linalg.det(Vh)
        c0 = ph * np.prod(sig, axis=1)
        P1 = np.empty((W, N))
        P2 = np.zeros((W, N, N))
        for i in range(N):
            P1[:, i] = np.prod(np.delete(sig, i, axis=1), axis=1)
            for j in range(N):
                if j != i:
                    P2[:, i, j] = np.prod(np.delete(sig, [i, j], axis=1), axis=1)
        V = np.conj(np.swapaxes(Vh, 1, 2))
        Uh = np.conj(np.swapaxes(U, 1, 2))
        K = Uh[:, None] @ Ys @ V[:, None]                      # [W, G, N, N]
        d = np.diagonal(K, axis1=2, axis2=3)                  # [W, G, N]
        c1 = ph[:, None] * np.sum(d * P1[:, None, :], axis=2)
        dP2d = np.sum((d @ P2) * d, axis=2)
        kkp = np.sum(K * np.swapaxes(K, 2, 3) * P2[:, None], axis=(2, 3))
        c2 = ph[:, None] * 0.5 * (dP2d - kkp)
        return c0, c1, c2

    def _det_terms(self, i: int, phi_sp):
        """Matrix elements of determinant i with each walker (Sec. II, Eq. 1).

        By Thouless' theorem <D|exp(t A)|phi> = det(D^T exp(tA) phi), so for a
        one-body operator A, <D|A|phi> is the t^1 coefficient of
        det(D^T phi + t D^T A phi), and <D|A^2|phi> is 2 x the t^2 coefficient
        of det(D^T phi + t D^T A phi) plus the t^1 coefficient with A^2.  With
        H = e_core + sum_ij h_ij E_ij + 1/2 sum_gamma (Lhat_gamma^2 - (L_gamma L_gamma)^)
        (Eq. 1 rewritten with V_ijkl = sum L_ik L_jl) the A^2 one-body pieces
        cancel, and over the two spins (product of the per-spin determinants)
          <D|phi>          = c0u c0d
          <D|H1|phi>       = c1u(h) c0d + c0u c1d(h)
          <D|Lhat_g|phi>   = c1u(L_g) c0d + c0u c1d(L_g)
          <D|H2|phi>       = sum_g [c2u(L_g) c0d + c1u(L_g) c1d(L_g) + c0u c2d(L_g)].
        Returns (N0 [W], N_H [W] = <D|H|phi>, NL [W, G]).
        """
        W = phi_sp[0].shape[0]
        G = self.n_chol
        coeffs = []
        for s in range(2):
            if self.nel[s] == 0:
                coeffs.append((np.ones(W, dtype=complex), np.zeros((W, 1), dtype=complex),
                               np.zeros((W, G), dtype=complex), np.zeros((W, G), dtype=complex)))
                continue
            occ = self.occ[i][s]
            D = self.D[i][s]
            S = np.einsum("ma,wmb->wab", D, phi_sp[s], optimize=True)
            Yh = (self.hfull[s][occ, :] @ phi_sp[s])[:, None]
            YL = self.Lfull[s][:, occ, :][None] @ phi_sp[s][:, None]
            c0, c1h, _ = self._det_poly_coeffs(S, Yh)
            _, c1L, c2L = self._det_poly_coeffs(S, YL)
            coeffs.append((c0, c1h, c1L, c2L))
        (u0, u1h, u1L, u2L), (d0, d1h, d1L, d2L) = coeffs
        N0 = u0 * d0
        N1 = u1h[:, 0] * d0 + u0 * d1h[:, 0]
        NL = u1L * d0[:, None] + u0[:, None] * d1L
        N2 = np.sum(u2L * d0[:, None] + u1L * d1L + u0[:, None] * d2L, axis=1)
        return N0, self.e_core * N0 + N1 + N2, NL

    def measure(self, phi: np.ndarray):
        """Overlap, local energy and force-bias input of each walker.

        <Psi_T|phi> = sum_i c_i <D_i|phi> (Sec. III), and by definition
        E_L = <Psi_T|H|phi> / <Psi_T|phi> and v_gamma = <Psi_T|Lhat_gamma|phi> /
        <Psi_T|phi> (Sec. II), the latter being the mixed estimate the force
        bias is built from.  Each determinant is evaluated directly (no
        low-rank update).  Each spin block of phi is scaled by a per-walker
        constant g (the largest singular value of the reference overlap) to
        keep the products in range; log <Psi_T|phi> adds N_sigma log g back.
        """
        phi_sp = list(self.split(phi))
        logscale = np.zeros(phi.shape[0], dtype=np.complex128)
        for s in range(2):
            if self.nel[s] == 0:
                continue
            S0 = np.einsum("ma,wmb->wab", self.D[0][s], phi_sp[s], optimize=True)
            g = np.linalg.svd(S0, compute_uv=False)[:, 0]
            g = np.where(g > 0, g, 1.0)
            phi_sp[s] = phi_sp[s] / g[:, None, None]
            logscale = logscale + self.nel[s] * np.log(g)
        tot = 0.0
        num_h = 0.0
        num_l = 0.0
        for i in range(self.n_det):
            N0, NH, NL = self._det_terms(i, phi_sp)
            tot = tot + self.coeff[i] * N0
            num_h = num_h + self.coeff[i] * NH
            num_l = num_l + self.coeff[i] * NL
        with np.errstate(all="ignore"):
            logS = np.log(tot + 0j) + logscale
            eloc = num_h / tot
            v = num_l / tot[:, None]
        return {"logS": logS, "eloc": eloc, "v": v}

    def local_energy(self, st: WalkerState) -> float:
        """Refresh logS, E_L, v of every walker; return the mixed energy."""
        m = self.measure(st.phi)
        st.logS, st.eloc, st.v = m["logS"], m["eloc"], m["v"]
        return self.mixed_energy(st)

    @staticmethod
    def mixed_energy(st: WalkerState) -> float:
        """E_mix = sum_w W_w Re E_L,w / sum_w W_w (NaN once every walker has
        died: 0 / 0, without a warning)."""
        with np.errstate(invalid="ignore"):
            return float(np.sum(st.weight * st.eloc.real) / np.sum(st.weight))

    # -- propagation ---------------------------------------------------------
    def propagator_matrix(self, xs: np.ndarray, dt: float) -> np.ndarray:
        """A = i sqrt(dt) sum_gamma (x_gamma - xbar_gamma) L_gamma per walker (Eqs. 2-3)."""
        return 1j * np.sqrt(dt) * np.einsum("wg,gij->wij", xs, self.L, optimize=True)

    def apply_propagator(self, phi: np.ndarray, xs: np.ndarray, dt: float, order: int):
        """B1 exp(A) B1 phi for shifted fields xs = x - xbar (Eqs. 2-3, Thouless).

        Returns (phi', mf) where mf = -i sqrt(dt) sum_gamma xs_gamma lbar_gamma is
        the log of the scalar factor exp(-i sqrt(dt) sum xs lbar) that the
        mean-field shift attaches to the determinant.
        """
        A = self.propagator_matrix(xs, dt)
        mf = -1j * np.sqrt(dt) * (xs @ self.lbar)
        B1 = self.B1(dt)
        phi = B1 @ phi
        phi = taylor_apply(A, phi, order)
        phi = B1 @ phi
        return phi, mf

    def shifted_step(self, st: WalkerState, x: np.ndarray, dt: float, order: int):
        """Propagate every walker with fields x shifted by the force bias.

        Returns (phi', measure(phi'), log r, log I): r = <Psi_T|phi'>/<Psi_T|phi>
        with the mean-field phase factor, and the hybrid importance function
        I = r exp(sum_gamma (x_gamma xbar_gamma - xbar_gamma^2 / 2)), whose
        Gaussian average over x is <Psi_T|B1 exp(-dt/2 sum (L - lbar)^2) B1|phi>
        / <Psi_T|phi> for any complex shift xbar (Eq. 2 after x -> x - xbar).
        """
        xbar = -1j * np.sqrt(dt) * (st.v - self.lbar[None, :])
        phi, mf = self.apply_propagator(st.phi, x - xbar, dt, order)
        with np.errstate(all="ignore"):
            m = self.measure(phi)
            logr = m["logS"] - st.logS + mf
            logI = logr + np.sum(x * xbar - 0.5 * xbar * xbar, axis=1)
        return phi, m, logr, logI

    def step(self, st: WalkerState, t: int, seed: int, dt: float, opt: Options):
        """One timestep for every walker; returns the mixed energy after it.

        1. fields x (Eq. 2);  2. force bias xbar = -i sqrt(dt)(v - lbar)
        (Sec. II);  3. phi <- B1 exp(A) B1 phi with exp by Taylor series
        (Eq. 3, Thouless);  4. new overlap, E_L and v;  5. phaseless weight
        update with dtheta = Im log(<Psi_T|phi'>/<Psi_T|phi>) including the
        mean-field phase factor (Sec. II).
        """
        x = gaussian_fields(seed, t, st.index, self.n_chol, opt.system_id)
        phi, m, logr, logI = self.shifted_step(st, x, dt, opt.taylor_order)
        measuring = opt.weight_mode == 0 or (t + 1) % max(opt.meas_every, 1) == 0
        with np.errstate(all="ignore"):
            cosd = np.cos(logr.imag)
            if opt.weight_mode == 0:
                wnew = st.weight * np.exp(-dt * (m["eloc"].real - opt.e_trial)) * np.maximum(0.0, cosd)
            else:
                wnew = (st.weight * np.exp(logI.real - dt * (self.e0_shift - opt.e_trial))
                        * np.maximum(0.0, cosd))
        ok = (np.isfinite(wnew) & np.isfinite(m["logS"])
              & np.all(np.isfinite(m["v"]), axis=1) & (wnew > 0))
        if measuring:
            ok &= np.isfinite(m["eloc"])
        st.phi = phi
        st.weight = np.where(ok, wnew, 0.0)
        st.logS, st.eloc, st.v = m["logS"], m["eloc"], m["v"]
        self._reset_dead(st, ~ok)
        return self.mixed_energy(st) if measuring else float("nan")

    def _reset_dead(self, st: WalkerState, dead: np.ndarray):
        if not np.any(dead):
            return
        ref = self.init_walkers(1)
        st.phi[dead] = ref.phi[0]
        st.logS[dead] = ref.logS[0]
        st.eloc[dead] = ref.eloc[0]
        st.v[dead] = ref.v[0]
        st.weight[dead] = 0.0

    def orthonormalize(self, st: WalkerState):
        """MGS per spin (Sec. IV.A); weights, E_L and v unchanged, logS recomputed."""
        up, dn = self.split(st.phi)
        parts = [mgs_orthonormalize(p) if p.shape[-1] > 0 else p for p in (up, dn)]
        st.phi = np.concatenate(parts, axis=2)
        st.logS = self.measure(st.phi)["logS"]

    def reconfigure(self, st: WalkerState, seed: int, pc_index: int, system_id: int = 0) -> float:
        """Comb (population control); copies walker state, resets weights to 1."""
        xi = comb_uniform(seed, pc_index, system_id)
        parents, norm = comb_parents(st.weight, xi)
        if not (norm > 0.0 and np.isfinite(norm)):
            return 0.0  # every walker dead: population left as it is
        st.phi = st.phi[parents].copy()
        st.logS = st.logS[parents].copy()
        st.eloc = st.eloc[parents].copy()
        st.v = st.v[parents].copy()
        st.weight = np.ones_like(st.weight)
        return norm

    def propagate(self, st: WalkerState, n_steps: int, dt: float, seed: int, step0: int,
                  opt: Options) -> np.ndarray:
        """n_steps timesteps; returns E_mix after each step.

        The call begins by refreshing logS, E_L and v from phi.  After step t
        (global index), walkers are orthonormalized when (t+1) is a multiple
        of ortho_every and combed (pc_index = t) when (t+1) is a multiple of
        pc_every; E_mix is recorded before either.
        """
        m = self.measure(st.phi)
        st.logS, st.eloc, st.v = m["logS"], m["eloc"], m["v"]
        emix = np.zeros(n_steps)
        for s in range(n_steps):
            t = step0 + s
            emix[s] = self.step(st, t, seed, dt, opt)
            if opt.ortho_every > 0 and (t + 1) % opt.ortho_every == 0:
                self.orthonormalize(st)
            if opt.pc_every > 0 and (t + 1) % opt.pc_every == 0:
                self.reconfigure(st, seed, t, opt.system_id)
        return emix
