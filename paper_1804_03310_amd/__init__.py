"""MI355X (gfx950) phaseless AFQMC walker update (arXiv 1804.03310).

Python binding of the C ABI in include/afqmc.h.  This module only marshals
arguments: host inputs go in as numpy float64 arrays, walker state lives in
torch CUDA tensors (device memory) and work is enqueued on torch's current
stream.  Every step of the walker update runs in the HIP kernels of
libafqmc.so; importing this package builds that library when it is missing or
stale (hipcc, gfx950) and fails if it cannot be built or loaded.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import _abi
from ._abi import AfqmcError, GroupMemberStruct, OptionsStruct, WalkersStruct, check

__all__ = ["Hamiltonian", "Trial", "Walkers", "Options", "AfqmcError", "propagate",
           "local_energy", "orthonormalize", "reconfigure", "fields", "walkers_from_trial",
           "timing_enable", "timing_read", "reblock", "cs_difference", "Group", "GroupMember",
           "resident_supported", "tune_cache_path"]

_lib = _abi.load()


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None) -> Optional[int]:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _host(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


class Hamiltonian:
    """h [M,M], L [n_chol,M,M] (V_ijkl = sum_g L_g,ik L_g,jl) and e_core, copied to the device."""

    def __init__(self, h, L, e_core: float = 0.0, device: int = 0, stream=None):
        h = _host(h)
        L = _host(L)
        self.M = h.shape[0]
        self.n_chol = L.shape[0]
        self.device = device
        out = ctypes.c_void_p()
        check(_lib.afqmc_init_hamiltonian(ctypes.byref(out), device, _stream_ptr(stream), self.M,
                                          self.n_chol, h.ctypes.data, L.ctypes.data if L.size else None,
                                          float(e_core)))
        self._h = out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.afqmc_free_hamiltonian(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None


class Trial:
    """Psi_T = sum_i coeff[i] |D_i> over orbitals C_up / C_dn (columns)."""

    def __init__(self, ham: Hamiltonian, n_up: int, n_dn: int, C_up, C_dn, coeff=None, exc=None,
                 mf_subtract: bool = True):
        C_up = _host(C_up)
        C_dn = _host(C_dn)
        self.ham = ham
        self.n_up, self.n_dn = int(n_up), int(n_dn)
        n_det = 1 if coeff is None else int(np.asarray(coeff).size)
        cptr = eptr = None
        if coeff is not None:
            self._coeff = _host(coeff)
            self._exc = np.ascontiguousarray(exc, dtype=np.int32)
            cptr, eptr = self._coeff.ctypes.data, self._exc.ctypes.data
        out = ctypes.c_void_p()
        check(_lib.afqmc_init_trial(ctypes.byref(out), ham._h, self.n_up, self.n_dn,
                                    C_up.ctypes.data, C_dn.ctypes.data, n_det, cptr, eptr,
                                    1 if mf_subtract else 0))
        self._t = out
        self.n_det = n_det

    def workspace_bytes(self, n_walkers: int) -> int:
        b = ctypes.c_size_t()
        check(_lib.afqmc_walker_workspace_bytes(self._t, int(n_walkers), ctypes.byref(b)))
        return int(b.value)

    @property
    def exchange_route(self) -> str:
        """"ltilde" (per-vector X_g = Ltil_g Theta) or "q" (two-index tensor Q)."""
        r = ctypes.c_int()
        check(_lib.afqmc_trial_exchange_route(self._t, ctypes.byref(r)))
        return "q" if r.value == 1 else "ltilde"

    @exchange_route.setter
    def exchange_route(self, route: str) -> None:
        codes = {"ltilde": 0, "q": 1}
        if route not in codes:
            raise ValueError(f"exchange route must be one of {sorted(codes)}")
        check(_lib.afqmc_trial_set_exchange_route(self._t, codes[route]))

    def __del__(self):
        t = getattr(self, "_t", None)
        if t and _lib is not None:
            try:
                _lib.afqmc_free_trial(t)
            except Exception:  # interpreter shutdown
                pass
            self._t = None


class Walkers:
    """Caller-owned device buffers of a walker batch (torch tensors)."""

    def __init__(self, trial: Trial, n_walkers: int, system_id: int = 0, device: Optional[int] = None):
        torch = _torch()
        dev = torch.device("cuda", trial.ham.device if device is None else device)
        M, nt = trial.ham.M, trial.n_up + trial.n_dn
        f64 = dict(dtype=torch.float64, device=dev)
        self.trial = trial
        self.n_walkers = int(n_walkers)
        self.system_id = int(system_id)
        self.phi_re = torch.zeros((n_walkers, M, nt), **f64)
        self.phi_im = torch.zeros((n_walkers, M, nt), **f64)
        self.weight = torch.ones(n_walkers, **f64)
        self.logovlp = torch.zeros((2, n_walkers), **f64)
        self.eloc = torch.zeros((2, n_walkers), **f64)
        nbytes = trial.workspace_bytes(n_walkers)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.struct = WalkersStruct(
            self.n_walkers, self.system_id, self.phi_re.data_ptr(), self.phi_im.data_ptr(),
            self.weight.data_ptr(), self.logovlp[0].data_ptr(), self.logovlp[1].data_ptr(),
            self.eloc[0].data_ptr(), self.eloc[1].data_ptr(), self.workspace.data_ptr(), nbytes)


@dataclass
class Options:
    taylor_order: int = 6
    ortho_every: int = 0
    pc_every: int = 0
    e_trial: float = 0.0
    chol_prec: str = "fp64"
    taylor_prec: str = "fp64"
    weight_mode: str = "local"   # "local" (local-energy form) or "hybrid"
    meas_every: int = 1          # hybrid: E_L / E_mix after steps t with (t+1) % meas_every == 0

    def struct(self) -> OptionsStruct:
        return OptionsStruct(self.taylor_order, self.ortho_every, self.pc_every, float(self.e_trial),
                             _abi.PREC[self.chol_prec], _abi.PREC[self.taylor_prec],
                             _abi.WEIGHT_MODES[self.weight_mode], int(self.meas_every))


def walkers_from_trial(ham: Hamiltonian, trial: Trial, w: Walkers, stream=None) -> None:
    check(_lib.afqmc_walkers_from_trial(ham._h, trial._t, ctypes.byref(w.struct), _stream_ptr(stream)))


def propagate(ham: Hamiltonian, trial: Trial, w: Walkers, n_steps: int, dt: float, seed: int,
              step0: int, opt: Options, emix=None, stream=None):
    """Enqueue n_steps timesteps; returns the device tensor of E_mix after each step."""
    torch = _torch()
    if emix is None:
        emix = torch.empty(max(n_steps, 1), dtype=torch.float64, device=w.weight.device)
    o = opt.struct()
    check(_lib.afqmc_propagate(ham._h, trial._t, ctypes.byref(w.struct), int(n_steps), float(dt),
                               int(seed), int(step0), ctypes.byref(o), emix.data_ptr(),
                               _stream_ptr(stream)))
    return emix


@dataclass
class GroupMember:
    """One system of a group: its Hamiltonian, trial, walkers, time step,
    field seed and options (afqmc_group_member)."""
    ham: Hamiltonian
    trial: Trial
    walkers: Walkers
    dt: float
    seed: int
    opt: Options


def resident_supported(trial: Trial) -> bool:
    ok = ctypes.c_int()
    check(_lib.afqmc_resident_supported(trial._t, ctypes.byref(ok)))
    return bool(ok.value)


def tune_cache_path(path: Optional[str]) -> None:
    check(_lib.afqmc_tune_cache_path(None if path is None else path.encode()))


class Group:
    """Several systems propagated together by the walker-resident kernel
    (afqmc_group_*): one launch per segment of steps over every walker of
    every member, each segment a replayed HIP graph."""

    def __init__(self, members, stream=None):
        self.members = list(members)
        n = len(self.members)
        self._structs = (GroupMemberStruct * n)()
        for k, m in enumerate(self.members):
            self._structs[k] = GroupMemberStruct(m.ham._h, m.trial._t, ctypes.pointer(m.walkers.struct),
                                                 float(m.dt), int(m.seed), m.opt.struct())
        out = ctypes.c_void_p()
        check(_lib.afqmc_group_create(ctypes.byref(out), n, self._structs, _stream_ptr(stream)))
        self._g = out

    def propagate(self, n_steps: int, step0: int = 0, emix=None, stream=None):
        """Enqueue n_steps steps of every member; returns the list of E_mix
        device tensors (one per member, [n_steps])."""
        torch = _torch()
        if emix is None:
            emix = [torch.empty(max(n_steps, 1), dtype=torch.float64, device=m.walkers.weight.device)
                    for m in self.members]
        ptrs = (ctypes.c_void_p * len(self.members))(
            *[e.data_ptr() if e is not None else None for e in emix])
        check(_lib.afqmc_group_propagate(self._g, int(n_steps), int(step0), ptrs, _stream_ptr(stream)))
        return emix

    def tune(self, steps: int = 40, stream=None) -> float:
        us = ctypes.c_double()
        check(_lib.afqmc_group_tune(self._g, int(steps), ctypes.byref(us), _stream_ptr(stream)))
        return us.value

    @property
    def config(self):
        """(threads per walker block, segment steps, tuned: 0 default / 1 measured / 2 cached)."""
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(_lib.afqmc_group_config(self._g, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def set_config(self, threads: int, segment_steps: int) -> None:
        check(_lib.afqmc_group_set_config(self._g, int(threads), int(segment_steps)))

    def timing(self, enable: bool) -> None:
        """Time the resident launches with HIP events (segments then launch
        directly, not as graphs)."""
        check(_lib.afqmc_group_timing(self._g, 1 if enable else 0))

    def timing_read(self):
        """(launches, steps covered, total ms) of the timed resident launches; clears them."""
        n, s, ms = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        check(_lib.afqmc_group_timing_read(self._g, ctypes.byref(n), ctypes.byref(s), ctypes.byref(ms)))
        return n.value, s.value, ms.value

    def __del__(self):
        g = getattr(self, "_g", None)
        if g and _lib is not None:
            try:
                _lib.afqmc_free_group(g)
            except Exception:  # interpreter shutdown
                pass
            self._g = None


def local_energy(ham: Hamiltonian, trial: Trial, w: Walkers, stream=None) -> float:
    out = ctypes.c_double()
    check(_lib.afqmc_local_energy(ham._h, trial._t, ctypes.byref(w.struct), ctypes.byref(out),
                                  _stream_ptr(stream)))
    return out.value


def orthonormalize(ham: Hamiltonian, trial: Trial, w: Walkers, stream=None) -> None:
    check(_lib.afqmc_orthonormalize(ham._h, trial._t, ctypes.byref(w.struct), _stream_ptr(stream)))


def reconfigure(trial: Trial, w: Walkers, seed: int, pc_index: int, stream=None) -> float:
    out = ctypes.c_double()
    check(_lib.afqmc_reconfigure(trial._t, ctypes.byref(w.struct), int(seed), int(pc_index),
                                 ctypes.byref(out), _stream_ptr(stream)))
    return out.value


def reblock(x, max_levels: int = 64):
    """Blocking analysis of a correlated energy series on the host (C ABI
    afqmc_reblock).  Returns (mean, [standard error per level], plateau
    level or -1)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    sem = np.zeros(max_levels)
    mean = ctypes.c_double()
    nl, pl = ctypes.c_int(), ctypes.c_int()
    check(_lib.afqmc_reblock(x.ctypes.data, x.size, max_levels, ctypes.byref(mean), sem.ctypes.data,
                             ctypes.byref(nl), ctypes.byref(pl)))
    return mean.value, [float(v) for v in sem[:nl.value]], pl.value


def cs_difference(a, b, first: int = 0):
    """Correlated-sampling difference of two [repeats][steps] energy series on
    the host (C ABI afqmc_cs_difference).  Returns (mean[steps], sem[steps]) of
    the cumulative average of b - a over the repeats."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64))
    if a.shape != b.shape or a.ndim != 2:
        raise ValueError("a and b must be [repeats][steps] of the same shape")
    mean = np.zeros(a.shape[1])
    sem = np.zeros(a.shape[1])
    check(_lib.afqmc_cs_difference(a.ctypes.data, b.ctypes.data, a.shape[0], a.shape[1], int(first),
                                   mean.ctypes.data, sem.ctypes.data))
    return mean, sem


def timing_enable(ham: Hamiltonian, classes=True) -> None:
    """Time the kernel classes named in `classes` (True: all, False: none)."""
    if classes is True:
        mask = (1 << len(_abi.KERNEL_CLASSES)) - 1
    elif classes is False or classes is None:
        mask = 0
    else:
        mask = 0
        for c in classes:
            mask |= 1 << _abi.KERNEL_CLASSES.index(c)
    check(_lib.afqmc_timing_enable(ham._h, mask))


def timing_read(ham: Hamiltonian, kernel_class: str):
    """(launches, total_ms) of one kernel class since the last read."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    check(_lib.afqmc_timing_read(ham._h, _abi.KERNEL_CLASSES.index(kernel_class), ctypes.byref(n),
                                 ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def fields(seed: int, t: int, n_walkers: int, n_chol: int, system_id: int = 0, device: int = 0,
           stream=None):
    torch = _torch()
    x = torch.empty((n_walkers, n_chol), dtype=torch.float64, device=torch.device("cuda", device))
    check(_lib.afqmc_fields(int(seed), int(t), int(n_walkers), int(n_chol), int(system_id),
                            x.data_ptr(), _stream_ptr(stream)))
    return x
