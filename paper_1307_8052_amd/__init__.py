"""MI355X (gfx950) library for the RPA correlation energy in the PAW method:
chi0(q; G, G'; i w) from pair densities and E_c(q) (arXiv 1307.8052).

This module only marshals arguments to the C ABI of ``include/rpa.h``; every
step of the computation runs in the HIP library. Device arrays are torch
tensors on a ROCm device; the work is ordered on torch's current stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

from . import _capi
from ._capi import PRECISION, RpaCell, RpaFreq, RpaQSpec, RpaStates

__all__ = ["RpaError", "Context", "States", "SymOp", "QSpec", "Freq", "gsphere", "PRECISION", "library_path",
           "ec_autograd"]


def library_path() -> str:
    return _capi.LIB_PATH


class RpaError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        msg = _capi.lib().rpa_status_string(status).decode()
        super().__init__(f"[{status}] {msg}: {detail}")


def _check(status: int, ctx=None):
    if status != 0:
        detail = _capi.lib().rpa_last_error(ctx).decode(errors="replace")
        raise RpaError(status, detail)


def _torch():
    import torch
    return torch


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr_i32(a: np.ndarray):
    return a.ctypes.data_as(_capi.P_i32)


def _ptr_f64(a: np.ndarray):
    return a.ctypes.data_as(_capi.P_f64)


def _dev_c128(t, device):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t, dtype=np.complex128))
    return t.to(device=device, dtype=torch.complex128).contiguous()


def _cell(A, grid) -> RpaCell:
    c = RpaCell()
    a = _f64(A).reshape(9)
    for i in range(9):
        c.A[i] = float(a[i])
    for i in range(3):
        c.n[i] = int(grid[i])
    return c


def gsphere(A, grid, q, ecut: float) -> np.ndarray:
    """The chi G-sphere |q+G|^2/2 <= ecut in the library's canonical order (host only)."""
    L = _capi.lib()
    cell = _cell(A, grid)
    qv = _f64(q)
    ng = ctypes.c_int(0)
    _check(L.rpa_gsphere(ctypes.byref(cell), _ptr_f64(qv), float(ecut), None, 0, ctypes.byref(ng)))
    out = np.zeros((max(ng.value, 1), 3), dtype=np.int32)
    _check(L.rpa_gsphere(ctypes.byref(cell), _ptr_f64(qv), float(ecut), _ptr_i32(out), ng.value, ctypes.byref(ng)))
    return out[: ng.value]


class SymOp:
    """A point operation carrying a state set at k1 (irreducible zone) to k = (-1)^s T k1 + G0 (rpa_symop):
    rot U (fractional x -> U x), time reversal s, gshift G0 (Miller units), kibz = k1 (Cartesian), and for
    PAW atoms the atom map b(a), lattice shifts L_a (T^-1 R_a = R_b + L_a) and the flat D blocks."""

    def __init__(self, rot, time_reversal, gshift, kibz, atom_map=None, atom_shift=None, proj_rot=None):
        self.rot = _i32(rot).reshape(3, 3)
        self.time_reversal = int(bool(time_reversal))
        self.gshift = _i32(gshift).reshape(3)
        self.kibz = _f64(kibz).reshape(3)
        self.atom_map = None if atom_map is None else _i32(atom_map)
        self.atom_shift = None if atom_shift is None else _i32(atom_shift).reshape(-1, 3)
        self.proj_rot = None if proj_rot is None else _f64(proj_rot)
        st = _capi.RpaSymop()
        for i in range(3):
            for j in range(3):
                st.rot[i][j] = int(self.rot[i, j])
            st.gshift[i] = int(self.gshift[i])
            st.kibz[i] = float(self.kibz[i])
        st.time_reversal = self.time_reversal
        st.atom_map = _ptr_i32(self.atom_map) if self.atom_map is not None else ctypes.cast(None, _capi.P_i32)
        st.atom_shift = _ptr_i32(self.atom_shift) if self.atom_shift is not None else ctypes.cast(None, _capi.P_i32)
        st.proj_rot = _ptr_f64(self.proj_rot) if self.proj_rot is not None else ctypes.cast(None, _capi.P_f64)
        self._st = st


class States:
    """One k (or k+q) state set; C and P live on the device, the rest on the host. With `sym` (a SymOp)
    the arrays are those at the operation's kibz and the set used is the one unfolded to `kpt`."""

    def __init__(self, C, miller, eps, f, P=None, proj_off=None, kpt=(0.0, 0.0, 0.0), weight=1.0,
                 device="cuda", dfde=None, sym=None):
        torch = _torch()
        self.device = device
        self.C = _dev_c128(C, device)
        self.miller = _i32(miller).reshape(-1, 3)
        self.eps = _f64(eps)
        self.f = _f64(f)
        self.proj_off = _i32(proj_off if proj_off is not None else [0])
        natoms = len(self.proj_off) - 1
        if P is None or natoms <= 0:
            self.P = torch.zeros((self.C.shape[0], 1), dtype=torch.complex128, device=device)
            self.natoms = 0
        else:
            self.P = _dev_c128(P, device)
            self.natoms = natoms
        self.kpt = _f64(kpt)
        self.weight = float(weight)
        self.dfde = None if dfde is None else _f64(dfde)
        self.sym = sym

    @classmethod
    def from_synth(cls, s, paw, device="cuda"):
        return cls(s.C, s.miller, s.eps, s.f, s.P, paw.offsets, s.kpt, s.weight, device,
                   dfde=getattr(s, "dfde", None))

    def struct(self) -> RpaStates:
        st = RpaStates()
        st.nbands = int(self.C.shape[0])
        st.nQ = int(self.C.shape[1])
        st.miller = _ptr_i32(self.miller)
        st.C = ctypes.c_void_p(self.C.data_ptr())
        st.eps = _ptr_f64(self.eps)
        st.f = _ptr_f64(self.f)
        st.natoms = int(self.natoms)
        st.proj_off = _ptr_i32(self.proj_off)
        st.P = ctypes.c_void_p(self.P.data_ptr())
        for i in range(3):
            st.kpt[i] = float(self.kpt[i])
        st.weight = self.weight
        st.dfde = _ptr_f64(self.dfde) if self.dfde is not None else ctypes.cast(None, _capi.P_f64)
        st.sym = ctypes.pointer(self.sym._st) if self.sym is not None else ctypes.POINTER(_capi.RpaSymop)()
        return st


class QSpec:
    """One q-point: its G-sphere, the PAW table Q(q+G) on the device and, at q -> 0, the nabla table."""

    def __init__(self, q, gmiller, Qpaw=None, optical=False, qhat=(1.0, 0.0, 0.0), Dpaw=None, weight=1.0,
                 device="cuda"):
        self.q = _f64(q)
        self.gmiller = _i32(gmiller).reshape(-1, 3)
        self.optical = bool(optical)
        self.qhat = _f64(qhat)
        self.Qpaw = _dev_c128(Qpaw, device) if Qpaw is not None else None
        self.Dpaw = _f64(Dpaw) if Dpaw is not None else None
        self.weight = float(weight)

    @property
    def NG(self) -> int:
        return int(self.gmiller.shape[0])

    def struct(self) -> RpaQSpec:
        s = RpaQSpec()
        for i in range(3):
            s.q[i] = float(self.q[i])
            s.qhat[i] = float(self.qhat[i])
        s.optical = int(self.optical)
        s.NG = self.NG
        s.gmiller = _ptr_i32(self.gmiller)
        s.Qpaw = ctypes.c_void_p(self.Qpaw.data_ptr()) if self.Qpaw is not None else None
        s.Dpaw = _ptr_f64(self.Dpaw) if self.Dpaw is not None else None
        s.weight = self.weight
        return s


class Freq:
    def __init__(self, omega, weight):
        self.omega = _f64(omega)
        self.weight = _f64(weight)

    @property
    def nw(self) -> int:
        return int(self.omega.size)

    def struct(self) -> RpaFreq:
        fr = RpaFreq()
        fr.nw = self.nw
        fr.omega = _ptr_f64(self.omega)
        fr.weight = _ptr_f64(self.weight)
        return fr


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _prec(p) -> int:
    if isinstance(p, str):
        return PRECISION[p]
    return int(p)


class Context:
    """A library context for one cell and FFT grid on one device."""

    def __init__(self, A, grid, device: int = 0, workspace_cap: int = 0):
        self._L = _capi.lib()
        self.A = _f64(A).reshape(3, 3)
        self.grid = tuple(int(x) for x in grid)
        self.device_index = int(device)
        self.device = f"cuda:{self.device_index}"
        self._cell = _cell(self.A, self.grid)
        h = ctypes.c_void_p()
        _check(self._L.rpa_create(ctypes.byref(h), ctypes.byref(self._cell), self.device_index, int(workspace_cap)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._L.rpa_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- calls -------------------------------------------------------------
    @staticmethod
    def _arrays(sets):
        arr = (RpaStates * len(sets))()
        for i, s in enumerate(sets):
            arr[i] = s.struct()
        return arr

    def pair_density(self, k: States, kq: States, qs: QSpec, pair_n, pair_m, precision="fp64"):
        torch = _torch()
        pn = _i32(pair_n)
        pm = _i32(pair_m)
        out = torch.empty((pn.size, qs.NG), dtype=torch.complex128, device=self.device)
        ks, kqs, q = k.struct(), kq.struct(), qs.struct()
        _check(self._L.rpa_pair_density(self._h, ctypes.byref(ks), ctypes.byref(kqs), ctypes.byref(q), int(pn.size),
                                        _ptr_i32(pn), _ptr_i32(pm), _prec(precision),
                                        ctypes.c_void_p(out.data_ptr()), _stream()), self._h)
        return out

    def chi0(self, ks: Sequence[States], kqs: Sequence[States], qs: QSpec, freq: Freq, precision="fp64"):
        torch = _torch()
        out = torch.empty((freq.nw, qs.NG, qs.NG), dtype=torch.complex128, device=self.device)
        a, b, q, fr = self._arrays(ks), self._arrays(kqs), qs.struct(), freq.struct()
        _check(self._L.rpa_chi0(self._h, a, b, len(ks), ctypes.byref(q), ctypes.byref(fr), _prec(precision),
                                ctypes.c_void_p(out.data_ptr()), _stream()), self._h)
        return out

    def chi0_real(self, ks: Sequence[States], kqs: Sequence[States], qs: QSpec, omega, eta: float,
                  precision="fp64"):
        """chi0(q, w + i eta) at the real frequencies `omega` (rpa_chi0_real); complex128 [nw, NG, NG]."""
        torch = _torch()
        om = _f64(omega)
        out = torch.empty((om.size, qs.NG, qs.NG), dtype=torch.complex128, device=self.device)
        a, b, q = self._arrays(ks), self._arrays(kqs), qs.struct()
        _check(self._L.rpa_chi0_real(self._h, a, b, len(ks), ctypes.byref(q), _ptr_f64(om), int(om.size),
                                     float(eta), _prec(precision), ctypes.c_void_p(out.data_ptr()), _stream()),
               self._h)
        return out

    def chi0_add(self, ks: Sequence[States], kqs: Sequence[States], qs: QSpec, freq: Freq, chi0, precision="fp64"):
        """chi0 += the contribution of these state sets (rpa_chi0_add); chi0 is a device complex128
        [nw, NG, NG] tensor, updated in place and returned."""
        torch = _torch()
        if chi0.dtype != torch.complex128 or not chi0.is_contiguous() or tuple(chi0.shape) != (freq.nw, qs.NG, qs.NG):
            raise ValueError("chi0 must be a contiguous complex128 [nw, NG, NG] device tensor")
        a, b, q, fr = self._arrays(ks), self._arrays(kqs), qs.struct(), freq.struct()
        _check(self._L.rpa_chi0_add(self._h, a, b, len(ks), ctypes.byref(q), ctypes.byref(fr), _prec(precision),
                                    ctypes.c_void_p(chi0.data_ptr()), _stream()), self._h)
        return chi0

    def ec(self, ks: Sequence[States], kqs: Sequence[States], qs: QSpec, freq: Freq, precision="fp64"):
        """E_c(q) (device double [1]) and F(w) (device double [nw]); asynchronous."""
        torch = _torch()
        ec = torch.empty(1, dtype=torch.float64, device=self.device)
        F = torch.empty(freq.nw, dtype=torch.float64, device=self.device)
        a, b, q, fr = self._arrays(ks), self._arrays(kqs), qs.struct(), freq.struct()
        _check(self._L.rpa_ec(self._h, a, b, len(ks), ctypes.byref(q), ctypes.byref(fr), _prec(precision),
                              ctypes.c_void_p(ec.data_ptr()), ctypes.c_void_p(F.data_ptr()), _stream()), self._h)
        return ec, F

    def ec_noalloc(self, ks: Sequence[States], kqs: Sequence[States], qs: QSpec, freq: Freq, precision="fp64",
                   out=None):
        """rpa_ec_noalloc: E_c(q) with every workspace in the library's per-device scratch (no allocation
        by the library). Pass preallocated `out` = (ec [1], F [nw]) device tensors to allocate nothing here
        either; returns (ec, F)."""
        torch = _torch()
        if out is None:
            out = (torch.empty(1, dtype=torch.float64, device=self.device),
                   torch.empty(freq.nw, dtype=torch.float64, device=self.device))
        ec, F = out
        a, b, q, fr = self._arrays(ks), self._arrays(kqs), qs.struct(), freq.struct()
        _check(self._L.rpa_ec_noalloc(self._h, a, b, len(ks), ctypes.byref(q), ctypes.byref(fr), _prec(precision),
                                      ctypes.c_void_p(ec.data_ptr()), ctypes.c_void_p(F.data_ptr()), _stream()),
               self._h)
        return ec, F

    def ec_batched(self, ks: Sequence[States], kqs: Sequence[States], qspecs: Sequence[QSpec], freq: Freq,
                   precision="fp64", use_graph: bool = False, out=None):
        """E_c(q) for every q of qspecs sharing the same state sets; returns (ec [nq + 1], F [nq, nw]) on the
        device, ec[nq] = sum_q w_q E_c(q). With use_graph the launch sequence is captured once and replayed
        while the inputs (host values and device pointers) stay the same; pass the same `out` tensors to replay."""
        torch = _torch()
        nq = len(qspecs)
        if out is None:
            out = (torch.empty(nq + 1, dtype=torch.float64, device=self.device),
                   torch.empty((nq, freq.nw), dtype=torch.float64, device=self.device))
        ec, F = out
        a, b, fr = self._arrays(ks), self._arrays(kqs), freq.struct()
        qarr = (RpaQSpec * nq)()
        for i, q in enumerate(qspecs):
            qarr[i] = q.struct()
        _check(self._L.rpa_ec_batched(self._h, a, b, len(ks), nq, qarr, ctypes.byref(fr), _prec(precision),
                                      ctypes.c_void_p(ec.data_ptr()), ctypes.c_void_p(F.data_ptr()),
                                      int(bool(use_graph)), _stream()), self._h)
        return ec, F

    def ec_batched_sets(self, sets, qspecs: Sequence[QSpec], freq: Freq, precision="fp64", use_graph: bool = False,
                        out=None):
        """E_c(q) for every q of qspecs, q-point j with its own state-set lists sets[j] = (ks, kqs)
        (rpa_ec_batched_sets); returns (ec [nq + 1], F [nq, nw]) on the device, as ec_batched."""
        torch = _torch()
        nq = len(qspecs)
        if len(sets) != nq:
            raise ValueError("one (ks, kqs) pair of lists per q-point")
        if out is None:
            out = (torch.empty(nq + 1, dtype=torch.float64, device=self.device),
                   torch.empty((nq, freq.nw), dtype=torch.float64, device=self.device))
        ec, F = out
        ka = [self._arrays(ks) for ks, _ in sets]
        kqa = [self._arrays(kqs) for _, kqs in sets]
        PS = ctypes.POINTER(RpaStates)
        kp = (PS * nq)(*[ctypes.cast(a, PS) for a in ka])
        kqp = (PS * nq)(*[ctypes.cast(a, PS) for a in kqa])
        nk = (ctypes.c_int * nq)(*[len(ks) for ks, kqs in sets])
        for ks, kqs in sets:
            if len(ks) != len(kqs):
                raise ValueError("k and k+q lists of a q-point differ in length")
        qarr = (RpaQSpec * nq)()
        for i, q in enumerate(qspecs):
            qarr[i] = q.struct()
        fr = freq.struct()
        _check(self._L.rpa_ec_batched_sets(self._h, nq, kp, kqp, nk, qarr, ctypes.byref(fr), _prec(precision),
                                           ctypes.c_void_p(ec.data_ptr()), ctypes.c_void_p(F.data_ptr()),
                                           int(bool(use_graph)), _stream()), self._h)
        return ec, F

    def ec_backward(self, k, kq, qs: QSpec, freq: Freq, dEc=1.0):
        """E_c(q) and its gradient (FP64) for one (k, k+q) pair of state sets, or for lists of pairs
        (Eq. chi0's k sum).

        Returns (ec [1], grads) with grads = dict(eps_k, C_k, P_k[, eps_kq, C_kq, P_kq]) as device tensors
        (a list of such dicts, one per pair, when k and kq are lists); complex gradients are dE/dRe + i
        dE/dIm. With kq[i] the same set as k[i] only the k entries of pair i are returned (both roles
        summed)."""
        torch = _torch()
        dev = self.device
        single = isinstance(k, States)
        ks, kqs = ([k], [kq]) if single else (list(k), list(kq))
        if len(ks) != len(kqs):
            raise ValueError("k and k+q lists differ in length")
        dE = torch.as_tensor(dEc, dtype=torch.float64, device=dev).reshape(1).contiguous()
        ec = torch.empty(1, dtype=torch.float64, device=dev)
        same = [b is a for a, b in zip(ks, kqs)]
        nbk = [int(s.C.shape[0]) for s in ks]
        nbq = [int(s.C.shape[0]) for s in kqs]
        ek = torch.empty(sum(nbk), dtype=torch.float64, device=dev)
        Ck = torch.empty(sum(s.C.numel() for s in ks), dtype=torch.complex128, device=dev)
        Pk = torch.empty(sum(s.P.numel() for s in ks), dtype=torch.complex128, device=dev)
        distinct = not all(same)
        eq = torch.empty(sum(nbq), dtype=torch.float64, device=dev) if distinct else None
        Cq = torch.empty(sum(s.C.numel() for s in kqs), dtype=torch.complex128, device=dev) if distinct else None
        Pq = torch.empty(sum(s.P.numel() for s in kqs), dtype=torch.complex128, device=dev) if distinct else None
        a, b, q, fr = self._arrays(ks), self._arrays(kqs), qs.struct(), freq.struct()

        def ptr(t):
            return ctypes.c_void_p(t.data_ptr()) if t is not None else None
        _check(self._L.rpa_ec_backward(self._h, a, b, len(ks), ctypes.byref(q), ctypes.byref(fr), ptr(dE), ptr(ec),
                                       ptr(ek), ptr(Ck), ptr(Pk), ptr(eq), ptr(Cq), ptr(Pq), _stream()), self._h)
        out = []
        oe = oc = op = qe = qc = qp_ = 0
        for s, t, sm in zip(ks, kqs, same):
            g = {"eps_k": ek[oe:oe + s.C.shape[0]], "C_k": Ck[oc:oc + s.C.numel()].view(s.C.shape),
                 "P_k": Pk[op:op + s.P.numel()].view(s.P.shape)}
            if not sm:
                g.update(eps_kq=eq[qe:qe + t.C.shape[0]], C_kq=Cq[qc:qc + t.C.numel()].view(t.C.shape),
                         P_kq=Pq[qp_:qp_ + t.P.numel()].view(t.P.shape))
            oe += s.C.shape[0]
            oc += s.C.numel()
            op += s.P.numel()
            qe += t.C.shape[0]
            qc += t.C.numel()
            qp_ += t.P.numel()
            out.append(g)
        return ec, (out[0] if single else out)

    def autotune(self, NG: int, npairs: int, nw: int = 16, precision="split_bf16") -> int:
        """Time the split rank-k kernel variants for this shape; returns the recorded variant."""
        _check(self._L.rpa_autotune(self._h, _prec(precision), int(NG), int(npairs), int(nw), _stream()), self._h)
        return self.tune_get(NG, precision)

    def set_pair_path(self, path: int):
        """0: register-resident pair transforms where the grid allows, 1: LDS radix passes."""
        _check(self._L.rpa_set_pair_path(self._h, int(path)), self._h)

    def set_autotune(self, enable: bool):
        """Split precisions: time the rank-k variants for each new sphere-size bucket (default on)."""
        _check(self._L.rpa_set_autotune(self._h, int(bool(enable))), self._h)

    def set_chunk_pairs(self, max_pairs: int):
        """Upper bound on the pairs of one grouped rank-k update (0: set by the workspace budget)."""
        _check(self._L.rpa_set_chunk_pairs(self._h, int(max_pairs)), self._h)

    def set_paw_window(self, max_bands: int):
        """max_bands > 0: the PAW term factorised per band m, at most max_bands bands per pass; 0: the form and
        the passes chosen automatically (rpa_set_paw_window)."""
        _check(self._L.rpa_set_paw_window(self._h, int(max_bands)), self._h)

    def tune_set(self, NG: int, variant: int, precision="split_bf16"):
        _check(self._L.rpa_tune_set(self._h, _prec(precision), int(NG), int(variant)), self._h)

    def tune_get(self, NG: int, precision="split_bf16") -> int:
        v = ctypes.c_int(0)
        _check(self._L.rpa_tune_get(self._h, _prec(precision), int(NG), ctypes.byref(v)), self._h)
        return v.value

    def tune_cache(self, path: str, save: bool):
        _check(self._L.rpa_tune_cache_io(self._h, path.encode(), int(bool(save))), self._h)

    def ec_from_chi0(self, qs: QSpec, freq: Freq, chi0):
        torch = _torch()
        chi0 = chi0.to(device=self.device, dtype=torch.complex128).contiguous()
        ec = torch.empty(1, dtype=torch.float64, device=self.device)
        F = torch.empty(freq.nw, dtype=torch.float64, device=self.device)
        q, fr = qs.struct(), freq.struct()
        _check(self._L.rpa_ec_from_chi0(self._h, ctypes.byref(q), ctypes.byref(fr), ctypes.c_void_p(chi0.data_ptr()),
                                        ctypes.c_void_p(ec.data_ptr()), ctypes.c_void_p(F.data_ptr()), _stream()),
               self._h)
        return ec, F

    STAGES = ("orbitals", "pair_xy", "pair_z_gather", "paw", "optical", "weights", "split_pack", "herk", "cholesky",
              "adjoint_inverse", "adjoint_gemm", "adjoint_pairs", "adjoint_rest")

    def profile(self, enable: bool = True):
        """Start (or stop) per-stage HIP-event timing; totals are cleared."""
        _check(self._L.rpa_profile(self._h, int(bool(enable))), self._h)

    def profile_get(self) -> dict:
        """{stage: (milliseconds, timed launch groups)} since the last profile() call."""
        out = {}
        for st in self.STAGES:
            ms = ctypes.c_double(0)
            n = ctypes.c_longlong(0)
            _check(self._L.rpa_profile_get(self._h, st.encode(), ctypes.byref(ms), ctypes.byref(n)), self._h)
            out[st] = (ms.value, n.value)
        return out

    def check(self):
        """Synchronize and raise RpaError for device-side failures (e.g. a non-positive pivot)."""
        _check(self._L.rpa_check(self._h, _stream()), self._h)


def _ec_function():
    import torch

    class EcFunction(torch.autograd.Function):
        """E_c(q) as a differentiable function of the eigenvalues (float64), the plane-wave coefficients
        (complex128) and the PAW projections (complex128) of one state set used at k and k+q. The forward
        pass and the hand-written adjoint both run in the HIP library; the pair densities are recomputed
        in the adjoint pass."""

        @staticmethod
        def forward(fctx, C, eps, P, context, template, qs, freq):
            st = States(C.detach(), template.miller, eps.detach().cpu().numpy(), template.f, P.detach(),
                        template.proj_off, template.kpt, template.weight, device=context.device)
            fctx.objs = (context, st, qs, freq)
            fctx.eps_device = eps.device
            ec, _ = context.ec([st], [st], qs, freq, "fp64")
            return ec[0].clone()

        @staticmethod
        def backward(fctx, grad):
            context, st, qs, freq = fctx.objs
            _, g = context.ec_backward(st, st, qs, freq, dEc=grad.detach().to(torch.float64))
            return g["C_k"], g["eps_k"].to(fctx.eps_device), g["P_k"], None, None, None, None

    return EcFunction


def ec_autograd(context, C, eps, P, template: "States", qs: "QSpec", freq: "Freq"):
    """Differentiable E_c(q) (see EcFunction): C, P complex128 device tensors, eps float64 tensor."""
    return _ec_function().apply(C, eps, P, context, template, qs, freq)
