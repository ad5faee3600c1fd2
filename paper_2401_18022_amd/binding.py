"""ctypes binding of libisrsgn.so (C ABI in include/isrsgn.h).

Argument marshalling only: every step of the model runs in the library's HIP kernels.
Device buffers are torch tensors (float64, contiguous, on the current HIP device) and
work is enqueued on torch's current stream.  There is no CPU fallback: if the library
is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import workloads as W

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libisrsgn.so")

ISRSGN_OK, ISRSGN_EINVAL, ISRSGN_ENOMEM, ISRSGN_EDEVICE, ISRSGN_EUNSUPPORTED = 0, -1, -2, -3, -4
ERRORS = {ISRSGN_EINVAL: "EINVAL", ISRSGN_ENOMEM: "ENOMEM", ISRSGN_EDEVICE: "EDEVICE",
          ISRSGN_EUNSUPPORTED: "EUNSUPPORTED"}
SYMBOLS = ["isrsgn_setup_fibre", "isrsgn_eta", "isrsgn_snr", "isrsgn_snr_grad", "isrsgn_snr_noalloc", "isrsgn_profile",
           "isrsgn_set_graph", "isrsgn_set_checks", "isrsgn_set_timing", "isrsgn_stage_times", "isrsgn_work_counts",
           "isrsgn_destroy", "isrsgn_last_error"]

_dp = C.POINTER(C.c_double)


class FibreDesc(C.Structure):
    _fields_ = [
        ("span_m", C.c_double), ("f_ref_hz", C.c_double),
        ("beta2", C.c_double), ("beta3", C.c_double), ("beta4", C.c_double),
        ("disp_from_d", C.c_int), ("d_s_per_m2", C.c_double), ("s_s_per_m3", C.c_double),
        ("sdot_s_per_m4", C.c_double),
        ("n_tab", C.c_int), ("tab_f_hz", _dp), ("alpha_per_m", _dp), ("aeff_m2", _dp),
        ("n2_m2_per_w", C.c_double), ("gamma_const_per_w_m", C.c_double),
        ("cr_per_w_m_hz", C.c_double), ("aeff_ref_m2", C.c_double), ("raman_cutoff_hz", C.c_double),
        ("profile", C.c_int), ("photon_ratio", C.c_int), ("n_steps", C.c_int),
        ("grid_s", C.c_int), ("grid_v", C.c_int), ("s_decades", C.c_double), ("ode_sub", C.c_int),
        ("precision", C.c_int), ("n_spans", C.c_int), ("rolloff", C.c_double), ("nli_points", C.c_int),
    ]


class PlanDesc(C.Structure):
    _fields_ = [("n_batch", C.c_int), ("ch_offsets", C.POINTER(C.c_int)), ("f_hz", _dp), ("rs_hz", _dp)]


class IsrsgnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libisrsgn.so (built in-tree by build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2401_18022_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.isrsgn_setup_fibre.argtypes = [C.POINTER(FibreDesc), C.POINTER(vp)]
        L.isrsgn_eta.argtypes = [vp, C.POINTER(PlanDesc), vp, vp, vp, vp, vp]
        L.isrsgn_snr.argtypes = [vp, C.POINTER(PlanDesc), vp, vp, C.c_double, vp, vp, vp]
        L.isrsgn_snr_grad.argtypes = [vp, C.POINTER(PlanDesc), vp, vp, C.c_double, vp, vp, vp, vp]
        L.isrsgn_snr_noalloc.argtypes = [vp, C.POINTER(PlanDesc), vp, vp, C.c_double, vp, vp, vp]
        L.isrsgn_profile.argtypes = [vp, C.POINTER(PlanDesc), vp, vp, vp, vp, vp, vp]
        L.isrsgn_set_timing.argtypes = [vp, C.c_int]
        L.isrsgn_set_graph.argtypes = [vp, C.c_int]
        L.isrsgn_set_checks.argtypes = [vp, C.c_int]
        L.isrsgn_stage_times.argtypes = [vp, _dp, C.c_int]
        L.isrsgn_work_counts.argtypes = [vp, _dp, C.c_int]
        L.isrsgn_destroy.argtypes = [vp]
        L.isrsgn_destroy.restype = None
        L.isrsgn_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != ISRSGN_OK:
        raise IsrsgnError(rc, lib().isrsgn_last_error().decode())


def _c64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def make_desc(fibre: W.Fibre, precision: Optional[int] = None):
    """isrsgn_fibre_desc for a workloads.Fibre (returns the struct and the arrays it points into)."""
    keep = [_c64(fibre.tab_f_hz), _c64(fibre.alpha_per_m), _c64(fibre.aeff_m2)]
    d = FibreDesc()
    d.span_m, d.f_ref_hz = fibre.span_m, fibre.f_ref_hz
    d.beta2, d.beta3, d.beta4 = fibre.beta2, fibre.beta3, fibre.beta4
    d.disp_from_d = int(fibre.disp_from_d)
    d.d_s_per_m2, d.s_s_per_m3, d.sdot_s_per_m4 = fibre.d_s_per_m2, fibre.s_s_per_m3, fibre.sdot_s_per_m4
    d.n_tab = len(keep[0])
    d.tab_f_hz, d.alpha_per_m, d.aeff_m2 = (k.ctypes.data_as(_dp) for k in keep)
    d.n2_m2_per_w, d.gamma_const_per_w_m = fibre.n2_m2_per_w, fibre.gamma_const_per_w_m
    d.cr_per_w_m_hz, d.aeff_ref_m2, d.raman_cutoff_hz = fibre.cr_per_w_m_hz, fibre.aeff_ref_m2, fibre.raman_cutoff_hz
    d.profile, d.photon_ratio = fibre.profile, int(fibre.photon_ratio)
    d.n_steps, d.grid_s, d.grid_v = fibre.n_steps, fibre.grid_s, fibre.grid_v
    d.s_decades, d.ode_sub = fibre.s_decades, fibre.ode_sub
    d.precision = fibre.precision if precision is None else precision
    d.n_spans = fibre.n_spans
    d.rolloff = float(getattr(fibre, "rolloff", 0.0))
    d.nli_points = int(getattr(fibre, "nli_points", 1))
    return d, keep


class PlanArgs:
    """Host-side isrsgn_plan for a workloads.Plan (keeps its arrays alive)."""

    def __init__(self, plan: W.Plan):
        self.off = np.ascontiguousarray(np.asarray(plan.offsets, dtype=np.int32))
        self.f = _c64(plan.f_hz)
        self.rs = _c64(plan.rs_hz)
        self.c = PlanDesc(len(self.off) - 1, self.off.ctypes.data_as(C.POINTER(C.c_int)),
                          self.f.ctypes.data_as(_dp), self.rs.ctypes.data_as(_dp))
        self.n_batch = len(self.off) - 1
        self.n_total = int(self.off[-1])
        self.n_tiles = int(np.sum(np.diff(self.off).astype(np.int64) ** 2))


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("isrsgn needs a GPU (torch.cuda.is_available() is False)")
    return torch


def _dev(t, n, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t, dtype=np.float64), device="cuda")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor with {n} elements")
    return t


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


class Engine:
    """One isrsgn_fibre handle (fibre, discretisation and precision form)."""

    def __init__(self, fibre: W.Fibre, precision: Optional[int] = None):
        _torch()
        d, keep = make_desc(fibre, precision)
        h = C.c_void_p()
        _check(lib().isrsgn_setup_fibre(C.byref(d), C.byref(h)))
        self.h = h
        self.fibre = fibre
        self.precision = d.precision
        self._plans = {}

    def close(self):
        if getattr(self, "h", None):
            lib().isrsgn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _plan(self, plan: W.Plan) -> PlanArgs:
        key = id(plan)
        pa = self._plans.get(key)
        if pa is None or pa.n_total != len(plan.f_hz):
            pa = PlanArgs(plan)
            self._plans = {key: pa}
        return pa

    def eta(self, plan: W.Plan, P, tiles: bool = False):
        torch = _torch()
        pa = self._plan(plan)
        P = _dev(P, pa.n_total, "P")
        eta = torch.empty(pa.n_total, dtype=torch.float64, device="cuda")
        pnli = torch.empty_like(eta)
        tl = torch.empty(pa.n_tiles, dtype=torch.float64, device="cuda") if tiles else None
        _check(lib().isrsgn_eta(self.h, C.byref(pa.c), _ptr(P), _ptr(eta), _ptr(pnli), _ptr(tl), _stream()))
        return eta, pnli, tl

    def snr(self, plan: W.Plan, P, nf, snr_trx_lin: float = 0.0):
        torch = _torch()
        pa = self._plan(plan)
        P, nf = _dev(P, pa.n_total, "P"), _dev(nf, pa.n_total, "nf")
        snr = torch.empty(pa.n_total, dtype=torch.float64, device="cuda")
        thr = torch.empty(pa.n_batch, dtype=torch.float64, device="cuda")
        _check(lib().isrsgn_snr(self.h, C.byref(pa.c), _ptr(P), _ptr(nf), float(snr_trx_lin), _ptr(snr), _ptr(thr),
                                _stream()))
        return snr, thr

    def snr_grad(self, plan: W.Plan, P, nf, snr_trx_lin: float = 0.0):
        torch = _torch()
        pa = self._plan(plan)
        P, nf = _dev(P, pa.n_total, "P"), _dev(nf, pa.n_total, "nf")
        snr = torch.empty(pa.n_total, dtype=torch.float64, device="cuda")
        thr = torch.empty(pa.n_batch, dtype=torch.float64, device="cuda")
        g = torch.empty(pa.n_total, dtype=torch.float64, device="cuda")
        _check(lib().isrsgn_snr_grad(self.h, C.byref(pa.c), _ptr(P), _ptr(nf), float(snr_trx_lin), _ptr(snr),
                                     _ptr(thr), _ptr(g), _stream()))
        return snr, thr, g

    def snr_noalloc(self, plan: W.Plan, P, nf, snr_trx_lin: float = 0.0, out=None):
        """isrsgn_snr_noalloc: the SNR call on the library's static device scratch (no allocation
        inside the library); `out` = (snr, thr) tensors to write into, else new ones."""
        torch = _torch()
        pa = self._plan(plan)
        P, nf = _dev(P, pa.n_total, "P"), _dev(nf, pa.n_total, "nf")
        if out is None:
            out = (torch.empty(pa.n_total, dtype=torch.float64, device="cuda"),
                   torch.empty(pa.n_batch, dtype=torch.float64, device="cuda"))
        snr, thr = _dev(out[0], pa.n_total, "snr"), _dev(out[1], pa.n_batch, "thr")
        _check(lib().isrsgn_snr_noalloc(self.h, C.byref(pa.c), _ptr(P), _ptr(nf), float(snr_trx_lin), _ptr(snr),
                                        _ptr(thr), _stream()))
        return snr, thr

    def profile(self, plan: W.Plan, P):
        torch = _torch()
        pa = self._plan(plan)
        P = _dev(P, pa.n_total, "P")
        M = self.fibre.n_steps
        zm = torch.empty(pa.n_batch * M, dtype=torch.float64, device="cuda")
        dz = torch.empty_like(zm)
        ell = torch.empty(pa.n_total * M, dtype=torch.float64, device="cuda")
        ellL = torch.empty(pa.n_total, dtype=torch.float64, device="cuda")
        _check(lib().isrsgn_profile(self.h, C.byref(pa.c), _ptr(P), _ptr(zm), _ptr(dz), _ptr(ell), _ptr(ellL),
                                    _stream()))
        return zm, dz, ell, ellL

    def set_graph(self, on: bool = True):
        _check(lib().isrsgn_set_graph(self.h, int(on)))

    def set_checks(self, on: bool = True):
        _check(lib().isrsgn_set_checks(self.h, int(on)))

    def set_timing(self, on: bool = True):
        _check(lib().isrsgn_set_timing(self.h, int(on)))

    def stage_times(self) -> dict:
        out = np.zeros(6)
        _check(lib().isrsgn_stage_times(self.h, out.ctypes.data_as(_dp), 6))
        return dict(zip(["profile", "tiles", "reduce", "adjoint_tiles", "adjoint_rest", "total"], out.tolist()))

    def work_counts(self) -> dict:
        out = np.zeros(7)
        _check(lib().isrsgn_work_counts(self.h, out.ctypes.data_as(_dp), 7))
        return dict(nodes=out[0], node_steps=out[1], tiles=out[2], variant=int(out[3]), grad_batches=int(out[4]),
                    lowrank_plans=int(out[5]), lowrank_terms=int(out[6]))


def tiles_to_blocks(tiles, plan: W.Plan):
    """Split the concatenated tile vector into per-plan N_b x N_b arrays (host numpy)."""
    t = tiles.cpu().numpy() if hasattr(tiles, "cpu") else np.asarray(tiles)
    out, pos = [], 0
    for b in range(plan.n_batch):
        n = int(plan.offsets[b + 1] - plan.offsets[b])
        out.append(t[pos:pos + n * n].reshape(n, n))
        pos += n * n
    return out
