"""ctypes front-end of the FP64 CPU oracle (oracle/isrsgn_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU-baseline
leg of bench.py.  The product path (paper_2401_18022_amd) never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "isrsgn_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class Problem(C.Structure):
    _fields_ = [
        ("span_m", C.c_double), ("f_ref_hz", C.c_double), ("beta2", C.c_double),
        ("beta3", C.c_double), ("beta4", C.c_double),
        ("n_tab", C.c_int), ("tab_f_hz", _dp), ("tab_alpha_per_m", _dp), ("tab_aeff_m2", _dp),
        ("n2", C.c_double), ("gamma_const", C.c_double), ("cr", C.c_double), ("aeff_ref", C.c_double),
        ("raman_cutoff", C.c_double),
        ("profile", C.c_int), ("photon_ratio", C.c_int),
        ("n_steps", C.c_int), ("grid_s", C.c_int), ("grid_v", C.c_int),
        ("s_decades", C.c_double), ("ode_sub", C.c_int),
        ("n_ch", C.c_int), ("f_hz", _dp), ("rs_hz", _dp), ("p_w", _dp), ("nf_lin", _dp),
        ("snr_trx", C.c_double), ("dp", _dp), ("n_threads", C.c_int), ("unfold", C.c_int),
        ("mode", C.c_int), ("n_spans", C.c_int), ("rolloff", C.c_double), ("nli_points", C.c_int),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (plain C++17, -O2, threads)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = C.POINTER(Problem)
        L.orc_beta_from_dispersion.argtypes = [C.c_double] * 4 + [_dp]
        L.orc_phi.argtypes = [C.c_double] * 6
        L.orc_phi.restype = C.c_double
        L.orc_steps.argtypes = [C.c_double, C.c_double, C.c_int, _dp, _dp, _dp]
        L.orc_profile.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_lnrho.argtypes = [P, C.c_int, _ip, _dp, _dp]
        L.orc_forward.argtypes = [P, C.c_int, _ip, _dp, _dp, _dp, _dp, _dp]
        L.orc_forward_dual.argtypes = [P, C.c_int, _ip] + [_dp] * 8
        L.orc_forward_dualn.argtypes = [P, C.c_int, _dp, C.c_int, _ip] + [_dp] * 8
        L.orc_max_dirs.restype = C.c_int
        L.orc_tiles.argtypes = [P, C.c_int, _ip, _ip, _dp]
        L.orc_psi.argtypes = [P, C.c_int, C.c_int, _dp, _dp, _dp]
        L.orc_paper_quadrants.argtypes = [P, C.c_int, _dp]
        L.orc_gamma.argtypes = [P, _dp]
        L.orc_tiles_at.argtypes = [P, C.c_int, _dp, _ip, _dp]
        L.orc_paper_quadrants_at.argtypes = [P, C.c_double, _dp]
        L.orc_nli_points.argtypes = [P, C.c_int, _dp, _dp]
        L.orc_psd.argtypes = [P, C.c_int, C.c_int, _dp, _dp, _dp]
        L.orc_spectrum_laplace.argtypes = [C.c_double] * 3
        L.orc_spectrum_laplace.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _arr(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def betas(fibre) -> tuple:
    """Dispersion at f_ref: the fibre's betas, or eqs. (d)-(d_curve) applied to D, S, dS/dlambda."""
    if not fibre.disp_from_d:
        return fibre.beta2, fibre.beta3, fibre.beta4
    out = np.zeros(3)
    lib().orc_beta_from_dispersion(299792458.0 / fibre.f_ref_hz, fibre.d_s_per_m2, fibre.s_s_per_m3,
                                   fibre.sdot_s_per_m4, _ptr(out))
    return float(out[0]), float(out[1]), float(out[2])


class Oracle:
    """One channel plan (a single CSR entry) on one fibre."""

    def __init__(self, fibre, plan, n_threads: Optional[int] = None, unfold: int = 0, mode: int = 0):
        assert plan.n_batch == 1, "the oracle takes one plan at a time (Plan.sub)"
        self.fibre, self.plan = fibre, plan
        self._keep = []
        b2, b3, b4 = betas(fibre)
        pb = Problem()
        pb.span_m, pb.f_ref_hz = fibre.span_m, fibre.f_ref_hz
        pb.beta2, pb.beta3, pb.beta4 = b2, b3, b4
        tf, ta, te = _arr(fibre.tab_f_hz), _arr(fibre.alpha_per_m), _arr(fibre.aeff_m2)
        self._keep += [tf, ta, te]
        pb.n_tab, pb.tab_f_hz, pb.tab_alpha_per_m, pb.tab_aeff_m2 = len(tf), _ptr(tf), _ptr(ta), _ptr(te)
        pb.n2, pb.gamma_const, pb.cr = fibre.n2_m2_per_w, fibre.gamma_const_per_w_m, fibre.cr_per_w_m_hz
        pb.aeff_ref, pb.raman_cutoff = fibre.aeff_ref_m2, fibre.raman_cutoff_hz
        pb.profile, pb.photon_ratio = fibre.profile, fibre.photon_ratio
        pb.n_steps, pb.grid_s, pb.grid_v = fibre.n_steps, fibre.grid_s, fibre.grid_v
        pb.s_decades, pb.ode_sub = fibre.s_decades, fibre.ode_sub
        f, r, p, nf = _arr(plan.f_hz), _arr(plan.rs_hz), _arr(plan.p_w), _arr(plan.nf_lin)
        self._keep += [f, r, p, nf]
        pb.n_ch, pb.f_hz, pb.rs_hz, pb.p_w, pb.nf_lin = len(f), _ptr(f), _ptr(r), _ptr(p), _ptr(nf)
        pb.snr_trx = plan.snr_trx_lin
        pb.dp = None
        pb.n_threads = int(n_threads or min(16, os.cpu_count() or 1))
        pb.unfold, pb.mode = unfold, mode
        pb.n_spans = int(getattr(fibre, "n_spans", 1))
        pb.rolloff = float(getattr(fibre, "rolloff", 0.0))
        pb.nli_points = int(getattr(fibre, "nli_points", 1))
        self.pb = pb
        self.n = len(f)

    @property
    def threads(self) -> int:
        return self.pb.n_threads

    def profile(self):
        n, M = self.n, self.fibre.n_steps
        ab = C.c_double()
        edge, zm, dz = np.zeros(M + 1), np.zeros(M), np.zeros(M)
        ell, ellL = np.zeros((M, n)), np.zeros(n)
        rc = lib().orc_profile(C.byref(self.pb), C.byref(ab), _ptr(edge), _ptr(zm), _ptr(dz), _ptr(ell), _ptr(ellL))
        assert rc == 0, "oracle rejected the problem"
        return dict(alpha_bar=ab.value, edge=edge, zm=zm, dz=dz, ell=ell, ell_L=ellL)

    def lnrho(self, m: Sequence[int], F: Sequence[float]) -> np.ndarray:
        m = np.ascontiguousarray(np.asarray(m, dtype=np.int32))
        F = _arr(F)
        out = np.zeros(len(F))
        rc = lib().orc_lnrho(C.byref(self.pb), len(F), m.ctypes.data_as(_ip), _ptr(F), _ptr(out))
        assert rc == 0
        return out

    def forward(self, coi: Optional[Sequence[int]] = None) -> dict:
        coi = np.arange(self.n, dtype=np.int32) if coi is None else np.ascontiguousarray(np.asarray(coi, dtype=np.int32))
        q = len(coi)
        tiles, pnli, eta, snr = np.zeros((q, self.n)), np.zeros(q), np.zeros(q), np.zeros(q)
        thr = C.c_double()
        rc = lib().orc_forward(C.byref(self.pb), q, coi.ctypes.data_as(_ip), _ptr(tiles), _ptr(pnli),
                               _ptr(eta), _ptr(snr), C.byref(thr))
        assert rc == 0, "oracle rejected the problem"
        return dict(coi=coi, tiles=tiles, pnli=pnli, eta=eta, snr=snr, thr=thr.value)

    def forward_dual(self, direction: np.ndarray, coi: Optional[Sequence[int]] = None) -> dict:
        d = _arr(direction)
        assert len(d) == self.n
        coi = np.arange(self.n, dtype=np.int32) if coi is None else np.ascontiguousarray(np.asarray(coi, dtype=np.int32))
        q = len(coi)
        tiles, dtiles = np.zeros((q, self.n)), np.zeros((q, self.n))
        pnli, dpnli, snr, dsnr = np.zeros(q), np.zeros(q), np.zeros(q), np.zeros(q)
        thr, dthr = C.c_double(), C.c_double()
        self.pb.dp = _ptr(d)
        try:
            rc = lib().orc_forward_dual(C.byref(self.pb), q, coi.ctypes.data_as(_ip), _ptr(tiles), _ptr(dtiles),
                                        _ptr(pnli), _ptr(dpnli), _ptr(snr), _ptr(dsnr), C.byref(thr), C.byref(dthr))
        finally:
            self.pb.dp = None
        assert rc == 0
        return dict(coi=coi, tiles=tiles, dtiles=dtiles, pnli=pnli, dpnli=dpnli, snr=snr, dsnr=dsnr,
                    thr=thr.value, dthr=dthr.value)

    def forward_dualn(self, directions: np.ndarray, coi: Optional[Sequence[int]] = None) -> dict:
        """forward_dual along several directions (rows of `directions`, at most 16) in one pass:
        dtiles [q, n, dir], dpnli and dsnr [q, dir], dthr [dir]."""
        d = _arr(np.atleast_2d(directions))
        nd = d.shape[0]
        assert d.shape[1] == self.n and 1 <= nd <= lib().orc_max_dirs()
        K = lib().orc_max_dirs()
        coi = np.arange(self.n, dtype=np.int32) if coi is None else np.ascontiguousarray(np.asarray(coi, dtype=np.int32))
        q = len(coi)
        tiles, dtiles = np.zeros((q, self.n)), np.zeros((q, self.n, K))
        pnli, dpnli, snr, dsnr = np.zeros(q), np.zeros((q, K)), np.zeros(q), np.zeros((q, K))
        thr, dthr = C.c_double(), np.zeros(K)
        rc = lib().orc_forward_dualn(C.byref(self.pb), nd, _ptr(d), q, coi.ctypes.data_as(_ip), _ptr(tiles),
                                     _ptr(dtiles), _ptr(pnli), _ptr(dpnli), _ptr(snr), _ptr(dsnr), C.byref(thr),
                                     _ptr(dthr))
        assert rc == 0
        return dict(coi=coi, tiles=tiles, dtiles=dtiles[:, :, :nd], pnli=pnli, dpnli=dpnli[:, :nd], snr=snr,
                    dsnr=dsnr[:, :nd], thr=thr.value, dthr=dthr[:nd])

    def tiles(self, coi: Sequence[int], intf: Sequence[int]) -> np.ndarray:
        """tile(coi[q], intf[q]) for a list of pairs (the rows of forward() restricted to those pairs)."""
        ci = np.ascontiguousarray(np.asarray(coi, dtype=np.int32))
        ki = np.ascontiguousarray(np.asarray(intf, dtype=np.int32))
        assert ci.shape == ki.shape
        out = np.zeros(len(ci))
        rc = lib().orc_tiles(C.byref(self.pb), len(ci), ci.ctypes.data_as(_ip), ki.ctypes.data_as(_ip), _ptr(out))
        assert rc == 0, "oracle rejected the problem or a pair"
        return out

    def tiles_at(self, f, intf) -> np.ndarray:
        """tile(f[q], intf[q]) at arbitrary NLI frequencies f (no 16/27 gamma^2 factor)."""
        f = _arr(f)
        ki = np.ascontiguousarray(np.asarray(intf, dtype=np.int32))
        assert f.shape == ki.shape
        out = np.zeros(len(f))
        assert lib().orc_tiles_at(C.byref(self.pb), len(f), _ptr(f), ki.ctypes.data_as(_ip), _ptr(out)) == 0
        return out

    def psi(self, i: int, x, y) -> np.ndarray:
        x, y = _arr(x), _arr(y)
        out = np.zeros(len(x))
        assert lib().orc_psi(C.byref(self.pb), i, len(x), _ptr(x), _ptr(y), _ptr(out)) == 0
        return out

    def paper_quadrants(self, i: int) -> np.ndarray:
        out = np.zeros(4)
        assert lib().orc_paper_quadrants(C.byref(self.pb), i, _ptr(out)) == 0
        return out

    def paper_quadrants_at(self, f: float) -> np.ndarray:
        """The paper's quadrants at NLI frequency f (no tiles); their sum times 16/27 gamma(f)^2 is G(f)."""
        out = np.zeros(4)
        assert lib().orc_paper_quadrants_at(C.byref(self.pb), float(f), _ptr(out)) == 0
        return out

    def nli_points(self, c: int):
        """Points (Hz) and weights (Hz) of channel c's within-channel NLI rule."""
        n = self.pb.nli_points
        f, q = np.zeros(n), np.zeros(n)
        assert lib().orc_nli_points(C.byref(self.pb), int(c), _ptr(f), _ptr(q)) == 0
        return f, q

    def psd(self, c: int, F):
        """Transmit PSD of channel c at frequencies F (W/Hz), and gamma at F."""
        F = _arr(F)
        out, g = np.zeros(len(F)), np.zeros(len(F))
        assert lib().orc_psd(C.byref(self.pb), int(c), len(F), _ptr(F), _ptr(out), _ptr(g)) == 0
        return out, g

    def gamma(self) -> np.ndarray:
        out = np.zeros(self.n)
        assert lib().orc_gamma(C.byref(self.pb), _ptr(out)) == 0
        return out


def phi(x, y, w, b2, b3, b4) -> float:
    return lib().orc_phi(float(x), float(y), float(w), float(b2), float(b3), float(b4))


def steps(alpha_bar: float, L: float, n: int):
    edge, zm, dz = np.zeros(n + 1), np.zeros(n), np.zeros(n)
    assert lib().orc_steps(alpha_bar, L, n, _ptr(edge), _ptr(zm), _ptr(dz)) == 0
    return edge, zm, dz


def spectrum_laplace(a: float, R: float, beta: float) -> float:
    return lib().orc_spectrum_laplace(float(a), float(R), float(beta))


def beta_from_dispersion(lam, D, S, Sdot):
    out = np.zeros(3)
    lib().orc_beta_from_dispersion(lam, D, S, Sdot, _ptr(out))
    return out
