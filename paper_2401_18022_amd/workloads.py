"""Seeded synthetic inputs for the ISRS GN numerical-integral engine.

This module only *describes* problems: channel grids, symbol rates, launch
powers, amplifier noise figures and fibre tables, drawn from
``numpy.random.default_rng(seed)``.  It holds none of the model's arithmetic
(no dispersion conversion, no gamma, no power profile, no integral), so the
CPU oracle and the GPU library can both consume it without sharing any of the
method.

The shapes follow the paper's scenarios (Table I: 96 GBaud channels on a
100 GHz grid, one 80 km SSMF span; Table II: per-band amplifier noise
figures; the O-to-U system of Sec. IV spans 1260-1675 nm with 589 channels).
The paper's own fibre data (mode-solver A_eff(lambda), measured Raman gain,
attenuation coefficients) is not available, so the fibre tables are synthetic
stand-ins with the same ranges.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

C_LIGHT = 299792458.0  # m/s, used only to place channels on a wavelength grid

PROFILE_CLOSED_FORM = 0
PROFILE_ODE = 1
FP32 = 0
FP64 = 1

# Table II: amplifier noise figure per band (dB) with ITU band edges (nm).
BAND_EDGES_NM = [("O", 1260.0, 1360.0, 7.0), ("E", 1360.0, 1460.0, 7.0),
                 ("S", 1460.0, 1530.0, 7.0), ("C", 1530.0, 1565.0, 5.0),
                 ("L", 1565.0, 1625.0, 6.0), ("U", 1625.0, 1675.0, 8.0)]


@dataclasses.dataclass
class Fibre:
    """Fibre description in SI units (see include/isrsgn.h, isrsgn_fibre_desc)."""
    span_m: float
    f_ref_hz: float
    beta2: float = 0.0            # s^2/m at f_ref
    beta3: float = 0.0            # s^3/m
    beta4: float = 0.0            # s^4/m
    disp_from_d: int = 0          # 1: derive betas from D, S, Sdot at lambda = c/f_ref
    d_s_per_m2: float = 0.0       # D  [s/m^2]
    s_s_per_m3: float = 0.0       # S  [s/m^3]
    sdot_s_per_m4: float = 0.0    # dS/dlambda [s/m^4]
    tab_f_hz: np.ndarray = None   # table abscissae, ascending
    alpha_per_m: np.ndarray = None
    aeff_m2: np.ndarray = None
    n2_m2_per_w: float = 2.6e-20
    gamma_const_per_w_m: float = 0.0   # >0 overrides the gamma(f) formula
    cr_per_w_m_hz: float = 0.0         # Raman gain slope at aeff_ref
    aeff_ref_m2: float = 80e-12
    raman_cutoff_hz: float = 0.0       # <=0: linear gain over the whole band
    profile: int = PROFILE_CLOSED_FORM
    photon_ratio: int = 0
    n_steps: int = 112
    grid_s: int = 64
    grid_v: int = 64
    s_decades: float = 14.0
    ode_sub: int = 2
    precision: int = FP32
    n_spans: int = 1                   # identical spans, each followed by an amplifier
    rolloff: float = 0.0               # raised-cosine roll-off of the transmit spectra (0: rectangular)
    nli_points: int = 1                # points of the within-channel NLI rule (1: locally white)

    def replace(self, **kw) -> "Fibre":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class Plan:
    """One or more channel plans, concatenated CSR-style (offsets has n_batch+1 entries)."""
    f_hz: np.ndarray
    rs_hz: np.ndarray
    p_w: np.ndarray
    nf_lin: np.ndarray
    offsets: np.ndarray
    snr_trx_lin: float = 0.0

    @property
    def n_batch(self) -> int:
        return len(self.offsets) - 1

    def sub(self, b: int) -> "Plan":
        lo, hi = int(self.offsets[b]), int(self.offsets[b + 1])
        return Plan(self.f_hz[lo:hi].copy(), self.rs_hz[lo:hi].copy(), self.p_w[lo:hi].copy(),
                    self.nf_lin[lo:hi].copy(), np.array([0, hi - lo], dtype=np.int32), self.snr_trx_lin)

    def with_power(self, p_w: np.ndarray) -> "Plan":
        return dataclasses.replace(self, p_w=np.asarray(p_w, dtype=np.float64).copy())


@dataclasses.dataclass
class Workload:
    name: str
    fibre: Fibre
    plan: Plan
    note: str = ""

    def replace_fibre(self, **kw) -> "Workload":
        return dataclasses.replace(self, fibre=self.fibre.replace(**kw))

    def with_plan(self, plan: Plan) -> "Workload":
        return dataclasses.replace(self, plan=plan)


# ----------------------------------------------------------------------------- helpers

def dbm_to_w(dbm):
    return 1e-3 * np.power(10.0, np.asarray(dbm, dtype=np.float64) / 10.0)


def db_to_lin(db):
    return np.power(10.0, np.asarray(db, dtype=np.float64) / 10.0)


def nf_by_band(f_hz: np.ndarray) -> np.ndarray:
    """Noise figure (linear) per channel from Table II, bands split at ITU edges."""
    lam_nm = C_LIGHT / np.asarray(f_hz) * 1e9
    nf_db = np.full(lam_nm.shape, BAND_EDGES_NM[-1][3])
    for _, lo, hi, nf in BAND_EDGES_NM:
        nf_db = np.where((lam_nm >= lo) & (lam_nm < hi), nf, nf_db)
    return db_to_lin(nf_db)


def synthetic_alpha_db_per_km(lam_um: np.ndarray, oh_peak: bool) -> np.ndarray:
    """Synthetic SSMF loss: Rayleigh lambda^-4 term + infrared tail (+ optional OH bump at 1383 nm)."""
    lam_um = np.asarray(lam_um, dtype=np.float64)
    a = 0.93 / lam_um ** 4 + 6e11 * np.exp(-48.0 / lam_um)
    if oh_peak:
        a = a + 0.10 * np.exp(-0.5 * ((lam_um - 1.383) / 0.0085) ** 2)
    return a


def _fibre_table(f_lo: float, f_hi: float, aeff_lam_nm, aeff_um2, oh_peak: bool,
                 spacing_hz: float = 50e9):
    """alpha(f) and A_eff(f) sampled on a uniform frequency grid (linear interpolation in f)."""
    n = int(math.ceil((f_hi - f_lo) / spacing_hz)) + 1
    f = f_lo + spacing_hz * np.arange(n, dtype=np.float64)
    lam_nm = C_LIGHT / f * 1e9
    alpha = synthetic_alpha_db_per_km(lam_nm * 1e-3, oh_peak) * math.log(10.0) / 10.0 / 1e3
    (l0, l1), (a0, a1) = aeff_lam_nm, aeff_um2
    aeff = (a0 + (a1 - a0) * (lam_nm - l0) / (l1 - l0)) * 1e-12
    return f, alpha, aeff


def _aeff_at(lam_nm: float, aeff_lam_nm, aeff_um2) -> float:
    (l0, l1), (a0, a1) = aeff_lam_nm, aeff_um2
    return (a0 + (a1 - a0) * (lam_nm - l0) / (l1 - l0)) * 1e-12


def single_plan(f_hz, rs_hz, p_w, nf_lin, snr_trx_lin=0.0) -> Plan:
    f_hz = np.asarray(f_hz, dtype=np.float64)
    n = len(f_hz)
    return Plan(f_hz, np.broadcast_to(np.asarray(rs_hz, dtype=np.float64), (n,)).copy(),
                np.broadcast_to(np.asarray(p_w, dtype=np.float64), (n,)).copy(),
                np.broadcast_to(np.asarray(nf_lin, dtype=np.float64), (n,)).copy(),
                np.array([0, n], dtype=np.int32), float(snr_trx_lin))


def concat_plans(plans: List[Plan]) -> Plan:
    offs = np.zeros(len(plans) + 1, dtype=np.int32)
    for b, p in enumerate(plans):
        offs[b + 1] = offs[b] + len(p.f_hz)
    return Plan(np.concatenate([p.f_hz for p in plans]), np.concatenate([p.rs_hz for p in plans]),
                np.concatenate([p.p_w for p in plans]), np.concatenate([p.nf_lin for p in plans]),
                offs, plans[0].snr_trx_lin)


# ----------------------------------------------------------------------------- the fibres

F_1550 = C_LIGHT / 1550e-9


def tiny_fibre(**kw) -> Fibre:
    """Constant-parameter SSMF: alpha 0.2 dB/km, beta2 -21.7 ps^2/km, beta3 0.14 ps^3/km,
    gamma 1.3 /W/km, Raman slope 0.028 /W/km/THz (closed-form profile)."""
    fb = Fibre(span_m=80e3, f_ref_hz=F_1550, beta2=-21.7e-27, beta3=0.14e-39, beta4=0.0,
               tab_f_hz=np.array([F_1550]), alpha_per_m=np.array([0.2 * math.log(10.0) / 10.0 / 1e3]),
               aeff_m2=np.array([80e-12]), gamma_const_per_w_m=1.3e-3, cr_per_w_m_hz=0.028 / 1e3 / 1e12,
               aeff_ref_m2=80e-12, raman_cutoff_hz=0.0, profile=PROFILE_CLOSED_FORM, photon_ratio=0,
               n_steps=112, grid_s=64, grid_v=64, s_decades=14.0)
    return fb.replace(**kw)


CL_AEFF = ((1530.0, 1610.0), (75.0, 90.0))
OU_AEFF = ((1260.0, 1675.0), (60.0, 100.0))


def cl_fibre(**kw) -> Fibre:
    """C+L band SSMF: alpha(lambda) without OH, betas at 1550 nm, A_eff 75->90 um^2, n2 2.6e-20."""
    f, a, ae = _fibre_table(183e12, 199e12, *CL_AEFF, oh_peak=False)
    fb = Fibre(span_m=80e3, f_ref_hz=F_1550, beta2=-21.7e-27, beta3=0.14e-39, beta4=-4.79e-52,
               tab_f_hz=f, alpha_per_m=a, aeff_m2=ae, n2_m2_per_w=2.6e-20,
               cr_per_w_m_hz=0.028 / 1e3 / 1e12, aeff_ref_m2=_aeff_at(1550.0, *CL_AEFF),
               raman_cutoff_hz=15e12, profile=PROFILE_ODE, photon_ratio=1,
               n_steps=112, grid_s=256, grid_v=256, s_decades=14.0)
    return fb.replace(**kw)


def ou_fibre(**kw) -> Fibre:
    """O-to-U SSMF: zero dispersion at 1310 nm (G.652 form, S0 = 0.090 ps/nm^2/km), alpha with
    OH bump, A_eff 60->100 um^2, triangular Raman gain to 15 THz with photon-number ratio."""
    s0 = 0.090 * 1e-12 / (1e-18 * 1e3)            # ps/nm^2/km -> s/m^3
    lam0 = 1310e-9
    f, a, ae = _fibre_table(176e12, 241e12, *OU_AEFF, oh_peak=True)
    fb = Fibre(span_m=80e3, f_ref_hz=C_LIGHT / lam0, disp_from_d=1, d_s_per_m2=0.0, s_s_per_m3=s0,
               sdot_s_per_m4=-3.0 * s0 / lam0, tab_f_hz=f, alpha_per_m=a, aeff_m2=ae,
               n2_m2_per_w=2.6e-20, cr_per_w_m_hz=0.028 / 1e3 / 1e12,
               aeff_ref_m2=_aeff_at(1550.0, *OU_AEFF), raman_cutoff_hz=15e12,
               profile=PROFILE_ODE, photon_ratio=1, n_steps=112, grid_s=128, grid_v=128,
               s_decades=14.0)
    return fb.replace(**kw)


# ----------------------------------------------------------------------------- the workloads

def ou_grid() -> np.ndarray:
    """589 channel centres on a 100 GHz grid from 1675 nm (+50 GHz) to ~1260 nm."""
    return C_LIGHT / 1675e-9 + 50e9 + 100e9 * np.arange(589, dtype=np.float64)


def config_tiny(**fib) -> Workload:
    """5 x 96 GBaud at 100 GHz around 1550 nm, 0 dBm flat, one 80 km span, closed-form profile."""
    f = F_1550 + 100e9 * (np.arange(5) - 2.0)
    plan = single_plan(f, 96e9, 1e-3, db_to_lin(5.0))
    return Workload("tiny-5ch", tiny_fibre(**fib), plan, "5 ch, constant fibre, P1, G=64, N_M=112")


def config_cl(seed: int = 2, **fib) -> Workload:
    """95 x 96 GBaud at 100 GHz over 1530-1610 nm, i.i.d. U(-1,+2) dBm launch."""
    rng = np.random.default_rng(seed)
    f = 191.0746e12 + 100e9 * (np.arange(95) - 47.0)
    p = dbm_to_w(rng.uniform(-1.0, 2.0, size=95))
    plan = single_plan(f, 96e9, p, nf_by_band(f))
    return Workload("cl-95ch", cl_fibre(**fib), plan, "95 ch C+L, ODE profile, G=256, N_M=112")


def config_ou(seed: int = 3, **fib) -> Workload:
    """589 x 96 GBaud at 100 GHz over 1260-1675 nm, i.i.d. U(-2,+2) dBm launch."""
    rng = np.random.default_rng(seed)
    f = ou_grid()
    p = dbm_to_w(rng.uniform(-2.0, 2.0, size=589))
    plan = single_plan(f, 96e9, p, nf_by_band(f))
    return Workload("ou-589ch", ou_fibre(**fib), plan, "589 ch O-to-U, ODE profile, G=128, N_M=112")


# Table I: 32 guard channels, 5 nm guard-band gaps.  The paper gives the gap width and, in Table II,
# the occupied channels per band (171/143/88/38/65/52), not where the gaps sit: on this grid the
# gaps [e - 2, e + 3) nm at the interior ITU band edges e (and [1457.5, 1462.5) at 1460 nm) leave
# exactly those counts.
GUARD_GAPS_NM = [(1358.0, 1363.0), (1457.5, 1462.5), (1528.0, 1533.0), (1563.0, 1568.0), (1623.0, 1628.0)]


def guard_mask(f_hz: np.ndarray) -> np.ndarray:
    """True for the channels whose centre lies in one of the guard-band gaps."""
    lam_nm = C_LIGHT / np.asarray(f_hz) * 1e9
    m = np.zeros(len(lam_nm), dtype=bool)
    for lo, hi in GUARD_GAPS_NM:
        m |= (lam_nm >= lo) & (lam_nm < hi)
    return m


def config_ou_guarded(seed: int = 3, **fib) -> Workload:
    """The O-to-U system with the paper's 32 empty guard channels (P = 0, the set A of eq. loss) at the
    band edges; the 557 occupied channels launch i.i.d. U(-2,+2) dBm."""
    rng = np.random.default_rng(seed)
    f = ou_grid()
    p = np.where(guard_mask(f), 0.0, dbm_to_w(rng.uniform(-2.0, 2.0, size=589)))
    plan = single_plan(f, 96e9, p, nf_by_band(f))
    return Workload("ou-589ch-guarded", ou_fibre(**fib), plan, "589 ch O-to-U, 32 guard channels, G=128, N_M=112")


def fd_channels(seed: int = 4, n_ch: int = 589, count: int = 16) -> np.ndarray:
    """The seeded channels on which finite differences check the adjoint gradient."""
    return np.sort(np.random.default_rng(seed).choice(n_ch, count, replace=False))


def config_batch(n_profiles: int = 256, seed: int = 5, n_min: int = 95, n_max: int = 589,
                 **fib) -> Workload:
    """Launch-power profiles (linear tilt +-3 dB + 1 dB sinusoidal ripple, random phase) over
    random contiguous sub-bands of the O-to-U grid with 95..589 channels each."""
    rng = np.random.default_rng(seed)
    grid = ou_grid()
    plans = []
    for _ in range(n_profiles):
        n = int(rng.integers(n_min, n_max + 1))
        start = int(rng.integers(0, len(grid) - n + 1))
        tilt = rng.uniform(-3.0, 3.0)
        cyc = int(rng.integers(1, 6))
        ph0 = rng.uniform(0.0, 2.0 * math.pi)
        k = np.arange(n, dtype=np.float64)
        pdb = tilt * (2.0 * k / (n - 1) - 1.0) + 1.0 * np.sin(2.0 * math.pi * cyc * k / n + ph0)
        f = grid[start:start + n]
        plans.append(single_plan(f, 96e9, dbm_to_w(pdb), nf_by_band(f)))
    fb = ou_fibre(grid_s=64, grid_v=64, n_steps=80).replace(**fib)
    return Workload(f"batch-{n_profiles}", fb, concat_plans(plans),
                    "profiles over uneven O-to-U sub-bands, G=64, N_M=80")


def two_channel(delta_hz: float, p_i_w: float = 1e-3, p_k_w: float = 1e-3, **fib) -> Workload:
    """COI plus one interferer delta_hz away on the tiny fibre (Raman off unless overridden)."""
    f = F_1550 + np.array([0.0, delta_hz])
    order = np.argsort(f)
    p = np.array([p_i_w, p_k_w])[order]
    fib.setdefault("cr_per_w_m_hz", 0.0)
    plan = single_plan(f[order], 96e9, p, db_to_lin(5.0))
    return Workload(f"two-ch-{delta_hz/1e9:.0f}GHz", tiny_fibre(**fib), plan)


def single_channel(p_w: float = 1e-3, **fib) -> Workload:
    fib.setdefault("cr_per_w_m_hz", 0.0)
    plan = single_plan(np.array([F_1550]), 96e9, p_w, db_to_lin(5.0))
    return Workload("single-ch", tiny_fibre(**fib), plan)


def random_small(n_ch: int, seed: int, profile: int = PROFILE_ODE, rolloff: float = 0.0, **fib) -> Workload:
    """A small C+L-like system with ragged spacing/symbol rates for parity tests (with a roll-off,
    the spacing leaves room for the wider raised-cosine spectra)."""
    rng = np.random.default_rng(seed)
    rs = rng.uniform(30e9, 96e9, size=n_ch)
    gaps = rng.uniform(2e9, 40e9, size=n_ch)
    f = np.empty(n_ch)
    f[0] = 190e12
    for c in range(1, n_ch):
        f[c] = f[c - 1] + 0.5 * (1.0 + rolloff) * (rs[c - 1] + rs[c]) + gaps[c]
    p = dbm_to_w(rng.uniform(-2.0, 4.0, size=n_ch))
    plan = Plan(f, rs, p, nf_by_band(f), np.array([0, n_ch], dtype=np.int32))
    if profile == PROFILE_ODE:
        fb = cl_fibre(grid_s=16, grid_v=16, n_steps=24)
    else:
        fb = tiny_fibre(grid_s=16, grid_v=16, n_steps=24)
    return Workload(f"rand-{n_ch}ch-s{seed}", fb.replace(rolloff=rolloff, **fib), plan)
