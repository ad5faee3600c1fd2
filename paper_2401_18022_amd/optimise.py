"""Launch-power optimisation with the adjoint gradient (Sec. IV).

* ``gradient_ascent``: per-channel powers in dBm, Adam on the throughput, projected to
  [-5, +5] dBm after every step.
* ``segment_lbfgsb``: the paper's segment scheme -- per band N_B = round(B_band / B_p)
  edges (B_p = 750 GHz in the O band, 1.5 THz elsewhere, at least two per band), equally
  spaced over the band's channels, in dBm, channel powers linearly interpolated between
  edges, L-BFGS-B with bounds +-5 dBm and stop at max|grad L| <= 0.01 -- but with the
  exact adjoint gradient instead of finite differences.

    python -m paper_2401_18022_amd.optimise [--grid 64] [--steps 50] [--lbfgsb | --two-stage] [--guards]

--guards runs the O-to-U plan with the paper's 32 empty guard channels (Table I), whose occupied
channels per band give Table II's 23/10/6/3/4/3 segments.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import workloads as W

LN10_10 = math.log(10.0) / 10.0


def band_of(f_hz: np.ndarray) -> np.ndarray:
    lam = W.C_LIGHT / np.asarray(f_hz) * 1e9
    out = np.full(len(lam), len(W.BAND_EDGES_NM) - 1)
    for b, (_, lo, hi, _) in enumerate(W.BAND_EDGES_NM):
        out[(lam >= lo) & (lam < hi)] = b
    return out


def segment_counts(channels_per_band, spacing_hz: float = 100e9):
    """N_B = round(B_band / B_p) with B_band = channels x spacing, B_p = 0.75 THz (O) / 1.5 THz."""
    out = []
    for b, n in enumerate(channels_per_band):
        bp = 0.75e12 if b == 0 else 1.5e12
        out.append(max(2, int(math.floor(n * spacing_hz / bp + 0.5))) if n > 0 else 0)
    return out


def segment_matrix(f_hz: np.ndarray, spacing_hz: float = 100e9, occupied=None):
    """Interpolation matrix A (n_ch x n_edges): channel dBm = A @ edge dBm (linear in frequency
    between equally spaced edges of each band).  Only occupied channels (default: all) count
    towards a band's width and get a row; the rows of empty (guard) channels are zero."""
    bands = band_of(f_hz)
    occ = np.ones(len(f_hz), dtype=bool) if occupied is None else np.asarray(occupied, dtype=bool)
    counts = segment_counts([int(np.sum((bands == b) & occ)) for b in range(len(W.BAND_EDGES_NM))], spacing_hz)
    cols, col0 = [], 0
    A = np.zeros((len(f_hz), sum(counts)))
    for b, ne in enumerate(counts):
        idx = np.nonzero((bands == b) & occ)[0]
        if len(idx) == 0:
            continue
        fe = np.linspace(f_hz[idx[0]], f_hz[idx[-1]], ne)
        for c in idx:
            j = min(max(int(np.searchsorted(fe, f_hz[c], side="right")) - 1, 0), ne - 2)
            t = (f_hz[c] - fe[j]) / (fe[j + 1] - fe[j])
            A[c, col0 + j] += 1.0 - t
            A[c, col0 + j + 1] += t
        cols.append((col0, ne))
        col0 += ne
    return A, counts


def gradient_ascent(engine, plan, p_dbm0, steps=50, lr_db=0.05, lo=-5.0, hi=5.0, progress=None):
    from .autograd import optimise_launch_power
    return optimise_launch_power(engine, plan, p_dbm0, steps=steps, lr_db=lr_db, lo_dbm=lo, hi_dbm=hi,
                                 progress=progress)


def fd_check(plan, fibre, channels, rel_step=10 ** 1e-4 - 1):
    """dT/dP_k of the FP32 and FP64 adjoints against central differences of the FP64 form at
    P_k (1 +- rel_step) (a 1e-3 dB change moves T by ~1e-7, below FP32 resolution)."""
    import torch
    from . import binding as B
    e32, e64 = B.Engine(fibre, W.FP32), B.Engine(fibre, W.FP64)
    P0 = torch.tensor(plan.p_w, dtype=torch.float64, device="cuda")
    nf = torch.tensor(plan.nf_lin, dtype=torch.float64, device="cuda")
    g32 = e32.snr_grad(plan, P0, nf)[2].cpu().numpy()
    g64 = e64.snr_grad(plan, P0, nf)[2].cpu().numpy()
    rows = []
    for j, c in enumerate(channels):
        Pp, Pm = P0.clone(), P0.clone()
        Pp[c] *= 1 + rel_step
        Pm[c] *= 1 - rel_step
        tp = e64.snr(plan, Pp, nf)[1].sum().item()
        tm = e64.snr(plan, Pm, nf)[1].sum().item()
        fd = (tp - tm) / (2 * rel_step * plan.p_w[c])
        rows.append(dict(channel=int(c), fd=fd, adj64=float(g64[c]), adj32=float(g32[c]),
                         rel64=abs(g64[c] - fd) / abs(fd), rel32=abs(g32[c] - fd) / abs(fd)))
        print(f"[fd] {j + 1}/{len(channels)} channel {c}: rel err FP64 {rows[-1]['rel64']:.2e} "
              f"FP32 {rows[-1]['rel32']:.2e}", file=sys.stderr, flush=True)
    return rows


def segment_powers(A, occupied, x):
    """Channel powers (W) from segment edges x (dBm): interpolated in dBm, 0 W on empty channels."""
    return np.where(occupied, 1e-3 * np.power(10.0, (A @ x) / 10.0), 0.0)


def segment_objective(engine, plan, A, occupied, hist=None, progress=None):
    """fg(x) -> (L, dL/dx): the cost of eq. (loss), L = -sum over occupied channels of
    log2(1 + SNR_i), and its gradient with respect to the segment edges in dBm, through the
    adjoint: dL/dx = A^T (dL/dP_k P_k ln10/10)."""
    import torch
    nf = torch.tensor(plan.nf_lin, dtype=torch.float64, device="cuda")
    bch = float(plan.rs_hz[0])
    hist = [] if hist is None else hist

    def fg(x):
        if progress:
            progress(len(hist), hist[-1] if hist else float("nan"))
        P = segment_powers(A, occupied, np.asarray(x, dtype=np.float64))
        snr, thr, g = engine.snr_grad(plan, torch.tensor(P, dtype=torch.float64, device="cuda"), nf)
        T = float(thr.sum().item())
        gP = g.cpu().numpy()
        loss = -T / (2.0 * bch)
        dloss_dp = -(gP * P * LN10_10) / (2.0 * bch)
        hist.append(T)
        return loss, A.T @ dloss_dp

    return fg


def segment_lbfgsb(engine, plan, x0_dbm=None, lo=-5.0, hi=5.0, pgtol=0.01, maxiter=200, progress=None):
    """Minimise L = -sum log2(1 + SNR_i) (eq. loss) over segment edges in dBm.  Channels launched
    at P = 0 are empty (guard) channels: they stay empty and do not count towards the segments."""
    from scipy.optimize import minimize
    occupied = np.asarray(plan.p_w) > 0
    A, counts = segment_matrix(plan.f_hz, occupied=occupied)
    hist = []
    fg = segment_objective(engine, plan, A, occupied, hist, progress)
    x0 = np.zeros(A.shape[1]) if x0_dbm is None else np.asarray(x0_dbm, dtype=np.float64)
    res = minimize(fg, x0, jac=True, method="L-BFGS-B", bounds=[(lo, hi)] * A.shape[1],
                   options=dict(gtol=pgtol, maxiter=maxiter))
    p_dbm = np.where(occupied, A @ res.x, -np.inf)
    return res.x, p_dbm, hist, res, counts


def two_stage(fibre, plan, coarse: dict, fine: dict, progress=None, maxiter=200):
    """The paper's schedule (Sec. IV): segment L-BFGS-B at coarse integration parameters from a
    0 dBm start, then again at fine parameters from the coarse optimum.  ``coarse`` and ``fine``
    are fibre overrides (grid_s, grid_v, n_steps).  Returns one dict per stage."""
    from . import binding as B
    stages, x0 = [], None
    for name, kw in (("coarse", coarse), ("fine", fine)):
        eng = B.Engine(fibre.replace(**kw), W.FP32)
        t0 = time.perf_counter()
        x, p_dbm, hist, res, counts = segment_lbfgsb(eng, plan, x0_dbm=x0, progress=progress, maxiter=maxiter)
        stages.append(dict(stage=name, params=dict(kw), seconds=time.perf_counter() - t0, evaluations=len(hist),
                           converged=bool(res.success), throughput_tbps=[hist[0] / 1e12, max(hist) / 1e12],
                           edges_dbm=x, p_dbm=p_dbm, counts=counts))
        eng.close()
        x0 = x
    return stages


def main(argv=None):
    import torch
    from . import binding as B
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=int, default=64)
    ap.add_argument("--n-steps", type=int, default=112)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--lbfgsb", action="store_true")
    ap.add_argument("--two-stage", action="store_true",
                    help="segment L-BFGS-B at G=64, N_M=80 (1 step/km), then at --grid/--n-steps from its optimum")
    ap.add_argument("--no-fp64-check", action="store_true", help="skip the FP64-form re-check")
    ap.add_argument("--fd-check", type=int, default=0, metavar="N",
                    help="only compare the adjoints with FP64 central differences on N seeded channels")
    ap.add_argument("--guards", action="store_true", help="the O-to-U plan with 32 empty guard channels")
    args = ap.parse_args(argv)
    make = W.config_ou_guarded if args.guards else W.config_ou
    wl = make(grid_s=args.grid, grid_v=args.grid, n_steps=args.n_steps)
    out = {"workload": f"O-to-U 589 ch{' (32 guard)' if args.guards else ''}, G={args.grid}, N_M={args.n_steps}, "
                       "FP32 form"}

    def note(k, thr):
        print(f"[optimise] evaluation {k}: throughput {thr / 1e12:.4f} Tb/s", file=sys.stderr, flush=True)

    if args.fd_check:
        t0 = time.perf_counter()
        rows = fd_check(wl.plan, wl.fibre, W.fd_channels()[:args.fd_check])
        out.update(method="adjoint vs FP64 central differences (P x 10^(+-1e-4))", channels=rows,
                   max_rel_fp64=max(r["rel64"] for r in rows), max_rel_fp32=max(r["rel32"] for r in rows),
                   seconds=time.perf_counter() - t0)
        print(json.dumps(out), flush=True)
        return
    if args.two_stage:
        fine = dict(grid_s=args.grid, grid_v=args.grid, n_steps=args.n_steps)
        st = two_stage(wl.fibre, wl.plan, dict(grid_s=64, grid_v=64, n_steps=80), fine, progress=note)
        out = {"workload": "O-to-U 589 ch, FP32 form", "method": "segment L-BFGS-B, coarse then fine",
               "stages": [{k: v for k, v in d.items() if k not in ("edges_dbm", "p_dbm")} for d in st],
               "seconds": sum(d["seconds"] for d in st)}
        plan = wl.plan.with_power(1e-3 * np.power(10.0, np.asarray(st[-1]["p_dbm"]) / 10.0))
        P = torch.tensor(plan.p_w, dtype=torch.float64, device="cuda")
        nf = torch.tensor(plan.nf_lin, dtype=torch.float64, device="cuda")
        if not args.no_fp64_check:
            e64 = B.Engine(wl.fibre.replace(**fine), W.FP64)
            out["fp64_recheck_tbps"] = e64.snr(plan, P, nf)[1].item() / 1e12
        print(json.dumps(out), flush=True)
        return
    eng = B.Engine(wl.fibre, W.FP32)
    p0 = np.where(wl.plan.p_w > 0, 10 * np.log10(np.maximum(wl.plan.p_w, 1e-300) / 1e-3), -np.inf)
    t0 = time.perf_counter()
    if args.lbfgsb:
        x, p_dbm, hist, res, counts = segment_lbfgsb(eng, wl.plan, progress=note)
        out.update(method="segment L-BFGS-B", edges=int(len(x)), segments_per_band=counts,
                   evaluations=len(hist), converged=bool(res.success), message=str(res.message))
    else:
        p_dbm, hist = gradient_ascent(eng, wl.plan, p0, steps=args.steps, progress=note)
        out.update(method="Adam gradient ascent in dBm", steps=args.steps)
    out["seconds"] = time.perf_counter() - t0
    out["throughput_tbps"] = {"initial": hist[0] / 1e12, "final": hist[-1] / 1e12}
    plan = wl.plan.with_power(1e-3 * np.power(10.0, np.asarray(p_dbm) / 10.0))
    P = torch.tensor(plan.p_w, dtype=torch.float64, device="cuda")
    nf = torch.tensor(plan.nf_lin, dtype=torch.float64, device="cuda")
    snr32, thr32 = eng.snr(plan, P, nf)
    out["throughput_tbps"]["final_fp32"] = thr32.item() / 1e12
    if not args.no_fp64_check:  # the optimised powers re-evaluated with the FP64 form
        e64 = B.Engine(wl.fibre, W.FP64)
        snr64, thr64 = e64.snr(plan, P, nf)
        occ = plan.p_w > 0
        d = 10 * np.log10(snr32.cpu().numpy()[occ] / snr64.cpu().numpy()[occ])
        out["fp64_recheck"] = {"throughput_tbps": thr64.item() / 1e12, "max_abs_dsnr_db": float(np.abs(d).max())}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
