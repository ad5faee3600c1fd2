"""Launch-power optimisation at the O-to-U size (Sec. IV): the segment-edge gradient against central
differences, and the optimisers' end points re-checked with the FP64 oracle.

The re-check feeds the optimisers' final launch powers to the oracle -- the check the workload
asks for: the SNR the optimiser reports at its own optimum, against the oracle's at those powers,
on the 16 seeded channels.  It is not one of the seeded-input parity pins.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_18022_amd import binding as B
from paper_2401_18022_amd import optimise as OPT
from paper_2401_18022_amd import workloads as W

pytestmark = pytest.mark.gpu


def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need an MI355X"
    return t


def dev(a):
    t = torch()
    return t.tensor(np.asarray(a, dtype=np.float64), dtype=t.float64, device="cuda")


def test_segment_edge_gradient_matches_central_differences():
    """dL/dx of the segment scheme (A^T through the adjoint) along three edges -- first O-band, a
    C-band and the last U-band edge -- against central differences of the FP64 form (+-3e-3 dB),
    on the guarded O-to-U plan at G=32, N_M=40 with seeded edge powers."""
    wl = W.config_ou_guarded(grid_s=32, grid_v=32, n_steps=40)
    occ = wl.plan.p_w > 0
    A, counts = OPT.segment_matrix(wl.plan.f_hz, occupied=occ)
    x0 = np.random.default_rng(12).uniform(-1.0, 2.0, A.shape[1])
    edges = [0, sum(counts[:3]) + 1, A.shape[1] - 1]
    e64 = B.Engine(wl.fibre, W.FP64)
    e32 = B.Engine(wl.fibre, W.FP32)
    f64 = OPT.segment_objective(e64, wl.plan, A, occ)
    f32 = OPT.segment_objective(e32, wl.plan, A, occ)
    _, g64 = f64(x0)
    _, g32 = f32(x0)
    h = 3e-3
    for j in edges:
        d = np.zeros_like(x0)
        d[j] = h
        fd = (f64(x0 + d)[0] - f64(x0 - d)[0]) / (2 * h)
        r64, r32 = abs(g64[j] / fd - 1), abs(g32[j] / fd - 1)
        print(f"[segment] edge {j}: dL/dx {fd:.6e}; rel error FP64 {r64:.1e}, FP32 {r32:.1e}", flush=True)
        assert r64 <= 1e-5 and r32 <= 1e-4


def oracle_recheck(wl, p_dbm, label):
    """GPU FP32 and FP64 SNR at the optimised powers against the oracle's on the 16 seeded channels."""
    t = torch()
    plan = wl.plan.with_power(np.where(np.isfinite(p_dbm), 1e-3 * np.power(10.0, np.asarray(p_dbm) / 10.0), 0.0))
    coi = [int(c) for c in W.fd_channels() if plan.p_w[c] > 0]
    P, nf = dev(plan.p_w), dev(plan.nf_lin)
    s32 = B.Engine(wl.fibre, W.FP32).snr(plan, P, nf)[0]
    s64 = B.Engine(wl.fibre, W.FP64).snr(plan, P, nf)[0]
    t.cuda.synchronize()
    print(f"[optimise] {label}: oracle re-check of {len(coi)} seeded channels", flush=True)
    r = O.Oracle(wl.fibre, plan).forward(coi)
    d32 = np.abs(10 * np.log10(s32.cpu().numpy()[coi] / r["snr"]))
    d64 = np.abs(10 * np.log10(s64.cpu().numpy()[coi] / r["snr"]))
    print(f"[optimise] {label}: max |dSNR| vs oracle FP32 {d32.max():.2e} dB, FP64 {d64.max():.2e} dB", flush=True)
    assert d32.max() <= 0.01 and d32.max() <= 1e-5
    assert d64.max() <= 1e-10


@pytest.mark.timeout(400)
def test_adam_50_steps_at_589_channels_rechecked_by_oracle():
    """50 Adam steps in dBm (lr 0.05 dB, bounds +-5 dBm) on the O-to-U system at G=64, N_M=112."""
    from paper_2401_18022_amd.autograd import optimise_launch_power
    wl = W.config_ou(grid_s=64, grid_v=64, n_steps=112)
    eng = B.Engine(wl.fibre, W.FP32)
    p0 = 10 * np.log10(wl.plan.p_w / 1e-3)
    print("[optimise] Adam, 50 steps", flush=True)
    p, hist = optimise_launch_power(eng, wl.plan, p0, steps=50, lr_db=0.05)
    print(f"[optimise] Adam: {hist[0] / 1e12:.3f} -> {hist[-1] / 1e12:.3f} Tb/s", flush=True)
    assert hist[-1] > hist[0] and np.all(np.abs(p) <= 5.0)
    oracle_recheck(wl, p, "Adam")


@pytest.mark.timeout(400)
def test_segment_lbfgsb_with_guards_rechecked_by_oracle():
    """The paper's segment L-BFGS-B (49 edges with the 32 guard channels, Table II) at G=64, N_M=112,
    converged to max|grad L| <= 0.01 from 0 dBm."""
    wl = W.config_ou_guarded(grid_s=64, grid_v=64, n_steps=112)
    eng = B.Engine(wl.fibre, W.FP32)
    print("[optimise] segment L-BFGS-B", flush=True)
    x, p, hist, res, counts = OPT.segment_lbfgsb(eng, wl.plan)
    print(f"[optimise] L-BFGS-B: {len(hist)} evaluations, {hist[0] / 1e12:.3f} -> {max(hist) / 1e12:.3f} Tb/s, "
          f"{res.message}", flush=True)
    assert counts == [23, 10, 6, 3, 4, 3] and len(x) == 49
    assert res.success and max(hist) > hist[0]
    assert np.all(np.isneginf(p[wl.plan.p_w == 0]))
    oracle_recheck(wl, p, "L-BFGS-B")
