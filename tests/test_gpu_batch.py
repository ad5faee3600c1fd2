"""Batching (many plans of uneven size in one persistent launch), graph mode and the tile-kernel
autotuner, all checked against eager single calls or the oracle."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_18022_amd import binding as B
from paper_2401_18022_amd import workloads as W

pytestmark = pytest.mark.gpu


def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def test_graph_replays_match_eager():
    """Each replay of a captured call, with eager torch work and synchronisations between replays,
    equals the eager result bit for bit."""
    t = torch()
    plans = [W.random_small(n, seed=80 + n).plan for n in (7, 3, 12)]
    fb = W.random_small(7, seed=87, grid_s=16, grid_v=16, n_steps=20).fibre
    plan = W.concat_plans(plans)
    P = t.tensor(plan.p_w * 20, dtype=t.float64, device="cuda")
    nf = t.tensor(plan.nf_lin, dtype=t.float64, device="cuda")
    ref = B.Engine(fb, W.FP32)
    snr0, thr0, g0 = ref.snr_grad(plan, P, nf, 50.0)
    eta0, pnli0, tl0 = ref.eta(plan, P, tiles=True)
    eng = B.Engine(fb, W.FP32)
    eng.set_graph(True)
    for rep in range(4):
        noise = t.randn(1000, device="cuda").sum()   # eager work between replays
        snr, thr, g = eng.snr_grad(plan, P, nf, 50.0)
        eta, pnli, tl = eng.eta(plan, P, tiles=True)
        t.cuda.synchronize()
        # forward results are bitwise reproducible; the adjoint sums with FP64 atomics, whose
        # order varies from run to run
        assert t.equal(snr, snr0) and t.equal(thr, thr0), rep
        assert t.allclose(g, g0, rtol=1e-12, atol=1e-12 * g0.abs().max().item()), rep
        assert t.equal(eta, eta0) and t.equal(pnli, pnli0) and t.equal(tl, tl0), rep
        assert t.isfinite(noise)
    # new input values flow through the copy-in of the same graph
    P2 = P * 1.7
    snr2, thr2, g2 = eng.snr_grad(plan, P2, nf, 50.0)
    snr2e, thr2e, g2e = ref.snr_grad(plan, P2, nf, 50.0)
    t.cuda.synchronize()
    assert t.equal(thr2, thr2e) and t.allclose(g2, g2e, rtol=1e-12, atol=1e-12 * g2e.abs().max().item())


def test_adjoint_repeat_runs_agree():
    """The adjoint accumulates with FP64 atomics: repeated runs agree to rounding (FP64 form 1e-12,
    FP32 form 1e-6 of the gradient's scale) while the forward stays bitwise identical."""
    t = torch()
    wl = W.config_cl(grid_s=16, grid_v=16, n_steps=24)
    P = t.tensor(wl.plan.p_w, dtype=t.float64, device="cuda")
    nf = t.tensor(wl.plan.nf_lin, dtype=t.float64, device="cuda")
    for prec, tol in ((W.FP64, 1e-12), (W.FP32, 1e-6)):
        eng = B.Engine(wl.fibre, prec)
        runs = [eng.snr_grad(wl.plan, P, nf) for _ in range(3)]
        t.cuda.synchronize()
        for snr, thr, g in runs[1:]:
            assert t.equal(snr, runs[0][0]) and t.equal(thr, runs[0][1])
            scale = runs[0][2].abs().max().item()
            assert (g - runs[0][2]).abs().max().item() <= tol * scale


def test_every_tile_variant_agrees():
    """All autotuner candidates compute the same tiles (same arithmetic, different scheduling)."""
    t = torch()
    wl = W.random_small(9, seed=3, grid_s=24, grid_v=40, n_steps=30)
    P = t.tensor(wl.plan.p_w, dtype=t.float64, device="cuda")
    out = []
    try:
        for v in range(6):
            os.environ["ISRSGN_TILE_VARIANT"] = str(v)
            eng = B.Engine(wl.fibre, W.FP32)
            _, _, tl = eng.eta(wl.plan, P, tiles=True)
            out.append(tl.cpu().numpy())
            assert eng.work_counts()["variant"] == v
    finally:
        del os.environ["ISRSGN_TILE_VARIANT"]
    for v in range(1, 6):
        np.testing.assert_allclose(out[v], out[0], rtol=1e-6)


def test_batch_workload_sample_matches_oracle():
    """Eight profiles of the seeded batch workload (uneven sub-bands of the O-to-U grid) at a
    reduced grid, in one launch: three tile rows per profile against the oracle."""
    t = torch()
    wl = W.config_batch(n_profiles=8, grid_s=12, grid_v=12, n_steps=16)
    eng = B.Engine(wl.fibre, W.FP32)
    P = t.tensor(wl.plan.p_w, dtype=t.float64, device="cuda")
    nf = t.tensor(wl.plan.nf_lin, dtype=t.float64, device="cuda")
    eta, pnli, tl = eng.eta(wl.plan, P, tiles=True)
    snr, thr = eng.snr(wl.plan, P, nf)
    t.cuda.synchronize()
    blocks = B.tiles_to_blocks(tl, wl.plan)
    for b in range(wl.plan.n_batch):
        sub = wl.plan.sub(b)
        n = len(sub.f_hz)
        coi = [0, n // 2, n - 1]
        print(f"[batch] plan {b} n={n}", flush=True)
        r = O.Oracle(wl.fibre, sub).forward(coi)
        np.testing.assert_allclose(blocks[b][coi], r["tiles"], rtol=2e-6)
        lo = int(wl.plan.offsets[b])
        np.testing.assert_allclose(snr.cpu().numpy()[lo + np.array(coi)], r["snr"], rtol=2e-6)


@pytest.mark.parametrize("prec", [W.FP32, W.FP64])
def test_row_batched_gradient_matches_recompute(prec):
    """Gradient with S kept per batch of COI rows -- store disabled (S recomputed by the
    adjoint), a 5 MiB store (a dozen row batches) and the default store -- gives the same
    gradient (to the rounding of FP64 atomics and of the FP32 run sums), and the same SNR and
    throughput as the SNR-only call, bit for bit."""
    t = torch()
    wl = W.config_cl(grid_s=16, grid_v=16, n_steps=24)
    P = t.tensor(wl.plan.p_w, dtype=t.float64, device="cuda")
    nf = t.tensor(wl.plan.nf_lin, dtype=t.float64, device="cuda")
    res, nodes, batches = {}, {}, {}
    for mb in ("0", "5", "16384"):
        os.environ["ISRSGN_STORE_MB"] = mb
        try:
            eng = B.Engine(wl.fibre, prec)
            res[mb] = eng.snr_grad(wl.plan, P, nf)
            t.cuda.synchronize()
            wc = eng.work_counts()
            nodes[mb], batches[mb] = wc["nodes"], wc["grad_batches"]
        finally:
            del os.environ["ISRSGN_STORE_MB"]
    assert batches["0"] == 0 and batches["5"] > 4 and batches["16384"] == 1, batches
    snr1, thr1 = eng.snr(wl.plan, P, nf)
    t.cuda.synchronize()
    ref = res["0"]
    scale = ref[2].abs().max().item()
    tol = 1e-6 if prec == W.FP32 else 1e-12
    for mb in ("5", "16384"):
        snr, thr, g = res[mb]
        assert t.equal(snr, ref[0]) and t.equal(thr, ref[1]), mb
        assert (g - ref[2]).abs().max().item() <= tol * scale, mb
        assert nodes[mb] == nodes["0"], mb
    assert t.equal(snr1, ref[0]) and t.equal(thr1, ref[1])


@pytest.mark.gpu
@pytest.mark.parametrize("profile,rolloff", [(W.PROFILE_ODE, 0.0), (W.PROFILE_CLOSED_FORM, 0.0), (W.PROFILE_ODE, 0.1)])
def test_adjoint_four_and_sixteen_wave_workgroups_agree(profile, rolloff):
    """The FP32 adjoint with the S store runs sixteen-wave workgroups where their LDS fits and
    four-wave ones otherwise (large plans).  Forced to four (ISRSGN_ADJOINT_WAVES=4) it gives the
    same gradient to the rounding of the FP64 atomics, and the same SNR bit for bit."""
    t = torch()
    wl = W.random_small(48, 7, profile=profile, rolloff=rolloff)
    P = t.tensor(wl.plan.p_w, dtype=t.float64, device="cuda")
    nf = t.tensor(wl.plan.nf_lin, dtype=t.float64, device="cuda")
    res = {}
    for waves in ("4", "16"):
        os.environ["ISRSGN_ADJOINT_WAVES"] = waves
        try:
            eng = B.Engine(wl.fibre, W.FP32)
            res[waves] = eng.snr_grad(wl.plan, P, nf)
            t.cuda.synchronize()
            assert eng.work_counts()["grad_batches"] >= 1
        finally:
            del os.environ["ISRSGN_ADJOINT_WAVES"]
    a, b = res["4"], res["16"]
    assert t.equal(a[0], b[0]) and t.equal(a[1], b[1])
    scale = a[2].abs().max().item()
    assert (a[2] - b[2]).abs().max().item() <= 1e-12 * scale


@pytest.mark.gpu
def test_adjoint_mixed_lowrank_and_gather_plans():
    """FP32 form with the ODE profile: the adjoint's low-rank instantiation takes the tiles of plans
    that have a low-rank profile table, the gather instantiation the others.  Capping the rank
    (ISRSGN_LOWRANK=N) below what some plans of a batch need leaves a mix in one launch; SNR and
    gradient then agree with the table reads everywhere (ISRSGN_LOWRANK=0)."""
    t = torch()
    wl = W.config_batch(n_profiles=12, grid_s=12, grid_v=12, n_steps=24)
    P = t.tensor(wl.plan.p_w, dtype=t.float64, device="cuda")
    nf = t.tensor(wl.plan.nf_lin, dtype=t.float64, device="cuda")
    res, plans = {}, {}
    for cap in ("0", "2", "3", "4", "5", "6", "7", "8"):
        os.environ["ISRSGN_LOWRANK"] = cap
        try:
            eng = B.Engine(wl.fibre, W.FP32)
            res[cap] = eng.snr_grad(wl.plan, P, nf)
            t.cuda.synchronize()
            plans[cap] = eng.work_counts()["lowrank_plans"]
        finally:
            del os.environ["ISRSGN_LOWRANK"]
    print(f"[mixed] low-rank plans by cap: {plans} of {wl.plan.n_batch}", flush=True)
    assert plans["0"] == 0
    mixed = [c for c in plans if 0 < plans[c] < wl.plan.n_batch]
    assert mixed, plans
    ref = res["0"]
    scale = ref[2].abs().max().item()
    for c in mixed + ["8"]:
        snr_db = 10 * t.log10(res[c][0] / ref[0])
        assert snr_db.abs().max().item() <= 1e-5
        assert (res[c][2] - ref[2]).abs().max().item() <= 1e-5 * scale
