"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle, element by element.

Tolerances (derivation in DESIGN.md, "Parity tolerances"):
  * FP64 form: tiles relative 1e-11 (rounding order only);
  * FP32 form: tiles relative 2e-6 -- a few FP32 ulps on each of ~100 step terms, the
    phase kept in FP64 -- well inside the model targets |dSNR| <= 0.01 dB, eta <= 1e-4.
"""
import os
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_18022_amd import binding as B
from paper_2401_18022_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_TILE = {W.FP64: 1e-11, W.FP32: 2e-6}
TOL_ETA = {W.FP64: 1e-11, W.FP32: 2e-6}
TOL_SNR_DB = {W.FP64: 1e-10, W.FP32: 1e-5}


def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need an MI355X"
    return t


def gpu_forward(wl, prec):
    t = torch()
    eng = B.Engine(wl.fibre, prec)
    P = t.tensor(wl.plan.p_w, dtype=t.float64, device="cuda")
    nf = t.tensor(wl.plan.nf_lin, dtype=t.float64, device="cuda")
    eta, pnli, tl = eng.eta(wl.plan, P, tiles=True)
    snr, thr = eng.snr(wl.plan, P, nf, wl.plan.snr_trx_lin)
    t.cuda.synchronize()
    return dict(eta=eta.cpu().numpy(), pnli=pnli.cpu().numpy(), tiles=B.tiles_to_blocks(tl, wl.plan),
                snr=snr.cpu().numpy(), thr=thr.cpu().numpy())


def check(wl, prec, coi=None, b=0, g=None, offset=0):
    print(f"[parity] {wl.name} prec={prec} coi={coi}", flush=True)
    orc = O.Oracle(wl.fibre, wl.plan.sub(b) if wl.plan.n_batch > 1 else wl.plan).forward(coi)
    g = g or gpu_forward(wl, prec)
    c = orc["coi"]
    tg = g["tiles"][b][c]
    np.testing.assert_allclose(tg, orc["tiles"], rtol=TOL_TILE[prec], atol=0)
    np.testing.assert_allclose(g["pnli"][offset + c], orc["pnli"], rtol=TOL_ETA[prec])
    ok = orc["snr"] > 0
    np.testing.assert_allclose(g["eta"][offset + c][ok], orc["eta"][ok], rtol=TOL_ETA[prec])
    assert np.all(np.isnan(g["eta"][offset + c][~ok]))
    d = np.abs(10 * np.log10(g["snr"][offset + c][ok] / orc["snr"][ok]))
    assert np.all(d <= TOL_SNR_DB[prec]), d.max()
    if coi is None:
        assert g["thr"][b] == pytest.approx(orc["thr"], rel=10 * TOL_ETA[prec])
    return g


@pytest.mark.parametrize("prec", [W.FP64, W.FP32])
def test_profile_matches_oracle(prec):
    t = torch()
    for wl in (W.config_tiny(n_steps=20), W.random_small(9, seed=3), W.config_cl(n_steps=40)):
        eng = B.Engine(wl.fibre, prec)
        P = t.tensor(wl.plan.p_w, dtype=t.float64, device="cuda")
        zm, dz, ell, ellL = eng.profile(wl.plan, P)
        t.cuda.synchronize()
        pr = O.Oracle(wl.fibre, wl.plan).profile()
        np.testing.assert_allclose(zm.cpu().numpy(), pr["zm"], rtol=1e-14)
        np.testing.assert_allclose(dz.cpu().numpy(), pr["dz"], rtol=1e-12)
        np.testing.assert_allclose(ell.cpu().numpy().reshape(pr["ell"].shape), pr["ell"], atol=1e-12, rtol=0)
        np.testing.assert_allclose(ellL.cpu().numpy(), pr["ell_L"], atol=1e-12, rtol=0)


@pytest.mark.parametrize("prec", [W.FP64, W.FP32])
@pytest.mark.parametrize("make", [
    lambda: W.config_tiny(),                                                   # 5 ch, closed form, G=64
    lambda: W.random_small(9, seed=3),                                         # ragged rates/gaps, ODE
    lambda: W.random_small(7, seed=5, profile=W.PROFILE_CLOSED_FORM, grid_s=24, grid_v=40, n_steps=30),
    lambda: W.single_channel(grid_s=64, grid_v=64),                            # SCI only
    lambda: W.two_channel(0.2e12, grid_s=48, grid_v=16, n_steps=50),           # grid_v below one wave
    lambda: W.random_small(1, seed=7),                                         # one channel, ODE
    lambda: W.random_small(2, seed=8),                                         # two channels, ODE
    # 8 channels 50 GHz apart, then 4 spread 2 THz apart: the mean-spacing estimate of a channel
    # index is off by up to 7, so the lookup's walk gives way to the binary search
    lambda: W.Workload("irregular-12ch", W.cl_fibre(grid_s=16, grid_v=16, n_steps=24),
                       W.single_plan(190e12 + np.concatenate([50e9 * np.arange(8), 2.35e12 + 2e12 * np.arange(4)]),
                                     32e9, 1e-3, W.db_to_lin(5.0))),
], ids=["tiny", "ragged-ode", "ragged-cf", "single", "two-ch", "single-ode", "two-ode", "irregular"])
def test_all_tiles_match_oracle(make, prec):
    check(make(), prec)


@pytest.mark.parametrize("prec", [W.FP64, W.FP32])
def test_guard_channels(prec):
    wl = W.config_tiny(grid_s=32, grid_v=32, n_steps=40)
    p = wl.plan.p_w.copy()
    p[[0, 3]] = 0.0
    check(wl.with_plan(wl.plan.with_power(p)), prec)


@pytest.mark.parametrize("prec", [W.FP64, W.FP32])
def test_several_spans_match_oracle(prec):
    """n identical spans: the library's phased-array factor per node and n-fold ASE against the
    oracle's explicit sum over the spans' fields."""
    base = W.random_small(8, seed=31, grid_s=16, grid_v=24, n_steps=24)
    for n in (2, 5):
        check(W.Workload(f"{base.name}-{n}-spans", base.fibre.replace(n_spans=n), base.plan), prec)


def test_transceiver_noise():
    wl = W.config_tiny(grid_s=32, grid_v=32)
    plan = wl.plan
    plan.snr_trx_lin = 100.0
    check(wl.with_plan(plan), W.FP32)


@pytest.mark.parametrize("prec", [W.FP64, W.FP32])
def test_batched_plans_match_per_plan_oracle(prec):
    """Several plans of uneven size (1 channel included) in one persistent launch."""
    plans = [W.random_small(n, seed=40 + n).plan for n in (6, 1, 11, 3)]
    fb = W.random_small(6, seed=46).fibre
    wl = W.Workload("batch-small", fb, W.concat_plans(plans))
    g = gpu_forward(wl, prec)
    for b in range(wl.plan.n_batch):
        sub = W.Workload(f"batch-small[{b}]", fb, wl.plan.sub(b))
        check(sub, prec, b=0, g=dict(tiles=[g["tiles"][b]], pnli=g["pnli"], eta=g["eta"], snr=g["snr"],
                                     thr=g["thr"][b:b + 1]), offset=int(wl.plan.offsets[b]))


def test_cl_band_full_grid_sampled():
    """C+L system at its full size (95 ch, G=256, N_M=112): COI rows 0, 47, 94 against the oracle,
    and the FP32 form against the FP64 form on all 9025 tiles."""
    wl = W.config_cl()
    g32 = check(wl, W.FP32, coi=[0, 47, 94])
    g64 = gpu_forward(wl, W.FP64)
    np.testing.assert_allclose(g32["tiles"][0], g64["tiles"][0], rtol=TOL_TILE[W.FP32])
    d = np.abs(10 * np.log10(g32["snr"] / g64["snr"]))
    assert d.max() <= 0.01


def test_ou_band_full_grid_sampled():
    """O-to-U system at its full size (589 ch, G=128, N_M=112): the middle COI's 589 tiles, and
    properties of the whole result that hold at any size."""
    wl = W.config_ou()
    g = check(wl, W.FP32, coi=[294])
    assert np.all(np.isfinite(g["tiles"][0])) and np.all(g["tiles"][0] > 0)
    assert np.all(g["snr"] > 0) and np.isfinite(g["thr"][0])


@pytest.mark.parametrize("make", [lambda: W.config_ou(grid_s=16, grid_v=16),
                                  lambda: W.config_batch(n_profiles=6, grid_s=12, grid_v=12, n_steps=40)])
def test_lowrank_profile_table_matches_table_reads(make):
    """With the ODE profile the FP32 step terms take the f1 + f2 profile values from a low-rank
    form of the plan's table when its factorisation meets its bound; that path and the table
    reads (ISRSGN_LOWRANK=0) give the same tiles and SNR to the FP32 tolerance and the same
    gradient to 1e-5 of its scale."""
    t = torch()
    wl = make()
    P = t.tensor(wl.plan.p_w, dtype=t.float64, device="cuda")
    nf = t.tensor(wl.plan.nf_lin, dtype=t.float64, device="cuda")
    res = {}
    for mode in ("1", "0"):            # "1": the default (up to 8 terms); "0": table reads
        if mode == "0":
            os.environ["ISRSGN_LOWRANK"] = "0"
        try:
            eng = B.Engine(wl.fibre, W.FP32)
            _, _, tl = eng.eta(wl.plan, P, tiles=True)
            wc = eng.work_counts()
            snr, thr, g = eng.snr_grad(wl.plan, P, nf)
            t.cuda.synchronize()
        finally:
            os.environ.pop("ISRSGN_LOWRANK", None)
        res[mode] = (tl.cpu().numpy(), snr.cpu().numpy(), g.cpu().numpy(), wc)
    print(f"[lowrank] {wl.name}: {res['1'][3]['lowrank_plans']} of {wl.plan.n_batch} plans, "
          f"{res['1'][3]['lowrank_terms']} terms", flush=True)
    assert 1 <= res["1"][3]["lowrank_plans"] <= wl.plan.n_batch and 1 <= res["1"][3]["lowrank_terms"] <= 8
    if wl.plan.n_batch == 1:
        assert res["1"][3]["lowrank_plans"] == 1
    assert res["0"][3]["lowrank_plans"] == 0
    np.testing.assert_allclose(res["1"][0], res["0"][0], rtol=TOL_TILE[W.FP32], atol=0)
    d = np.abs(10 * np.log10(res["1"][1] / res["0"][1]))
    assert d.max() <= TOL_SNR_DB[W.FP32], d.max()
    scale = np.abs(res["0"][2]).max()
    assert np.abs(res["1"][2] - res["0"][2]).max() <= 1e-5 * scale


def test_lowrank_cap_falls_back_to_table_reads():
    """The O-to-U profile table needs 8 terms; capped at 2 (ISRSGN_LOWRANK=2) the factorisation
    gives up and the kernel reads the table, exactly as with the low-rank form disabled."""
    t = torch()
    wl = W.config_ou(grid_s=8, grid_v=8, n_steps=24)
    P = t.tensor(wl.plan.p_w, dtype=t.float64, device="cuda")
    out = {}
    for mode in ("2", "0"):
        os.environ["ISRSGN_LOWRANK"] = mode
        try:
            eng = B.Engine(wl.fibre, W.FP32)
            _, _, tl = eng.eta(wl.plan, P, tiles=True)
            t.cuda.synchronize()
            out[mode] = (tl.cpu().numpy(), eng.work_counts()["lowrank_plans"])
        finally:
            del os.environ["ISRSGN_LOWRANK"]
    assert out["2"][1] == 0 and out["0"][1] == 0
    assert np.array_equal(out["2"][0], out["0"][0])


def test_deterministic_repeat():
    wl = W.config_cl(grid_s=32, grid_v=32, n_steps=40)
    a, b = gpu_forward(wl, W.FP32), gpu_forward(wl, W.FP32)
    assert np.array_equal(a["tiles"][0], b["tiles"][0])
    assert np.array_equal(a["snr"], b["snr"])


def test_invalid_plans_rejected():
    t = torch()
    eng = B.Engine(W.tiny_fibre(grid_s=8, grid_v=8, n_steps=8))
    P = t.ones(3, dtype=t.float64, device="cuda") * 1e-3
    for f in ([193e12, 193.05e12, 193.2e12], [193.2e12, 193.1e12, 193e12]):   # overlapping, unsorted
        plan = W.single_plan(np.array(f), 96e9, 1e-3, 1.0)
        with pytest.raises(B.IsrsgnError) as e:
            eng.eta(plan, P)
        assert e.value.code == B.ISRSGN_EINVAL
    big = W.single_plan(190e12 + 100e9 * np.arange(1100), 96e9, 1e-3, 1.0)
    with pytest.raises(B.IsrsgnError):
        eng.eta(big, t.ones(1100, dtype=t.float64, device="cuda"))
    ok = W.single_plan(np.array([193e12, 193.1e12, 193.2e12]), 96e9, 1e-3, 1.0)
    eta, _, _ = eng.eta(ok, P)
    assert t.isfinite(eta).all()


def test_allocation_failure_leaves_handle_usable():
    t = torch()
    eng = B.Engine(W.tiny_fibre(grid_s=8, grid_v=8, n_steps=8))
    plan = W.config_tiny().plan
    P = t.tensor(plan.p_w, dtype=t.float64, device="cuda")
    os.environ["ISRSGN_FAIL_ALLOC"] = "1"
    try:
        with pytest.raises(B.IsrsgnError) as e:
            eng.eta(plan, P)
        assert e.value.code == B.ISRSGN_ENOMEM
    finally:
        del os.environ["ISRSGN_FAIL_ALLOC"]
    eta, _, _ = eng.eta(plan, P)
    t.cuda.synchronize()
    assert t.isfinite(eta).all()


def test_invalid_powers_rejected_and_handle_usable():
    """The boundary's input rules: a negative or NaN launch power (or noise figure) is rejected with
    EINVAL naming its index, no output is written, and the handle keeps working; with the checks
    switched off the values are not validated (NaN propagates)."""
    t = torch()
    wl = W.config_tiny(grid_s=8, grid_v=8, n_steps=8)
    eng = B.Engine(wl.fibre)
    plan = wl.plan
    good = t.tensor(plan.p_w, dtype=t.float64, device="cuda")
    nf = t.tensor(plan.nf_lin, dtype=t.float64, device="cuda")
    pa = eng._plan(plan)
    for bad_value, idx in ((-1e-3, 3), (float("nan"), 1), (float("inf"), 0)):
        P = good.clone()
        P[idx] = bad_value
        snr = t.full((5,), 7.0, dtype=t.float64, device="cuda")
        thr = t.full((1,), 7.0, dtype=t.float64, device="cuda")
        g = t.full((5,), 7.0, dtype=t.float64, device="cuda")
        for call in ("snr", "grad"):
            if call == "snr":
                rc = B.lib().isrsgn_snr(eng.h, B.C.byref(pa.c), B._ptr(P), B._ptr(nf), 0.0, B._ptr(snr), B._ptr(thr),
                                        B._stream())
            else:
                rc = B.lib().isrsgn_snr_grad(eng.h, B.C.byref(pa.c), B._ptr(P), B._ptr(nf), 0.0, B._ptr(snr),
                                             B._ptr(thr), B._ptr(g), B._stream())
            assert rc == B.ISRSGN_EINVAL
            assert f"P_w_dev[{idx}]" in B.lib().isrsgn_last_error().decode()
        with pytest.raises(B.IsrsgnError) as e:
            eng.eta(plan, P)
        assert e.value.code == B.ISRSGN_EINVAL
        with pytest.raises(B.IsrsgnError):
            eng.profile(plan, P)
        t.cuda.synchronize()
        assert bool((snr == 7.0).all()) and bool((thr == 7.0).all()) and bool((g == 7.0).all())
    bad_nf = nf.clone()
    bad_nf[4] = -1.0
    with pytest.raises(B.IsrsgnError) as e:
        eng.snr(plan, good, bad_nf)
    assert e.value.code == B.ISRSGN_EINVAL and "nf_lin_dev[4]" in str(e.value)
    # the handle is still usable, and agrees with a fresh one
    s1, t1, g1 = eng.snr_grad(plan, good, nf)
    s2, t2, g2 = B.Engine(wl.fibre).snr_grad(plan, good, nf)
    t.cuda.synchronize()
    assert t.equal(s1, s2) and t.equal(t1, t2) and t.equal(g1, g2)
    # checks off: not validated, NaN propagates
    eng.set_checks(False)
    P = good.clone()
    P[2] = float("nan")
    snr, thr = eng.snr(plan, P, nf)
    t.cuda.synchronize()
    assert bool(t.isnan(thr).all())
