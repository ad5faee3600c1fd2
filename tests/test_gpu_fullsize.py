"""Parity at the workloads' full sizes, against stored oracle values.

The expected values are the FP64 CPU oracle's, written by tests/golden/make_oracle_golden.py
(which calls only oracle/ on the seeded inputs of workloads.py); each file carries a hash of its
inputs, checked here against the regenerated workload.  tests/test_golden.py recomputes samples
of every file with the current oracle on the CPU.

  * O-to-U, 589 channels, G=128, N_M=112: the tile rows, P_NLI, eta and SNR of the 16 seeded
    channels and of channels 0 and 588, in the FP32 and FP64 forms; the two forms' SNR over all
    589 channels within 0.01 dB of each other;
  * O-to-U at G=32, N_M=40: SNR of all 589 channels and the throughput gradient along the 16
    directions P_c e_c of the seeded channels against the oracle's dual numbers;
  * the batch workload (256 profiles, G=64, N_M=80): rows 0, N/2 and N-1 of 16 profiles, tiles
    from one eager call and SNR from the graph-captured call.

Tolerances: FP64 form tiles/eta 1e-11 relative, SNR 1e-10 dB, gradient 1e-8 relative per
direction; FP32 form tiles/eta 2e-6, SNR 1e-5 dB (the model targets are 1e-4 and 0.01 dB), gradient
1e-3 relative per direction (the target).
"""
import json
import os

import numpy as np
import pytest

from paper_2401_18022_amd import binding as B
from paper_2401_18022_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")

TOL_TILE = {W.FP64: 1e-11, W.FP32: 2e-6}
TOL_SNR_DB = {W.FP64: 1e-10, W.FP32: 1e-5}
TOL_GRAD = {W.FP64: 1e-8, W.FP32: 1e-3}


def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need an MI355X"
    return t


def golden(name, wl):
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_oracle_golden", os.path.join(GOLDEN, "make_oracle_golden.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    with open(os.path.join(GOLDEN, name)) as fh:
        g = json.load(fh)
    assert g["inputs_sha256"] == mk.inputs_sha256(wl), f"{name}: the workload changed; regenerate it"
    return g, mk


def dev(a):
    t = torch()
    return t.tensor(np.asarray(a, dtype=np.float64), dtype=t.float64, device="cuda")


def snr_db_diff(a, b):
    return np.abs(10 * np.log10(np.asarray(a) / np.asarray(b)))


_OU128 = {}


def ou128_gpu(prec):
    """eta with tiles and SNR of the O-to-U system at G=128 (cached per form within the module)."""
    if prec not in _OU128:
        t = torch()
        wl = W.config_ou(grid_s=128, grid_v=128, n_steps=112)
        eng = B.Engine(wl.fibre, prec)
        P, nf = dev(wl.plan.p_w), dev(wl.plan.nf_lin)
        eta, pnli, tl = eng.eta(wl.plan, P, tiles=True)
        snr, thr = eng.snr(wl.plan, P, nf)
        t.cuda.synchronize()
        n = len(wl.plan.f_hz)
        _OU128[prec] = dict(wl=wl, eta=eta.cpu().numpy(), pnli=pnli.cpu().numpy(),
                            tiles=tl.cpu().numpy().reshape(n, n), snr=snr.cpu().numpy())
    return _OU128[prec]


@pytest.mark.parametrize("prec", [W.FP32, W.FP64])
def test_ou_g128_seeded_channels_match_oracle(prec):
    print(f"[fullsize] O-to-U G=128 prec={prec}: 18 COI rows against the oracle", flush=True)
    g = ou128_gpu(prec)
    ref, _ = golden("oracle_ou_g128.json", g["wl"])
    coi = np.asarray(ref["coi"])
    assert len(coi) == 18 and coi[0] == 0 and coi[-1] == 588
    rt = np.asarray(ref["tiles"])
    rel = np.abs(g["tiles"][coi] / rt - 1)
    print(f"[fullsize] max tile rel error {rel.max():.2e}", flush=True)
    assert rel.max() <= TOL_TILE[prec]
    np.testing.assert_allclose(g["pnli"][coi], ref["pnli"], rtol=TOL_TILE[prec], atol=0)
    np.testing.assert_allclose(g["eta"][coi], ref["eta"], rtol=TOL_TILE[prec], atol=0)
    d = snr_db_diff(g["snr"][coi], ref["snr"])
    print(f"[fullsize] max |dSNR| {d.max():.2e} dB", flush=True)
    assert d.max() <= TOL_SNR_DB[prec]


def test_ou_g128_fp32_and_fp64_forms_agree_on_every_channel():
    """The FP32 form's SNR over all 589 channels within the model target 0.01 dB of the FP64 form's
    (observed far smaller), and eta within 1e-4."""
    a, b = ou128_gpu(W.FP32), ou128_gpu(W.FP64)
    d = snr_db_diff(a["snr"], b["snr"])
    print(f"[fullsize] FP32 vs FP64 form, 589 channels: max |dSNR| {d.max():.2e} dB", flush=True)
    assert d.max() <= 0.01 and d.max() <= TOL_SNR_DB[W.FP32]
    np.testing.assert_allclose(a["eta"], b["eta"], rtol=1e-4)


@pytest.mark.parametrize("prec", [W.FP32, W.FP64])
def test_ou_g32_gradient_matches_oracle_duals(prec):
    t = torch()
    wl = W.config_ou(grid_s=32, grid_v=32, n_steps=40)
    ref, mk = golden("oracle_ou_grad_g32.json", wl)
    fd, dirs = mk.grad_directions(wl)
    assert list(fd) == ref["channels"]
    print(f"[fullsize] O-to-U G=32 N_M=40 prec={prec}: gradient along 16 directions", flush=True)
    eng = B.Engine(wl.fibre, prec)
    snr, thr, grad = eng.snr_grad(wl.plan, dev(wl.plan.p_w), dev(wl.plan.nf_lin))
    t.cuda.synchronize()
    snr, thr, grad = snr.cpu().numpy(), thr.item(), grad.cpu().numpy()
    d = snr_db_diff(snr, ref["snr"])
    assert d.max() <= TOL_SNR_DB[prec], d.max()
    assert thr == pytest.approx(ref["thr"], rel=1e-6 if prec == W.FP32 else 1e-12)
    got = dirs @ grad
    want = np.asarray(ref["dthr"])
    rel = np.abs(got / want - 1)
    print(f"[fullsize] max |dSNR| {d.max():.2e} dB; gradient rel error per direction max {rel.max():.2e} "
          f"(smallest |dT| {np.abs(want).min():.3e})", flush=True)
    assert rel.max() <= TOL_GRAD[prec]


def test_batch_profiles_match_oracle_and_graph_call():
    """16 of the 256 profiles, rows first / middle / last: tiles and P_NLI of one eager eta call, and
    the SNR of the graph-captured SNR call (the whole batch as one graph replay)."""
    t = torch()
    wl = W.config_batch()
    ref, _ = golden("oracle_batch_g64.json", wl)
    eng = B.Engine(wl.fibre, W.FP32)
    P, nf = dev(wl.plan.p_w), dev(wl.plan.nf_lin)
    print("[fullsize] batch workload: eager eta with tiles", flush=True)
    eta, pnli, tl = eng.eta(wl.plan, P, tiles=True)
    t.cuda.synchronize()
    blocks = B.tiles_to_blocks(tl, wl.plan)
    pnli = pnli.cpu().numpy()
    del tl
    print("[fullsize] batch workload: graph-captured SNR call", flush=True)
    eng.set_graph(True)
    snr, thr = eng.snr(wl.plan, P, nf)
    t.cuda.synchronize()
    snr = snr.cpu().numpy()
    worst_t, worst_s = 0.0, 0.0
    for prof in ref["profiles"]:
        b, coi = prof["profile"], np.asarray(prof["coi"])
        off = int(wl.plan.offsets[b])
        assert prof["n"] == int(wl.plan.offsets[b + 1]) - off
        rel = np.abs(blocks[b][coi] / np.asarray(prof["tiles"]) - 1)
        worst_t = max(worst_t, float(rel.max()))
        np.testing.assert_allclose(pnli[off + coi], prof["pnli"], rtol=TOL_TILE[W.FP32], atol=0)
        worst_s = max(worst_s, float(snr_db_diff(snr[off + coi], prof["snr"]).max()))
    print(f"[fullsize] 16 profiles x 3 rows: tile rel error {worst_t:.2e}, |dSNR| {worst_s:.2e} dB", flush=True)
    assert worst_t <= TOL_TILE[W.FP32] and worst_s <= TOL_SNR_DB[W.FP32]
