"""The no-allocation SNR entry point (isrsgn_snr_noalloc) against the allocating one (isrsgn_snr).

Both go through the C ABI.  The no-allocation call works on the library's static device scratch;
two calls in a row, the second with a smaller input (fewer channels, two plans), must each agree
with isrsgn_snr on the same inputs to the precision form's bar (FP32: SNR within 1e-5 dB; FP64:
1e-10 dB), and a plan whose workspace exceeds the scratch is rejected before any device work.
"""
import numpy as np
import pytest

from paper_2401_18022_amd import binding as B
from paper_2401_18022_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_SNR_DB = {W.FP32: 1e-5, W.FP64: 1e-10}
TOL_THR = {W.FP32: 1e-7, W.FP64: 1e-12}


def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need an MI355X"
    return t


def dev(a):
    t = torch()
    return t.tensor(np.asarray(a, dtype=np.float64), dtype=t.float64, device="cuda")


def compare(eng_ref, eng_na, plan, prec):
    t = torch()
    P, nf = dev(plan.p_w), dev(plan.nf_lin)
    snr_na = t.full((len(plan.f_hz),), -1.0, dtype=t.float64, device="cuda")
    thr_na = t.full((plan.n_batch,), -1.0, dtype=t.float64, device="cuda")
    eng_na.snr_noalloc(plan, P, nf, plan.snr_trx_lin, out=(snr_na, thr_na))
    snr, thr = eng_ref.snr(plan, P, nf, plan.snr_trx_lin)
    t.cuda.synchronize()
    a, b = snr_na.cpu().numpy(), snr.cpu().numpy()
    ok = b > 0
    assert np.all(a[~ok] == 0.0)
    d = np.abs(10 * np.log10(a[ok] / b[ok]))
    assert d.max() <= TOL_SNR_DB[prec], d.max()
    np.testing.assert_allclose(thr_na.cpu().numpy(), thr.cpu().numpy(), rtol=TOL_THR[prec], atol=0)
    return float(d.max())


@pytest.mark.parametrize("prec", [W.FP32, W.FP64])
def test_noalloc_matches_snr_two_calls(prec):
    """589 channels, then a smaller call (two plans of 95 and 150 channels) on the same scratch."""
    wl = W.config_ou(grid_s=24, grid_v=24, n_steps=32)
    eng_ref = B.Engine(wl.fibre, prec)
    eng_na = B.Engine(wl.fibre, prec)
    print(f"[noalloc] prec={prec} call 1: 589 channels", flush=True)
    d1 = compare(eng_ref, eng_na, wl.plan, prec)
    grid, rng = W.ou_grid(), np.random.default_rng(7)
    plans = []
    for lo, n in ((40, 95), (300, 150)):
        f = grid[lo:lo + n]
        plans.append(W.single_plan(f, 96e9, W.dbm_to_w(rng.uniform(-2, 2, n)), W.nf_by_band(f)))
    small = W.concat_plans(plans)
    print(f"[noalloc] prec={prec} call 2: plans of 95 and 150 channels", flush=True)
    d2 = compare(eng_ref, eng_na, small, prec)
    print(f"[noalloc] max |dSNR| {d1:.1e} / {d2:.1e} dB", flush=True)


def test_noalloc_closed_form_with_guard_channels():
    """The closed-form profile (tiny system) with empty channels and a transceiver SNR."""
    wl = W.config_tiny(grid_s=16, grid_v=16, n_steps=24)
    p = wl.plan.p_w.copy()
    p[1] = 0.0
    plan = wl.plan.with_power(p)
    plan.snr_trx_lin = 100.0
    compare(B.Engine(wl.fibre), B.Engine(wl.fibre), plan, W.FP32)


def test_noalloc_rejects_a_plan_beyond_the_scratch():
    """The batch workload (256 plans, 3.6e7 tiles) needs ~290 MB of workspace: EINVAL, outputs untouched."""
    t = torch()
    wl = W.config_batch()
    eng = B.Engine(wl.fibre)
    n = len(wl.plan.f_hz)
    snr = t.full((n,), 7.0, dtype=t.float64, device="cuda")
    thr = t.full((wl.plan.n_batch,), 7.0, dtype=t.float64, device="cuda")
    with pytest.raises(B.IsrsgnError) as e:
        eng.snr_noalloc(wl.plan, dev(wl.plan.p_w), dev(wl.plan.nf_lin), out=(snr, thr))
    assert e.value.code == B.ISRSGN_EINVAL and "scratch" in str(e.value)
    t.cuda.synchronize()
    assert bool((snr == 7.0).all()) and bool((thr == 7.0).all())
