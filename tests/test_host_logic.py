"""Host logic of the launch-power optimiser against the paper's Table I and Table II (CPU only).

Table II lists, per band, the occupied channels (171/143/88/38/65/52) and the optimisation segments
(23/10/6/3/4/3); Table I the 589 channels and 32 guard channels in 5 nm guard-band gaps.
"""
import json
import os

import numpy as np

from paper_2401_18022_amd import optimise as OPT
from paper_2401_18022_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def table2():
    with open(os.path.join(GOLDEN, "table2_noise_figure.json")) as fh:
        return json.load(fh)


def test_segment_rule_gives_table2_from_its_channel_counts():
    """N_B = round(B_band / B_p), B_p = 750 GHz (O) and 1.5 THz (others), 100 GHz per channel."""
    t = table2()
    assert OPT.segment_counts(t["channels"]) == t["segments"]


def test_guarded_plan_matches_tables_1_and_2():
    wl = W.config_ou_guarded()
    occ = wl.plan.p_w > 0
    assert len(occ) == 589 and int((~occ).sum()) == 32
    bands = OPT.band_of(wl.plan.f_hz)
    t = table2()
    assert [int(np.sum(occ & (bands == b))) for b in range(6)] == t["channels"]
    A, counts = OPT.segment_matrix(wl.plan.f_hz, occupied=occ)
    assert counts == t["segments"] and A.shape == (589, 49)
    # the guard channels sit in 5 nm gaps at the interior band edges
    lam = W.C_LIGHT / wl.plan.f_hz[~occ] * 1e9
    for lo, hi in W.GUARD_GAPS_NM:
        assert hi - lo == 5.0
    assert all(any(lo <= x < hi for lo, hi in W.GUARD_GAPS_NM) for x in lam)


def test_segment_matrix_interpolates_between_edges():
    """Rows of occupied channels are convex weights of two neighbouring edges of their band (exact
    at the band's first and last channel); guard rows are zero; a linear profile in frequency is
    reproduced exactly."""
    wl = W.config_ou_guarded()
    occ = wl.plan.p_w > 0
    A, counts = OPT.segment_matrix(wl.plan.f_hz, occupied=occ)
    assert np.all(A[~occ] == 0.0)
    assert np.allclose(A[occ].sum(axis=1), 1.0) and np.all(A >= 0)
    assert np.all((A[occ] > 0).sum(axis=1) <= 2)
    bands = OPT.band_of(wl.plan.f_hz)
    col0 = 0
    for b, ne in enumerate(counts):
        idx = np.nonzero(occ & (bands == b))[0]
        fe = np.linspace(wl.plan.f_hz[idx[0]], wl.plan.f_hz[idx[-1]], ne)
        x = np.zeros(A.shape[1])
        x[col0:col0 + ne] = 0.3 + 2e-12 * (fe - fe[0])   # dBm linear in frequency
        np.testing.assert_allclose((A @ x)[idx], 0.3 + 2e-12 * (wl.plan.f_hz[idx] - fe[0]), atol=1e-12)
        assert A[idx[0], col0] == 1.0 and A[idx[-1], col0 + ne - 1] == 1.0
        col0 += ne


def test_segment_powers_keep_guards_empty():
    wl = W.config_ou_guarded()
    occ = wl.plan.p_w > 0
    A, _ = OPT.segment_matrix(wl.plan.f_hz, occupied=occ)
    p = OPT.segment_powers(A, occ, np.full(A.shape[1], 1.0))
    assert np.all(p[~occ] == 0.0)
    np.testing.assert_allclose(p[occ], 1e-3 * 10 ** 0.1)
