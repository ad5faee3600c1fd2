"""The stored oracle values of the full-size GPU parity tests are the current oracle's.

tests/golden/oracle_*.json were written by tests/golden/make_oracle_golden.py.  Here, on the CPU:
each file's input hash matches the regenerated workload, and samples of every file are recomputed
with the oracle as it stands (a few tiles at G=128 and G=64, one COI row's dual-number derivative
at G=32 with the scalar dual type) and must agree to rounding.
"""
import importlib.util
import json
import os

import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def maker():
    spec = importlib.util.spec_from_file_location("make_oracle_golden", os.path.join(GOLDEN, "make_oracle_golden.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    return mk


def load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def test_ou_g128_golden_is_the_oracles():
    mk = maker()
    wl = mk.ou_g128()
    g = load("oracle_ou_g128.json")
    assert g["inputs_sha256"] == mk.inputs_sha256(wl)
    assert g["coi"] == mk.ou_coi()
    coi = g["coi"]
    # three tiles: an edge COI's own SCI tile, a seeded COI's far interferer, the top edge row
    picks = [(0, 0), (5, 300), (len(coi) - 1, 587)]
    o = O.Oracle(wl.fibre, wl.plan)
    got = o.tiles([coi[q] for q, _ in picks], [k for _, k in picks])
    want = [g["tiles"][q][k] for q, k in picks]
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=0)


def test_batch_golden_is_the_oracles():
    mk = maker()
    wl = mk.batch_g64()
    g = load("oracle_batch_g64.json")
    assert g["inputs_sha256"] == mk.inputs_sha256(wl)
    assert [p["profile"] for p in g["profiles"]] == mk.BATCH_PROFILES
    for prof in (g["profiles"][0], g["profiles"][-1]):
        sub = wl.plan.sub(prof["profile"])
        o = O.Oracle(wl.fibre, sub)
        c = prof["coi"][1]
        got = o.tiles([c, c], [0, prof["n"] - 1])
        np.testing.assert_allclose(got, [prof["tiles"][1][0], prof["tiles"][1][-1]], rtol=1e-13, atol=0)


@pytest.mark.slow
def test_grad_golden_is_the_oracles():
    """One COI row's SNR derivative along one direction, with the scalar dual type (independent of
    the 16-wide dual type that wrote the file)."""
    mk = maker()
    wl = mk.ou_g32()
    g = load("oracle_ou_grad_g32.json")
    assert g["inputs_sha256"] == mk.inputs_sha256(wl)
    fd, dirs = mk.grad_directions(wl)
    assert list(fd) == g["channels"]
    q, coi = 3, int(fd[3])      # the direction of a seeded channel, and that channel's own row
    r = O.Oracle(wl.fibre, wl.plan).forward_dual(dirs[q], coi=[coi])
    assert r["snr"][0] == pytest.approx(g["snr"][coi], rel=1e-13)
    assert r["dsnr"][0] == pytest.approx(g["dsnr"][coi][q], rel=1e-11)
