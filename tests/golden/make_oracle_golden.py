"""Writes the oracle's expected values for the full-size parity tests (tests/golden/oracle_*.json).

    python tests/golden/make_oracle_golden.py [--threads N] [--only ou_g128|batch_g64|ou_grad_g32]

Every value comes from the FP64 CPU oracle (oracle/) on the seeded synthetic workloads of
paper_2401_18022_amd/workloads.py (which holds no model arithmetic); nothing is read from the
GPU library.  Each file records the workload, the oracle call and a SHA-256 of the inputs, so a
test can regenerate the inputs and see that they are unchanged.  Run times on 8 cores: about
15, 5 and 60 minutes.

  oracle_ou_g128.json     O-to-U 589 channels, G=128, N_M=112: tile rows, P_NLI, eta and SNR of
                          the 16 seeded finite-difference channels and of channels 0 and 588
  oracle_batch_g64.json   16 of the 256 launch-power profiles of the batch workload (G=64,
                          N_M=80): first, middle and last COI row of each
  oracle_ou_grad_g32.json O-to-U 589 channels at G=32, N_M=40: SNR of every channel, the
                          throughput, and its derivatives along the 16 directions P_c e_c of the
                          seeded channels c (dual numbers over all 589 COI rows)
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2401_18022_amd import workloads as W  # noqa: E402

BATCH_PROFILES = [int(round(x)) for x in np.linspace(0, 255, 16)]


# fibre fields that switch model extensions on: hashed only when on, so a workload's hash does not
# depend on extensions it does not use
EXTENSION_DEFAULTS = {"rolloff": 0.0, "nli_points": 1}


def inputs_sha256(wl) -> str:
    """Hash of everything the oracle reads: fibre fields and plan arrays."""
    h = hashlib.sha256()
    for f in dataclasses.fields(wl.fibre):
        v = getattr(wl.fibre, f.name)
        if f.name in EXTENSION_DEFAULTS and v == EXTENSION_DEFAULTS[f.name]:
            continue
        h.update(f.name.encode())
        h.update(np.ascontiguousarray(np.asarray(v, dtype=np.float64)).tobytes())
    p = wl.plan
    for a in (p.f_hz, p.rs_hz, p.p_w, p.nf_lin):
        h.update(np.ascontiguousarray(np.asarray(a, dtype=np.float64)).tobytes())
    h.update(np.asarray(p.offsets, dtype=np.int64).tobytes())
    h.update(np.float64(p.snr_trx_lin).tobytes())
    return h.hexdigest()


# the workloads, as the tests rebuild them
def ou_g128():
    return W.config_ou(grid_s=128, grid_v=128, n_steps=112)


def batch_g64():
    return W.config_batch()


def ou_g32():
    return W.config_ou(grid_s=32, grid_v=32, n_steps=40)


def ou_coi():
    return [0] + [int(c) for c in W.fd_channels()] + [588]


def grad_directions(wl):
    fd = W.fd_channels()
    d = np.zeros((len(fd), len(wl.plan.f_hz)))
    d[np.arange(len(fd)), fd] = wl.plan.p_w[fd]
    return fd, d


def write(name, payload):
    path = os.path.join(HERE, name)
    with open(path, "w") as fh:
        json.dump(payload, fh, indent=0)
        fh.write("\n")
    print(f"wrote {path}", flush=True)


def make_ou_g128(threads):
    wl = ou_g128()
    coi = ou_coi()
    t = time.time()
    r = orc.Oracle(wl.fibre, wl.plan, n_threads=threads).forward(coi=coi)
    write("oracle_ou_g128.json", dict(
        what="O-to-U 589 ch, G=128, N_M=112: oracle rows of the seeded channels and of the band edges",
        workload="workloads.config_ou(grid_s=128, grid_v=128, n_steps=112)",
        call="oracle.Oracle(fibre, plan).forward(coi)", inputs_sha256=inputs_sha256(wl),
        coi=coi, tiles=r["tiles"].tolist(), pnli=r["pnli"].tolist(), eta=r["eta"].tolist(),
        snr=r["snr"].tolist(), seconds=time.time() - t, threads=threads))


def make_batch_g64(threads):
    wl = batch_g64()
    rows = []
    t = time.time()
    for b in BATCH_PROFILES:
        sub = wl.plan.sub(b)
        n = len(sub.f_hz)
        coi = [0, n // 2, n - 1]
        r = orc.Oracle(wl.fibre, sub, n_threads=threads).forward(coi=coi)
        rows.append(dict(profile=b, n=n, coi=coi, tiles=r["tiles"].tolist(), pnli=r["pnli"].tolist(),
                         snr=r["snr"].tolist()))
        print(f"profile {b}: {n} channels, {time.time() - t:.0f} s", flush=True)
    write("oracle_batch_g64.json", dict(
        what="batch workload (256 profiles, G=64, N_M=80): oracle rows 0, N/2, N-1 of 16 profiles",
        workload="workloads.config_batch()", call="oracle.Oracle(fibre, plan.sub(b)).forward(coi)",
        inputs_sha256=inputs_sha256(wl), profiles=rows, seconds=time.time() - t, threads=threads))


def make_ou_grad_g32(threads):
    wl = ou_g32()
    fd, d = grad_directions(wl)
    t = time.time()
    r = orc.Oracle(wl.fibre, wl.plan, n_threads=threads).forward_dualn(d)
    write("oracle_ou_grad_g32.json", dict(
        what="O-to-U 589 ch, G=32, N_M=40: SNR, throughput and its derivative along P_c e_c for the "
             "16 seeded channels c (oracle dual numbers over all COI rows)",
        workload="workloads.config_ou(grid_s=32, grid_v=32, n_steps=40)",
        call="oracle.Oracle(fibre, plan).forward_dualn(directions)", inputs_sha256=inputs_sha256(wl),
        channels=[int(c) for c in fd], snr=r["snr"].tolist(), pnli=r["pnli"].tolist(), thr=r["thr"],
        dthr=r["dthr"].tolist(), dsnr=r["dsnr"].tolist(), seconds=time.time() - t, threads=threads))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", choices=("ou_g128", "batch_g64", "ou_grad_g32"))
    a = ap.parse_args()
    jobs = {"ou_g128": make_ou_g128, "batch_g64": make_batch_g64, "ou_grad_g32": make_ou_grad_g32}
    for name, fn in jobs.items():
        if a.only in (None, name):
            fn(a.threads)


if __name__ == "__main__":
    main()
