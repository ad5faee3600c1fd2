"""Benchmark of the ISRS GN pair-integral engine on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-fp64] [--grad|--no-grad]
                    [--copy-probe MIB] [--workload ou|batch]

One step = one full pass of the hot path on the O-to-U system (589 x 96 GBaud,
1260-1675 nm, 80 km SSMF, G=128, N_M=112, FP32 form): distance steps, ODE power
profile, all 589^2 COI x interferer pair integrals, NLI/SNR/throughput reduction and,
with --grad (default once the adjoint is built), the adjoint gradient of the throughput
with respect to all 589 launch powers.  --workload batch measures instead 256 launch-power
profiles over uneven sub-bands (95-589 channels) of the same grid in one call (G=64, N_M=80).  Inputs are seeded and synthetic and are resident
in HBM before the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Minimal VALU issue slots per node-step for eq. (psi_fin)'s step term on gfx950 (the design doc,
# "Roofline"): 4 transcendentals (sin, cos of the phase, sin of the sinc, exp of the power
# term) at a quarter of the FP32 rate = 16 slots, plus 14 single-rate FP32 operations.
SLOTS_PER_NODE_STEP = 30
# The adjoint, per node-step: the step term again (30), Q_m = c Re(conj(S) term_m) (3) and its
# five weighted sums over nodes (sum q, q t1, q t2, q w3a, q w3c: 5).  When it has to recompute
# S (no per-node store), another 30.
ADJ_SLOTS_PER_NODE_STEP = 38
FLOP_EQ_PER_SLOT = 2            # one FMA slot = 2 FLOP at the FP32 vector peak
PEAK_FP32_TFLOPS = 157.3        # MI355X FP32 vector (no matrix cores)

# HBM traffic per launch of the dominant kernels comes from rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs recorded in profiles/; it is reported only while the kernel's sources and build flags
# (build.py) are unchanged.
CSRC = os.path.join(ROOT, "paper_2401_18022_amd", "csrc")
TRAFFIC_RECORDS = {
    "pair_integral_forward": ("pair_integral_forward_ou589_g128_fp32.md",
                              ["isrsgn_kernels.hip", "isrsgn_device.h", "isrsgn_internal.h", "../build.py"]),
    "pair_integral_adjoint": ("pair_integral_adjoint_ou589_g128_fp32.md",
                              ["isrsgn_adjoint.hip", "isrsgn_device.h", "isrsgn_internal.h", "../build.py"]),
}


def kernel_sources_sha256(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel, grid):
    """(fetch, write) bytes per launch from the profile record, or None if absent or stale."""
    if kernel not in TRAFFIC_RECORDS or grid != 128:
        return None
    name, files = TRAFFIC_RECORDS[kernel]
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    sha = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    fetch = re.search(r"fetch_bytes_per_launch:\s*([0-9.eE+]+)", text)
    write = re.search(r"write_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (sha and fetch and write) or sha.group(1) != kernel_sources_sha256(files):
        return None
    return float(fetch.group(1)), float(write.group(1)), "profiles/" + name


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--no-fp64", action="store_true", help="skip timing the FP64 GPU form")
    ap.add_argument("--grad", dest="grad", action="store_true", default=None)
    ap.add_argument("--no-grad", dest="grad", action="store_false")
    ap.add_argument("--workload", choices=("ou", "batch"), default="ou")
    ap.add_argument("--fp64-calls", type=int, default=3, help="timed calls of the FP64 form (median reported)")
    ap.add_argument("--cpu-pairs", type=int, default=48,
                    help="interferers per seeded COI in the CPU-oracle sample (16 seeded COIs)")
    ap.add_argument("--rolloff", type=float, default=0.0,
                    help="raised-cosine roll-off of every transmit spectrum (0: rectangular)")
    ap.add_argument("--nli-points", type=int, default=1,
                    help="points of the within-channel NLI rule per COI (1: the COI centre)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device (calibrates rocprofv3 byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the pair integrals would shard by COI rows; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2401_18022_amd import binding as B
    from paper_2401_18022_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device="cuda")
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        del src
    if args.workload == "ou":
        wl = W.config_ou(grid_s=args.grid, grid_v=args.grid)
    else:
        wl = W.config_batch()
        args.grid = wl.fibre.grid_s
    spectra = args.rolloff > 0.0 or args.nli_points > 1
    if spectra:
        wl = wl.replace_fibre(rolloff=args.rolloff, nli_points=args.nli_points)
    n = len(wl.plan.f_hz)
    offs = np.asarray(wl.plan.offsets)
    pairs = int(np.sum(np.diff(offs) ** 2))
    P = torch.tensor(wl.plan.p_w, dtype=torch.float64, device="cuda")
    nf = torch.tensor(wl.plan.nf_lin, dtype=torch.float64, device="cuda")

    def make(prec):
        e = B.Engine(wl.fibre, prec)
        e.set_timing(True)
        return e

    eng = make(W.FP32)
    grad = args.grad
    if grad is None:
        try:
            eng.snr_grad(wl.plan, P, nf)
            torch.cuda.synchronize()
            grad = True
        except B.IsrsgnError as e:
            if e.code != B.ISRSGN_EUNSUPPORTED:
                raise
            grad = False

    def step(e):
        if grad:
            return e.snr_grad(wl.plan, P, nf)
        return e.snr(wl.plan, P, nf)

    def note(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    note(f"{'SNR+gradient' if grad else 'SNR'} step, FP32 form: warmup")
    keys = ("profile", "tiles", "reduce", "adjoint_tiles", "adjoint_rest", "total")
    eager = {k: 0.0 for k in keys}
    for _ in range(max(1, args.warmup)):
        step(eng)
        eager = eng.stage_times()
    torch.cuda.synchronize()
    graph = args.workload == "batch"
    if graph:
        # the whole call -- every plan's forward, reductions and adjoint -- is captured once and
        # then replays as one HIP graph; its stage split comes from the eager warmup call above
        note("graph mode: capture call")
        eng.set_graph(True)
        step(eng)
        torch.cuda.synchronize()
    stages = {k: 0.0 for k in keys}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step(eng)
        st = eng.stage_times()          # waits for this step's last event
        for k in stages:
            stages[k] += st[k]
        note(f"timed step done in {st['total']:.0f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    thr = out[1].sum().item()
    work = eng.work_counts()
    ms_step = 1e3 * elapsed / args.steps
    if graph:   # per-kernel times of the eager call, the graph's whole-call time
        stages = {k: eager[k] * args.steps for k in keys}
    tiles_ms = stages["tiles"] / args.steps
    node_steps = work["node_steps"]
    dominant, dom_ms, dom_slots = "pair_integral_forward", tiles_ms, SLOTS_PER_NODE_STEP
    if grad and stages["adjoint_tiles"] / args.steps > tiles_ms:
        dominant, dom_ms = "pair_integral_adjoint", stages["adjoint_tiles"] / args.steps
        dom_slots = ADJ_SLOTS_PER_NODE_STEP + (0 if work["grad_batches"] > 0 else SLOTS_PER_NODE_STEP)
    # stage times are sums over the call's launches of the kernel (one per batch of COI rows)
    launches = max(1, work["grad_batches"]) if grad else 1
    achieved = node_steps * dom_slots * FLOP_EQ_PER_SLOT / (dom_ms * 1e-3) / 1e12
    rec = recorded_traffic(dominant, args.grid) if args.workload == "ou" and not spectra else None

    fp64 = None
    if not args.no_fp64 and args.workload == "ou" and args.fp64_calls > 0:
        note("FP64 form: first call (autotune)")
        e64 = make(W.FP64)
        step(e64)
        torch.cuda.synchronize()
        times, tiles64 = [], []
        for q in range(args.fp64_calls):
            t1 = time.perf_counter()
            step(e64)
            s64 = e64.stage_times()
            torch.cuda.synchronize()
            times.append(1e3 * (time.perf_counter() - t1))
            tiles64.append(s64["tiles"])
            note(f"FP64 form: timed call {q + 1} of {args.fp64_calls} in {times[-1]:.0f} ms")
        med = float(np.median(times))
        fp64 = dict(ms_per_step=med, ms_per_step_calls=times, tiles_ms=float(np.median(tiles64)),
                    speedup_fp32_over_fp64=med / ms_step)
        e64.close()

    cpu = None
    if not args.no_cpu and args.cpu_pairs > 0:
        note("CPU oracle sample")
        from oracle import oracle as orc
        sub = wl.plan.sub(0) if wl.plan.n_batch > 1 else wl.plan
        n0 = len(sub.f_hz)
        # the 16 seeded COIs of the gradient check, each with a seeded set of interferers: pair
        # integrals cost about the same everywhere in the tile list, so the sample's rate stands
        # for the whole problem (the extrapolation below says so)
        cois = W.fd_channels(n_ch=n0)
        rng = np.random.default_rng(6)
        per = min(args.cpu_pairs, n0)
        ci = np.repeat(cois, per)
        ki = np.concatenate([np.sort(rng.choice(n0, per, replace=False)) for _ in cois])
        nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        threads = min(16, nproc)     # the host's CPU share per GPU
        o = orc.Oracle(wl.fibre, sub, n_threads=threads)
        tc = time.perf_counter()
        o.tiles(ci, ki)
        dt = time.perf_counter() - tc
        rate = len(ci) / dt
        model = "?"
        try:
            with open("/proc/cpuinfo") as fh:
                for line in fh:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
        full_pairs = int(np.sum(np.diff(np.asarray(sub.offsets)) ** 2))
        cpu = {"value": rate, "unit": "pair-integrals/s", "cores": threads, "kind": "oracle",
               "sample": f"FP64 oracle, forward pair integrals of the 16 seeded COIs x {per} seeded interferers "
                         f"each ({len(ci)} tiles; G={args.grid}, N_M={wl.fibre.n_steps}) in {dt:.1f} s on "
                         f"{threads} threads; no profile adjoint",
               "nproc": nproc, "cpu_model": model,
               "extrapolated_full_forward_s": full_pairs / rate,
               "extrapolation": f"linear: all {full_pairs} pair integrals of the plan at the sample's rate "
                                f"(the work per tile is the same on average; labelled estimate, not measured)"}

    what = ("SNR + adjoint gradient" if grad else "SNR (forward) only")
    if spectra:
        what += f"; raised-cosine spectra, roll-off {args.rolloff:g}, {args.nli_points} NLI point(s) per COI"

    if args.workload == "ou":
        workload = (f"O-to-U 589x96GBaud 100GHz 1260-1675nm, 80 km SSMF, ODE ISRS profile, "
                    f"G={args.grid}x{args.grid}, N_M={wl.fibre.n_steps}, FP32 form, " + what)
    else:
        workload = (f"{wl.plan.n_batch} launch-power profiles over uneven O-to-U sub-bands (95-589 ch), "
                    f"ODE ISRS profile, G={args.grid}x{args.grid}, N_M={wl.fibre.n_steps}, FP32 form, one call, "
                    + what)
    res = {
        "metric": "NLI pair-integrals/s + 589-ch SNR+gradient wall time, FP32 vs FP64 form, 1 GPU",
        "value": pairs / (ms_step * 1e-3),
        "unit": "pair-integrals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 integrand, f64 phase/accumulation",
        "data": "synthetic (seeded channel plan and fibre tables shaped like the paper's O-to-U system)",
        "config": {"workload": workload, "pairs_per_step": pairs, "grad": bool(grad)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": (rec[0] + rec[1]) if rec else None,
                     "traffic_fetch_write_bytes": [rec[0], rec[1]] if rec else None,
                     "traffic_source": rec[2] if rec else None, "kernel": dominant,
                     "kernel_ms_per_step": dom_ms, "launches_per_step": launches,
                     "node_steps_per_step": node_steps, "slots_per_node_step": dom_slots,
                     "work_count": "formula issue slots per node-step of eq. slow_vary (a transcendental "
                                   "counted as 4 FP32 slots), not the instructions the kernel issues",
                     "traffic_note": ("fabric bytes from rocprofv3 FETCH_SIZE/WRITE_SIZE per launch, mostly the "
                                      "write-back and reload of register spills in the node set-up") if rec else None,
                     "tile_variant": work["variant"]},
        "cpu_baseline": cpu,
        "stages_ms": {k: v / args.steps for k, v in stages.items()},
        "stages_source": "eager warmup call (the timed calls replay one HIP graph)" if graph else "timed calls",
        "graph_mode": graph,
        "snr_wall_ms": (stages["profile"] + stages["tiles"] + stages["reduce"]) / args.steps,
        "node_steps_per_s": node_steps / (tiles_ms * 1e-3),
        "throughput_tbps": thr / 1e12,
        "fp64_form": fp64,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
