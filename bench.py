#!/usr/bin/env python3
"""Benchmark of the SIMUS RF synthesis hot path on one MI355X.

One step = one simus_rf call on the 128-element, 50,000-scatterer plane-wave
workload (pw128_s50k): transmit weights, Green's-tile synthesis with both
contractions, finalisation and the inverse transform to RF, inputs already
resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Issue cost model of the synthesis loop (counted from the gfx950 ISA of
# k_synth<256, 8, 16, 1, false>: instructions per Green's term, see the
# design notes); transcendentals are weighted by their issue cost.
SYNTH_VALU_PER_G = 84          # full-rate VALU instructions per G term
SYNTH_TRANS_PER_G = 13         # transcendental instructions per G term
TRANS_ISSUE_COST = 4.0         # a transcendental issues at 1/4 of the FP32 rate (diag/valu_rate)
# MI355X FP32 vector peak 157.3 TFLOP/s = 78.6e12 FMA lane-instructions/s
# (256 CU x 128 FP32 lanes/clk x 2.4 GHz); one VALU "op" below = one lane slot.
VALU_PEAK = 256 * 128 * 2.4e9


def kernel_sources_digest() -> str:
    h = hashlib.sha256()
    for f in ["kernels.hip", "green.hpp", "kernels.hpp"]:
        with open(os.path.join(ROOT, "paper_2102_02738_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per synthesis launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"synth_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sources") != kernel_sources_digest():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(w, g, x, y, z, R, stride: int):
    """The FP64 oracle on every `stride`-th evaluated bin (all scatterers)."""
    import numpy as np
    from oracle import oracle as O
    from tests.helpers import oracle_setup
    su = oracle_setup(O, w)
    bins = np.arange(g["j_lo"], g["j_lo"] + g["n_bins"], stride, dtype=np.int32)
    t0 = time.perf_counter()
    O.spectrum(su, g["nfft"], w["delays"], w["apod"], x, y, z, R, bins)
    dt = time.perf_counter() - t0
    T = w["delays"].shape[0]
    evals = x.size * w["probe"]["n_elements"] * bins.size * T
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=evals / dt, unit="evals/s", cores=threads, kind="oracle",
                sample=f"{w['name']}: all {x.size} scatterers, every {stride}th of {g['n_bins']} "
                       f"bins ({bins.size} bins), direct FP64 sum, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="pw128_s50k")
    ap.add_argument("--cpu-stride", type=int, default=48)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding of this path is described in the design notes, not built.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 4, "copies": 3}))
        return

    import paper_2102_02738_amd as S
    from paper_2102_02738_amd import _lib, inputs
    from tests.helpers import concat_phantoms

    w = inputs.workload(args.workload)
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g = S.grid(w["probe"], w["medium"], w["options"], w["delays"], x, None, z)
    o = dict(w["options"], nfft=g["nfft"], n_t=g["n_t"])
    dev = torch.device("cuda:0")
    dx, dz, dR = (torch.from_numpy(a).to(dev) for a in (x, z, R))
    T, N = w["delays"].shape
    n_ph = len(w["phantoms"])
    offs = off if n_ph > 1 else None
    out = torch.empty((n_ph, T, N, g["n_t"]), dtype=torch.float32, device=dev)

    def step():
        _lib.rf_into(out, w["probe"], w["medium"], o, w["delays"], w["apod"], dx, None, dz, dR, offs)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    _lib.profile_reset()
    _lib.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _lib.profile_enable(False)
    synth_ms, synth_n = _lib.profile_read("synth")
    other = {k: _lib.profile_read(k) for k in ("wtable", "finalize", "idft")}

    ms_per_step = wall * 1e3 / args.steps
    S_tot = x.size
    evals = S_tot * N * g["n_bins"] * T
    value = evals / (ms_per_step * 1e-3)
    g_terms = S_tot * N * g["nu"] * g["n_bins"]   # each G term serves every transmit
    synth_avg_ms = synth_ms / max(synth_n, 1)
    slots = g_terms * (SYNTH_VALU_PER_G + TRANS_ISSUE_COST * SYNTH_TRANS_PER_G)
    achieved = slots / (synth_avg_ms * 1e-3)
    roof = dict(bound="alu", achieved=achieved / 1e12, peak=VALU_PEAK / 1e12, unit="TOP/s",
                frac=achieved / VALU_PEAK, traffic=measured_traffic(args.workload),
                kernel="k_synth", kernel_ms=synth_avg_ms,
                ops_per_unit=SYNTH_VALU_PER_G + TRANS_ISSUE_COST * SYNTH_TRANS_PER_G,
                unit_count=g_terms, unit_def="G term (sub-element x scatterer x bin)")
    res = {
        "metric": "scatterer*element*freq evals/s", "value": value, "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_elements": N, "n_scatterers": S_tot,
                   "n_tx": T, "n_phantoms": n_ph, "nfft": g["nfft"], "n_bins": g["n_bins"],
                   "n_t": g["n_t"], "nu": g["nu"]},
        "g_terms_per_s": g_terms / (ms_per_step * 1e-3),
        "rf_frames_per_s": n_ph * T / (ms_per_step * 1e-3),
        "kernel_ms": {"synth": synth_avg_ms, **{k: v[0] / max(v[1], 1) for k, v in other.items()}},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, g, x, y, z, R, args.cpu_stride)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
