#!/usr/bin/env python3
"""Benchmark of the SIMUS RF synthesis hot path on one MI355X.

Main line: one step = one simus_rf call on the 128-element, 50,000-scatterer
plane-wave workload (pw128_s50k): transmit weights, elevation table,
Green's-tile synthesis with both contractions, finalisation and the inverse
transform to RF, inputs already resident in HBM.  Prints one JSON line.

Extras in the same line (skipped with --no-extras), each against the plain
path (a per-transmit, per-phantom loop of single-transmit calls on the
vector path, no graph):
  batched_transmits   21 plane waves x 200,000 scatterers in one call
                      (transmit and receive contractions on the matrix cores)
  uneven_phantoms     16 convex-probe phantoms of 10k-500k scatterers x 11
                      diverging waves in one persistent launch replayed as a
                      HIP graph
  forward_adjoint     5 plane waves x 100,000 scatterers: forward, residual
                      against a perturbed phantom's RF, adjoint gradients
  two_d               the main workload in 2-D acoustics (Section V), with the
                      synthesis kernel's roofline
  large_t             128 focused transmits of a 64-element phased array,
                      40,000 scatterers (the shape of Fig. 12's sequence)

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-extras]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Issue-cost model of the synthesis kernel this workload runs,
# k_synth<256, 8, 27, 1, false, 1, true, 1>: instructions per Green's term in
# its innermost loop (two bins of 8 scatterers per lane and iteration),
# counted from the gfx950 assembly with paper_2102_02738_amd/diag/isa_count.py.
SYNTH_KERNEL = "_ZN5simus7k_synthILi256ELi8ELi27ELi1ELb0ELi1ELb1ELi1EEEvNS_9SynthArgsE"
SYNTH_TERMS_PER_ITER = 16
SYNTH_VALU_PER_G = 33.0        # full-rate VALU instructions per G term
SYNTH_TRANS_PER_G = 1.0        # transcendental instructions per G term
# The same kernel in 2-D acoustics (no elevation term, so 32-bin tiles fit),
# k_synth<256, 8, 32, 1, false, 2, true, 1>, counted the same way.
SYNTH2D_KERNEL = "_ZN5simus7k_synthILi256ELi8ELi32ELi1ELb0ELi2ELb1ELi1EEEvNS_9SynthArgsE"
SYNTH2D_VALU_PER_G = 17.875
SYNTH2D_TRANS_PER_G = 0.0
TRANS_ISSUE_COST = 4.0         # a transcendental issues at 1/4 of the FP32 rate (diag/valu_rate)
# MI355X FP32 vector peak 157.3 TFLOP/s = 78.6e12 FMA lane-instructions/s
# (256 CU x 128 FP32 lanes/clk x 2.4 GHz); one "slot" = one lane-instruction.
VALU_PEAK = 256 * 128 * 2.4e9
MFMA_FP32_PEAK = 157.3e12      # dense FP32 matrix-core FLOP/s


def kernel_sources_digest() -> str:
    h = hashlib.sha256()
    # the kernel and its launch configuration (items, tiles) decide the traffic
    for f in ["kernels.hip", "green.hpp", "kernels.hpp", "abi.cpp"]:
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


def _sync_ms(fn) -> float:
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3


def _median_ms(fn, steps: int, warmup: int = 1) -> float:
    for _ in range(warmup):
        _sync_ms(fn)
    return statistics.median(_sync_ms(fn) for _ in range(steps))


def _rel(a, b) -> float:
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b).clamp_min(1e-30))


class Case:
    """A workload on the device: scatterers, grid and options."""

    def __init__(self, name: str, flags: int = 0):
        import torch
        from paper_2102_02738_amd import inputs, grid
        self.w = w = inputs.workload(name)
        w["options"] = dict(w["options"], flags=flags)
        self.name = name
        x, y, z, R, off = inputs.concat_phantoms(w["phantoms"])
        self.host = (x, y, z, R)
        self.off = off
        self.g = grid(w["probe"], w["medium"], w["options"], w["delays"], x, None, z)
        self.o = dict(w["options"], nfft=self.g["nfft"], n_t=self.g["n_t"])
        dev = torch.device("cuda:0")
        self.x, self.z, self.R = (torch.from_numpy(a).to(dev) for a in (x, z, R))
        self.T, self.N = w["delays"].shape
        self.P = len(w["phantoms"])
        self.S = x.size
        self.n_t = self.g["n_t"]

    def evals(self) -> float:
        return float(self.S) * self.N * self.g["n_bins"] * self.T

    def offsets(self):
        return self.off if self.P > 1 else None


def extra_batched_transmits(steps: int) -> dict:
    """21 plane waves in one call vs 21 single-transmit calls."""
    import torch
    from paper_2102_02738_amd import _lib, FLAG_NO_MFMA
    c = Case("pw128x21_s200k")
    w = c.w
    out = torch.empty((1, c.T, c.N, c.n_t), device="cuda")
    plain = torch.empty_like(out)

    def batched():
        _lib.rf_into(out, w["probe"], w["medium"], c.o, w["delays"], w["apod"], c.x, None, c.z, c.R)

    po = dict(c.o, flags=FLAG_NO_MFMA)

    def loop():
        for t in range(c.T):
            _lib.rf_into(plain[:, t:t + 1], w["probe"], w["medium"], po, w["delays"][t:t + 1],
                         w["apod"][t:t + 1], c.x, None, c.z, c.R)

    _lib.profile_reset()
    _lib.profile_enable(True)
    b_ms = _median_ms(batched, steps)
    _lib.profile_enable(False)
    synth_ms, n = _lib.profile_read("synth")
    synth_ms /= max(n, 1)
    p_ms = _median_ms(loop, 1, warmup=0)
    # contraction flops (algorithmic, 21 transmits): Tx over nu N sub-elements
    # and Rx over N elements, 8 real flops per complex multiply-add
    flops = 8.0 * c.S * c.g["n_bins"] * c.T * (c.g["nu"] * c.N + c.N)
    return dict(workload=c.name, n_tx=c.T, n_scatterers=c.S, n_bins=c.g["n_bins"],
                batched_ms=b_ms, plain_ms=p_ms, speedup_vs_plain=p_ms / b_ms,
                evals_per_s=c.evals() / (b_ms * 1e-3), rf_frames_per_s=c.T / (b_ms * 1e-3),
                synth_kernel_ms=synth_ms,
                mfma_contraction_tflops=flops / (synth_ms * 1e-3) / 1e12,
                mfma_frac_of_fp32_peak=flops / (synth_ms * 1e-3) / MFMA_FP32_PEAK,
                rel_l2_batched_vs_plain=_rel(out, plain))


def extra_uneven_phantoms(steps: int) -> dict:
    """16 uneven phantoms x 11 diverging waves: one persistent graph launch
    vs a loop of single-phantom, single-transmit calls."""
    import torch
    from paper_2102_02738_amd import _lib, rf_plan, FLAG_PERSISTENT, FLAG_NO_MFMA
    c = Case("cvx128x11_p16")
    w = c.w
    out = torch.empty((c.P, c.T, c.N, c.n_t), device="cuda")
    plain = torch.empty_like(out)
    plan = rf_plan(w["probe"], w["medium"], dict(c.o, flags=FLAG_PERSISTENT), w["delays"], w["apod"],
                   offsets=c.off)

    def graph():
        plan.graph_launch_into(out, c.x, None, c.z, c.R)

    g_ms = _median_ms(graph, steps)
    first = out.clone()
    t0 = time.perf_counter()
    chosen = plan.autotune(c.x, None, c.z, c.R, c.n_t)
    tune_s = time.perf_counter() - t0
    gt_ms = _median_ms(graph, steps)
    tuned = out.clone()
    out.copy_(first)
    static = torch.empty_like(out)
    s_ms = _median_ms(lambda: _lib.rf_into(static, w["probe"], w["medium"], c.o, w["delays"],
                                           w["apod"], c.x, None, c.z, c.R, c.off), 1)
    po = dict(c.o, flags=FLAG_NO_MFMA)
    off = c.off

    def loop():
        for p in range(c.P):
            sl = slice(int(off[p]), int(off[p + 1]))
            for t in range(c.T):
                _lib.rf_into(plain[p:p + 1, t:t + 1], w["probe"], w["medium"], po,
                             w["delays"][t:t + 1], w["apod"][t:t + 1], c.x[sl], None, c.z[sl],
                             c.R[sl])

    p_ms = _median_ms(loop, 1, warmup=0)
    plan.close()
    return dict(workload=c.name, n_phantoms=c.P, n_tx=c.T, n_scatterers=c.S,
                scatterers_min=int(min(off[1:] - off[:-1])), scatterers_max=int(max(off[1:] - off[:-1])),
                graph_ms=g_ms, batched_static_call_ms=s_ms, plain_ms=p_ms,
                speedup_vs_plain=p_ms / min(g_ms, gt_ms), evals_per_s=c.evals() / (min(g_ms, gt_ms) * 1e-3),
                rf_frames_per_s=c.P * c.T / (min(g_ms, gt_ms) * 1e-3),
                autotune=dict(chosen=chosen, tuning_s=tune_s, graph_ms_default=g_ms,
                              graph_ms_autotuned=gt_ms, rel_l2_autotuned_vs_plain=_rel(tuned, plain)),
                rel_l2_graph_vs_plain=_rel(out, plain), graph_equals_static=bool(torch.equal(out, static)))


def extra_autotune(steps: int, name: str) -> dict:
    """A plan for the workload with the default launch shape against the
    same plan after simus_rf_plan_autotune."""
    import torch
    from paper_2102_02738_amd import rf_plan
    c = Case(name)
    w = c.w
    plan = rf_plan(w["probe"], w["medium"], c.o, w["delays"], w["apod"], offsets=c.off)
    out = torch.empty((c.P, c.T, c.N, c.n_t), device="cuda")
    d_ms = _median_ms(lambda: plan.execute_into(out, c.x, None, c.z, c.R), steps)
    first = out.clone()
    t0 = time.perf_counter()
    chosen = plan.autotune(c.x, None, c.z, c.R, c.n_t)
    tune_s = time.perf_counter() - t0
    t_ms = _median_ms(lambda: plan.execute_into(out, c.x, None, c.z, c.R), steps)
    plan.close()
    return dict(workload=name, chosen=chosen, tuning_s=tune_s, default_ms=d_ms, autotuned_ms=t_ms,
                gain=d_ms / t_ms, rel_l2_autotuned_vs_default=_rel(out, first))


def extra_pfield(steps: int) -> dict:
    """simus_pfield on a Fig. 9-like field: 64-element 2.7 MHz phased array
    focused at (10, 60) mm, 256 x 256 points over x in [-40, 40] mm, z in
    [5, 100] mm."""
    import numpy as np
    import torch
    from paper_2102_02738_amd import pfield, pfield_nf
    probe = dict(n_elements=64, fc=2.7e6, pitch=0.3e-3, width=0.25e-3, height=14e-3,
                 elev_focus=60e-3, bandwidth=0.74, radius=0.0, baffle=0, zeta=1.75)
    xe = 0.3e-3 * (np.arange(64) - 31.5)
    d = np.hypot(xe - 10e-3, 60e-3) / 1540.0
    dl = d.max() - d
    X, Z = np.meshgrid(np.linspace(-40e-3, 40e-3, 256), np.linspace(5e-3, 100e-3, 256))
    X, Z = X.ravel().astype(np.float32), Z.ravel().astype(np.float32)
    medium = dict(c=1540.0, alpha_db=0.5)
    options = dict(fs=4 * probe["fc"], n_cycles=1.0, nu=0, spectral_eps=1e-7, nfft=0, n_t=0)
    nf = pfield_nf(probe, medium, options, dl, X, None, Z)
    dX, dZ = (torch.from_numpy(a).cuda() for a in (X, Z))
    apod = np.ones(64, np.float32)
    out = {}

    def call():
        out["p"] = pfield(probe, medium, options, nf, dl, apod, dX, None, dZ)

    ms = _median_ms(call, max(steps, 5))
    from paper_2102_02738_amd import grid
    nu = grid(probe, medium, options, dl[None, :], X[:1], None, Z[:1])["nu"]
    evals = float(X.size) * 64 * nu * (nf + 1)
    return dict(workload="phased64 focused field 256x256", n_points=int(X.size), n_f=int(nf), nu=int(nu),
                ms_per_call=ms, points_per_s=X.size / (ms * 1e-3),
                point_subelement_freq_evals_per_s=evals / (ms * 1e-3),
                finite=bool(torch.isfinite(out["p"]).all()))


def extra_forward_adjoint(steps: int) -> dict:
    """Forward + residual + adjoint of the L2 misfit, 5 plane waves in one
    call each vs a per-transmit loop."""
    import torch
    from paper_2102_02738_amd import _lib, inputs, FLAG_NO_MFMA
    c = Case("pw128x5_s100k")
    w = c.w
    obs = inputs.perturbed(w["phantoms"][0])
    ox, oz, oR = (torch.from_numpy(obs[k]).cuda() for k in ("x", "z", "R"))
    rf_obs = torch.empty((1, c.T, c.N, c.n_t), device="cuda")
    _lib.rf_into(rf_obs, w["probe"], w["medium"], c.o, w["delays"], w["apod"], ox, None, oz, oR)
    out = torch.empty_like(rf_obs)
    grads = {k: torch.empty_like(c.x) for k in ("refl", "x", "z")}

    def fwd():
        _lib.rf_into(out, w["probe"], w["medium"], c.o, w["delays"], w["apod"], c.x, None, c.z, c.R)

    def step():
        fwd()
        res = out - rf_obs
        _lib.rf_backward_into(grads, w["probe"], w["medium"], c.o, w["delays"], w["apod"], c.x, None,
                              c.z, c.R, res)

    f_ms = _median_ms(fwd, steps)
    s_ms = _median_ms(step, steps)
    po = dict(c.o, flags=FLAG_NO_MFMA)
    pg = {k: torch.zeros_like(c.x) for k in grads}
    gt = {k: torch.empty_like(c.x) for k in grads}
    o1 = torch.empty((1, 1, c.N, c.n_t), device="cuda")

    def loop():
        for v in pg.values():
            v.zero_()
        for t in range(c.T):
            d, a = w["delays"][t:t + 1], w["apod"][t:t + 1]
            _lib.rf_into(o1, w["probe"], w["medium"], po, d, a, c.x, None, c.z, c.R)
            res = o1 - rf_obs[:, t:t + 1]
            _lib.rf_backward_into(gt, w["probe"], w["medium"], po, d, a, c.x, None, c.z, c.R, res)
            for k in pg:
                pg[k] += gt[k]

    p_ms = _median_ms(loop, 1)
    return dict(workload=c.name, n_tx=c.T, n_scatterers=c.S, forward_ms=f_ms, forward_adjoint_ms=s_ms,
                plain_forward_adjoint_ms=p_ms, speedup_vs_plain=p_ms / s_ms,
                rf_frames_per_s_forward=c.T / (f_ms * 1e-3),
                rf_frames_per_s_forward_adjoint=c.T / (s_ms * 1e-3),
                rel_l2_grad_vs_plain={k: _rel(grads[k], pg[k]) for k in grads})


def extra_large_t(steps: int) -> dict:
    """128 focused transmits in one call vs 128 single-transmit calls."""
    import torch
    from paper_2102_02738_amd import _lib, FLAG_NO_MFMA
    c = Case("ph64x128_s40k")
    w = c.w
    out = torch.empty((1, c.T, c.N, c.n_t), device="cuda")
    plain = torch.empty_like(out)

    def batched():
        _lib.rf_into(out, w["probe"], w["medium"], c.o, w["delays"], w["apod"], c.x, None, c.z, c.R)

    po = dict(c.o, flags=FLAG_NO_MFMA)

    def loop():
        for t in range(c.T):
            _lib.rf_into(plain[:, t:t + 1], w["probe"], w["medium"], po, w["delays"][t:t + 1],
                         w["apod"][t:t + 1], c.x, None, c.z, c.R)

    b_ms = _median_ms(batched, steps)
    p_ms = _median_ms(loop, 1)
    return dict(workload=c.name, n_tx=c.T, n_elements=c.N, n_scatterers=c.S, n_bins=c.g["n_bins"],
                batched_ms=b_ms, plain_ms=p_ms, speedup_vs_plain=p_ms / b_ms,
                evals_per_s=c.evals() / (b_ms * 1e-3), rf_frames_per_s=c.T / (b_ms * 1e-3),
                rel_l2_batched_vs_plain=_rel(out, plain))


def extra_two_d(steps: int, ms_3d: float) -> dict:
    """The main workload in 2-D acoustics: no elevation term, 1/sqrt(r)
    spreading (Section V)."""
    import torch
    from paper_2102_02738_amd import _lib, FLAG_2D
    c = Case("pw128_s50k", flags=FLAG_2D)
    w = c.w
    out = torch.empty((1, c.T, c.N, c.n_t), device="cuda")

    def step():
        _lib.rf_into(out, w["probe"], w["medium"], c.o, w["delays"], w["apod"], c.x, None, c.z, c.R)

    _lib.profile_reset()
    _lib.profile_enable(True)
    ms = _median_ms(step, steps * 5, warmup=2)
    _lib.profile_enable(False)
    synth_ms, n = _lib.profile_read("synth")
    synth_ms /= max(n, 1)
    g_terms = float(c.S) * c.N * c.g["nu"] * c.g["n_bins"]
    per_g = SYNTH2D_VALU_PER_G + TRANS_ISSUE_COST * SYNTH2D_TRANS_PER_G
    achieved = g_terms * per_g / (synth_ms * 1e-3)
    return dict(workload=c.name + " (2-D)", ms_per_call=ms, evals_per_s=c.evals() / (ms * 1e-3),
                speedup_vs_3d=ms_3d / ms if ms_3d == ms_3d else None, synth_kernel_ms=synth_ms,
                roofline=dict(bound="alu", achieved=achieved / 1e12, peak=VALU_PEAK / 1e12,
                              unit="TOP/s", frac=achieved / VALU_PEAK,
                              kernel="k_synth<256, 8, 32, 1, false, 2, true, 1>", ops_per_unit=per_g))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-stride", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extra-steps", type=int, default=2)
    ap.add_argument("--only-extra", default="",
                    help="run only this extra measurement and print its JSON (for profiling)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding of this path is described in the design notes, not built.",
              file=sys.stderr)
        sys.exit(2)

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

    from paper_2102_02738_amd import _lib

    if args.only_extra:
        fns = {"autotune": lambda k: extra_autotune(max(k, 5), "pw128_s50k"),
               "batched_transmits": extra_batched_transmits, "uneven_phantoms": extra_uneven_phantoms,
               "forward_adjoint": extra_forward_adjoint, "large_t": extra_large_t,
               "pfield": extra_pfield,
               "two_d": lambda k: extra_two_d(k, float("nan"))}
        if args.only_extra not in fns:
            print(f"unknown extra {args.only_extra!r}; one of {sorted(fns)}", file=sys.stderr)
            sys.exit(2)
        print(json.dumps({args.only_extra: fns[args.only_extra](args.extra_steps)}))
        return

    c = Case("pw128_s50k")
    w = c.w
    out = torch.empty((c.P, c.T, c.N, c.n_t), dtype=torch.float32, device="cuda")

    def step():
        _lib.rf_into(out, w["probe"], w["medium"], c.o, w["delays"], w["apod"], c.x, None, c.z, c.R,
                     c.offsets())

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
    value = c.evals() / (ms_per_step * 1e-3)
    g_terms = float(c.S) * c.N * c.g["nu"] * c.g["n_bins"]   # each G term serves every transmit
    synth_avg_ms = synth_ms / max(synth_n, 1)
    per_g = SYNTH_VALU_PER_G + TRANS_ISSUE_COST * SYNTH_TRANS_PER_G
    achieved = g_terms * per_g / (synth_avg_ms * 1e-3)
    roof = dict(bound="alu", achieved=achieved / 1e12, peak=VALU_PEAK / 1e12, unit="TOP/s",
                frac=achieved / VALU_PEAK, traffic=measured_traffic(c.name),
                kernel="k_synth<256, 8, 27, 1, false, 1, true, 1>", kernel_ms=synth_avg_ms,
                ops_per_unit=per_g, valu_per_unit=SYNTH_VALU_PER_G, trans_per_unit=SYNTH_TRANS_PER_G,
                unit_count=g_terms, unit_def="G term (sub-element x scatterer x bin)",
                op_def="lane issue slot: full-rate VALU 1, transcendental 4")
    res = {
        "metric": "scatterer*element*freq evals/s", "value": value, "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": c.name, "n_elements": c.N, "n_scatterers": c.S,
                   "n_tx": c.T, "n_phantoms": c.P, "nfft": c.g["nfft"], "n_bins": c.g["n_bins"],
                   "n_t": c.n_t, "nu": c.g["nu"]},
        "g_terms_per_s": g_terms / (ms_per_step * 1e-3),
        "rf_frames_per_s": c.P * c.T / (ms_per_step * 1e-3),
        "kernel_ms": {"synth": synth_avg_ms, **{k: v[0] / max(v[1], 1) for k, v in other.items()}},
        "roofline": roof,
    }
    if not args.no_extras:
        res["extras"] = {
            "autotune": extra_autotune(max(args.extra_steps, 5), c.name),
            "batched_transmits": extra_batched_transmits(args.extra_steps),
            "uneven_phantoms": extra_uneven_phantoms(args.extra_steps),
            "forward_adjoint": extra_forward_adjoint(args.extra_steps),
            "two_d": extra_two_d(args.extra_steps, ms_per_step),
            "large_t": extra_large_t(args.extra_steps),
            "pfield": extra_pfield(args.extra_steps),
        }
    if not args.no_cpu_baseline:
        x, y, z, R = c.host
        res["cpu_baseline"] = cpu_baseline(w, c.g, x, y, z, R, args.cpu_stride)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
