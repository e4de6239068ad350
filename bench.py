#!/usr/bin/env python3
"""Benchmark of the SIMUS RF synthesis hot path on one MI355X.

Main line: one step = one replay of the persistent HIP graph of a simus_rf
plan on the batched uneven-phantom workload (cvx128x11_p16): a convex
128-element array, 11 diverging waves, 16 phantoms of 10k-390k scatterers
(2.27 M in all).  A step runs every row of the path: transmit weights,
elevation table, Green's-tile synthesis with both contractions on the
matrix cores, finalisation and the inverse transform to RF, with the inputs
already resident in HBM.  The plan (host planning, upload) is built once
before the timed region; one whole simus_rf call is timed beside it.
Prints one JSON line.

Extras in the same line (skipped with --no-extras), each against the plain
path (a per-transmit, per-phantom loop of single-transmit calls on the
vector path, no graph) where one exists:
  single_transmit     the 128-element, 50,000-scatterer plane wave on the
                      vector path (k_synth), with its roofline
  autotune            the autotuner on the single-transmit and the uneven
                      workloads
  batched_transmits   21 plane waves x 200,000 scatterers in one call
  uneven_phantoms     the main workload against its plain loop
  forward_adjoint     5 plane waves x 100,000 scatterers: forward, residual
                      against a perturbed phantom's RF, adjoint gradients
  two_d               the single-transmit workload in 2-D acoustics
  large_t             128 focused transmits of a 64-element phased array,
                      40,000 scatterers (the shape of Fig. 12's sequence)
  pfield              the RMS field of a Fig. 9-like focused phased array

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

# Algorithmic work of the path, in lane issue slots of the FP32 vector unit
# (a full-rate VALU lane-instruction is one slot, a transcendental four; an
# FP32 MFMA lane-MAC is one slot as well, since the FP32 matrix rate equals
# the FP32 FMA rate on gfx950: 157.3 TFLOP/s each).  Counted from the
# formulas the library evaluates, not from the instructions its kernels
# issue: no pair set-up (it is amortised over a tile of bins), no address
# arithmetic, no padding of transmit groups, no waits.
#   One Green's term (Eqs. 10, 14-20, 39-40 by the bin recurrences and the
#   elevation table): q = j kappa (1); table coordinate r = rcp(|b| dw + 1)
#   (1 + 4), u = med3(fma(b, r, u0)) (2), interval and fraction (2); the
#   complex cubic (6); A = E s (2); G = A delta (4); rotor E dE (4); sinc
#   recurrence (2): 28 slots.
G_EVAL_SLOTS = 28.0
#   Element sum of Eqs. 32-33 for nu = 2: one complex add per element, i.e.
#   one slot per G term ((nu - 1) / nu * 2 in general).
#   The two contractions (Eq. 29 over elements after the sum, Eq. 33): two
#   complex MACs per (element, scatterer, transmit, bin).  On the matrix
#   cores each takes 12 bf16 MACs: 4 real products in FP32 accuracy, as three
#   products of bf16 high and low parts each; at the dense bf16 peak (2.5
#   PFLOP/s = 1.25e15 MAC/s) a bf16 MAC costs 78.64e12 / 1.25e15 = 0.0629
#   slots, so 0.755 slots per complex MAC.  With FP32 matrix-core products
#   (three-product form, SIMUS_FLAG_FP32_PRODUCTS): 3 slots; on the VALU: 4.
BF16_MAC_SLOTS = 256 * 128 * 2.4e9 / 1.25e15
CMAC_SLOTS_MFMA = 12 * BF16_MAC_SLOTS
CMAC_SLOTS_MFMA_FP32 = 3.0
CMAC_SLOTS_VALU = 4.0


def alg_slots(S: float, M: int, N: int, T: int, n_bins: int, nu: int, mfma: bool, cmac: float = None) -> float:
    """Algorithmic issue slots of one synthesis over S scatterers (see above)."""
    g_terms = S * M * n_bins
    per_g = G_EVAL_SLOTS + 2.0 * (nu - 1) / nu
    cm = cmac if cmac is not None else CMAC_SLOTS_MFMA if mfma else CMAC_SLOTS_VALU
    return g_terms * per_g + 2.0 * S * N * T * n_bins * cm + 2.0 * S * T * n_bins


# Instruction count of the single-transmit vector kernel,
# k_synth<256, 8, 27, 1, false, 1, true, 1>: instructions per Green's term in
# its innermost loop (two bins of 8 scatterers per lane and iteration),
# counted from the gfx950 assembly with paper_2102_02738_amd/diag/isa_count.py
# (its issue count, beside the algorithmic count above).
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
# The main workload's synthesis kernel (one group of 16 transmit columns,
# 128 element slots, 8 bins per item, split-bf16 products, nu = 2, y = 0,
# elevation table).
MT_KERNEL = "k_synth_mb<128, 2, false, true>"


def kernel_sources_digest(files) -> str:
    h = hashlib.sha256()
    # the kernel and its launch configuration (items, tiles) decide the counts
    for f in files:
        with open(os.path.join(ROOT, "paper_2102_02738_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


VECTOR_SOURCES = ["kernels.hip", "green.hpp", "kernels.hpp", "abi.cpp"]
MT_SOURCES = ["synth_mfma.hip", "green.hpp", "kernels.hpp", "abi.cpp"]


def profile_summary(name: str, files) -> dict:
    """key: value lines of a committed rocprofv3 summary under profiles/, if
    it was taken on the current kernel sources (else {})."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return {}
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sources") != kernel_sources_digest(files):
        return {}
    return vals


def measured_traffic(name: str, files):
    """HBM bytes per synthesis launch from a committed counter summary."""
    try:
        return float(profile_summary(name, files)["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, g, x, y, z, R, off, bin_stride: int, scat_stride: int):
    """The FP64 oracle, as it stands, on a bounded sample of the workload:
    every `bin_stride`-th evaluated bin and every `scat_stride`-th scatterer
    of each phantom, all transmits and elements.  Its cost is linear in
    scatterers and bins, so the rate (evals/s) stands for the whole job."""
    import numpy as np
    from oracle import oracle as O
    from tests.helpers import oracle_setup
    su = oracle_setup(O, w)
    bins = np.arange(g["j_lo"], g["j_lo"] + g["n_bins"], bin_stride, dtype=np.int32)
    t0 = time.perf_counter()
    n_s = 0
    for p in range(len(off) - 1):
        sl = slice(int(off[p]), int(off[p + 1]), scat_stride)
        if x[sl].size == 0:
            continue
        n_s += x[sl].size
        O.spectrum(su, g["nfft"], w["delays"], w["apod"], x[sl], y[sl], z[sl], R[sl], bins)
    dt = time.perf_counter() - t0
    T = w["delays"].shape[0]
    evals = n_s * w["probe"]["n_elements"] * bins.size * T
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=evals / dt, unit="evals/s", cores=threads, cpu_model=cpu_model(), kind="oracle",
                sample=f"{w['name']}: every {scat_stride}th scatterer of each of {len(off) - 1} phantoms "
                       f"({n_s} of {x.size}), every {bin_stride}th of {g['n_bins']} bins ({bins.size}), "
                       f"{T} transmits, direct FP64 sum, {dt:.1f} s")


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
    # contraction flops: Tx (Eq. 29, over elements after the element sum) and
    # Rx (Eq. 33), 8 real flops per complex multiply-add
    flops = 8.0 * c.S * c.g["n_bins"] * c.T * 2 * c.N
    alg = alg_slots(c.S, c.g["nu"] * c.N, c.N, c.T, c.g["n_bins"], c.g["nu"], True)
    return dict(workload=c.name, n_tx=c.T, n_scatterers=c.S, n_bins=c.g["n_bins"],
                batched_ms=b_ms, plain_ms=p_ms, speedup_vs_plain=p_ms / b_ms,
                evals_per_s=c.evals() / (b_ms * 1e-3), rf_frames_per_s=c.T / (b_ms * 1e-3),
                synth_kernel_ms=synth_ms,
                roofline=dict(bound="alu", achieved=alg / (synth_ms * 1e-3) / 1e12,
                              peak=VALU_PEAK / 1e12, unit="TOP/s",
                              frac=alg / (synth_ms * 1e-3) / VALU_PEAK),
                contraction_tflops=flops / (synth_ms * 1e-3) / 1e12,
                rel_l2_batched_vs_plain=_rel(out, plain))


def extra_uneven_phantoms(steps: int) -> dict:
    """The main workload's plan against a loop of single-phantom,
    single-transmit calls (vector path, no graph), and the autotuner on it."""
    import torch
    from paper_2102_02738_amd import _lib, rf_plan, FLAG_NO_MFMA
    c = Case("cvx128x11_p16")
    w = c.w
    out = torch.empty((c.P, c.T, c.N, c.n_t), device="cuda")
    plain = torch.empty_like(out)
    plan = rf_plan(w["probe"], w["medium"], c.o, w["delays"], w["apod"], offsets=c.off)

    def graph():
        plan.graph_launch_into(out, c.x, None, c.z, c.R)

    g_ms = _median_ms(graph, steps)
    first = out.clone()
    plan.close()
    plan, info = _autotune_cached(
        lambda: rf_plan(w["probe"], w["medium"], c.o, w["delays"], w["apod"], offsets=c.off),
        lambda p: p.autotune(c.x, None, c.z, c.R))
    gt_ms = _median_ms(graph, steps)
    tuned = out.clone()
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
    return dict(workload=c.name, graph_ms=g_ms, plain_ms=p_ms, speedup_vs_plain=p_ms / g_ms,
                autotune=dict(**info, graph_ms_default=g_ms, graph_ms_autotuned=gt_ms,
                              gain=g_ms / gt_ms, rel_l2_autotuned_vs_plain=_rel(tuned, plain)),
                rel_l2_graph_vs_plain=_rel(first, plain))


AUTOTUNE_SPACE = ("the distinct tile shapes of the default rule and SIMUS_FLAG_ALT_SHAPE (kernel, "
                  "element slots, transmit columns, bins per item) x "
                  "scatterers per item 0.5/1/2x the default (vector path also 1.5x, and static or "
                  "persistent launch)")


def _autotune_cached(make_plan, tune):
    """Tunes a first plan with an empty file cache (timed), then a second plan
    of the same problem class (answered from the cache)."""
    import tempfile
    import paper_2102_02738_amd as S
    with tempfile.TemporaryDirectory() as td:
        S.tune_cache(os.path.join(td, "tune.txt"))
        try:
            plan = make_plan()
            t0 = time.perf_counter()
            chosen = tune(plan)
            tune_s = time.perf_counter() - t0
            hits = S.tune_cache_hits()
            plan2 = make_plan()
            t0 = time.perf_counter()
            chosen2 = tune(plan2)
            cached_s = time.perf_counter() - t0
            assert S.tune_cache_hits() == hits + 1 and chosen2 == chosen
            plan2.close()
        finally:
            S.tune_cache(None)
    return plan, dict(chosen=chosen, tuning_s=tune_s, cached_tuning_s=cached_s, search_space=AUTOTUNE_SPACE)


def extra_autotune(steps: int, name: str) -> dict:
    """A plan for the workload with the default launch shape against a plan
    after simus_rf_plan_autotune (with the file cache: the tuning time, then
    the time of a second plan's autotune answered from the cache)."""
    import torch
    from paper_2102_02738_amd import rf_plan
    c = Case(name)
    w = c.w
    make = lambda: rf_plan(w["probe"], w["medium"], c.o, w["delays"], w["apod"], offsets=c.off)
    plan0 = make()
    out = torch.empty((c.P, c.T, c.N, c.n_t), device="cuda")
    d_ms = _median_ms(lambda: plan0.execute_into(out, c.x, None, c.z, c.R), steps)
    first = out.clone()
    plan0.close()
    plan, info = _autotune_cached(make, lambda p: p.autotune(c.x, None, c.z, c.R, c.n_t))
    t_ms = _median_ms(lambda: plan.execute_into(out, c.x, None, c.z, c.R), steps)
    plan.close()
    return dict(workload=name, **info, default_ms=d_ms, autotuned_ms=t_ms,
                gain=d_ms / t_ms, rel_l2_autotuned_vs_default=_rel(out, first))


# Algorithmic work of the field (Eqs. 22 and 42), in the same lane issue
# slots: per (point, sub-element, frequency) one Green's term (28, as above)
# and its complex MAC with the transmit weight (4); per (point, frequency)
# the product with P_Tx (4), |.|^2 (2) and the 1/j^2 scaling (1).
PF_TERM_SLOTS = G_EVAL_SLOTS + 4.0
PF_POINT_BIN_SLOTS = 7.0


def _pfield_case(workload: str, probe: dict, dl, X, Z, steps: int) -> dict:
    import numpy as np
    import torch
    from paper_2102_02738_amd import _lib, grid, pfield, pfield_nf
    medium = dict(c=1540.0, alpha_db=0.5)
    options = dict(fs=4 * probe["fc"], n_cycles=1.0, nu=0, spectral_eps=1e-7, nfft=0, n_t=0)
    nf = pfield_nf(probe, medium, options, dl, X, None, Z)
    dX, dZ = (torch.from_numpy(a).cuda() for a in (X, Z))
    apod = np.ones(probe["n_elements"], np.float32)
    out = {}

    def call():
        out["p"] = pfield(probe, medium, options, nf, dl, apod, dX, None, dZ)

    ms = _median_ms(call, max(steps, 5))
    # the field kernel alone: HIP events around its launches, on its stream
    _lib.profile_reset()
    _lib.profile_enable(True)
    for _ in range(max(steps, 5)):
        call()
    torch.cuda.synchronize()
    _lib.profile_enable(False)
    k_ms, k_n = _lib.profile_read("pfield")
    k_ms /= max(k_n, 1)
    nu = grid(probe, medium, options, dl[None, :], X[:1], None, Z[:1])["nu"]
    M = nu * probe["n_elements"]
    evals = float(X.size) * M * nf                  # j = 1 .. N_f (j = 0 adds nothing)
    alg = evals * PF_TERM_SLOTS + float(X.size) * nf * PF_POINT_BIN_SLOTS
    return dict(workload=workload, n_points=int(X.size), n_f=int(nf), nu=int(nu),
                ms_per_call=ms, points_per_s=X.size / (ms * 1e-3),
                point_subelement_freq_evals_per_s=evals / (ms * 1e-3),
                kernel_ms=k_ms,
                roofline=dict(bound="alu", achieved=alg / (k_ms * 1e-3) / 1e12, peak=VALU_PEAK / 1e12,
                              unit="TOP/s", frac=alg / (k_ms * 1e-3) / VALU_PEAK, traffic=None,
                              kernel="k_pfield<24, false, true>",
                              work_per_unit=dict(term=PF_TERM_SLOTS, point_bin=PF_POINT_BIN_SLOTS)),
                finite=bool(torch.isfinite(out["p"]).all()))


def extra_pfield_fig9(steps: int) -> dict:
    """Fig. 9-like field: 64-element 2.7 MHz phased array focused at (10, 60)
    mm, 256 x 256 points over x in [-40, 40] mm, z in [5, 100] mm."""
    import numpy as np
    probe = dict(n_elements=64, fc=2.7e6, pitch=0.3e-3, width=0.25e-3, height=14e-3,
                 elev_focus=60e-3, bandwidth=0.74, radius=0.0, baffle=0, zeta=1.75)
    xe = 0.3e-3 * (np.arange(64) - 31.5)
    d = np.hypot(xe - 10e-3, 60e-3) / 1540.0
    dl = d.max() - d
    X, Z = np.meshgrid(np.linspace(-40e-3, 40e-3, 256), np.linspace(5e-3, 100e-3, 256))
    X, Z = X.ravel().astype(np.float32), Z.ravel().astype(np.float32)
    return _pfield_case("phased64 focused field 256x256", probe, dl, X, Z, steps)


def extra_pfield_fig10(steps: int) -> dict:
    """Fig. 10-like field: 128-element 7.6 MHz linear array (pitch 0.27 mm,
    kerf 30 um), one plane wave tilted by 10 degrees, 256 x 256 points over x
    in [-25, 25] mm, z in [1, 50] mm."""
    import numpy as np
    from paper_2102_02738_amd import inputs
    lin = dict(inputs.linear_probe(128), pitch=0.27e-3, width=0.24e-3)
    dl = inputs.plane_wave_delays(lin, [10.0])[0]
    X, Z = np.meshgrid(np.linspace(-25e-3, 25e-3, 256), np.linspace(1e-3, 50e-3, 256))
    X, Z = X.ravel().astype(np.float32), Z.ravel().astype(np.float32)
    return _pfield_case("linear128 plane-wave field 256x256", lin, dl, X, Z, steps)


def extra_pfield(steps: int) -> dict:
    """simus_pfield on the two field shapes above (the Fig. 9 one first)."""
    res = extra_pfield_fig9(steps)
    res["linear128_plane_wave"] = extra_pfield_fig10(steps)
    return res


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


def extra_single_transmit(steps: int) -> dict:
    """One 0-degree plane wave, 128 elements, 50,000 scatterers on the vector
    path (k_synth), whole simus_rf calls, with the synthesis kernel's
    roofline: algorithmic slots, and the issue count of its bin loop."""
    import torch
    from paper_2102_02738_amd import _lib
    c = Case("pw128_s50k")
    w = c.w
    out = torch.empty((c.P, c.T, c.N, c.n_t), dtype=torch.float32, device="cuda")

    def step():
        _lib.rf_into(out, w["probe"], w["medium"], c.o, w["delays"], w["apod"], c.x, None, c.z, c.R)

    for _ in range(3):
        step()
    _lib.profile_reset()
    _lib.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    _lib.profile_enable(False)
    synth_ms, n = _lib.profile_read("synth")
    synth_ms /= max(n, 1)
    g_terms = float(c.S) * c.N * c.g["nu"] * c.g["n_bins"]
    alg = alg_slots(c.S, c.g["nu"] * c.N, c.N, c.T, c.g["n_bins"], c.g["nu"], False)
    issue = g_terms * (SYNTH_VALU_PER_G + TRANS_ISSUE_COST * SYNTH_TRANS_PER_G)
    return dict(workload=c.name, ms_per_call=ms, evals_per_s=c.evals() / (ms * 1e-3),
                g_terms_per_s=g_terms / (ms * 1e-3), rf_frames_per_s=c.T / (ms * 1e-3),
                synth_kernel_ms=synth_ms,
                roofline=dict(bound="alu", achieved=alg / (synth_ms * 1e-3) / 1e12,
                              peak=VALU_PEAK / 1e12, unit="TOP/s",
                              frac=alg / (synth_ms * 1e-3) / VALU_PEAK,
                              traffic=measured_traffic("synth_pw128_s50k_traffic.txt", VECTOR_SOURCES),
                              kernel="k_synth<256, 8, 27, 1, false, 1, true, 1>",
                              bin_loop_issue_frac=issue / (synth_ms * 1e-3) / VALU_PEAK))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-bin-stride", type=int, default=32)
    ap.add_argument("--cpu-scat-stride", type=int, default=100)
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

    from paper_2102_02738_amd import _lib, rf_plan

    if args.only_extra:
        fns = {"autotune": lambda k: extra_autotune(max(k, 5), "pw128_s50k"),
               "autotune_batched": lambda k: extra_autotune(max(k, 3), "pw128x21_s200k"),
               "single_transmit": lambda k: extra_single_transmit(max(k, 5)),
               "batched_transmits": extra_batched_transmits, "uneven_phantoms": extra_uneven_phantoms,
               "forward_adjoint": extra_forward_adjoint, "large_t": extra_large_t,
               "pfield": extra_pfield, "pfield_fig9": extra_pfield_fig9,
               "pfield_fig10": extra_pfield_fig10,
               "two_d": lambda k: extra_two_d(k, float("nan"))}
        if args.only_extra not in fns:
            print(f"unknown extra {args.only_extra!r}; one of {sorted(fns)}", file=sys.stderr)
            sys.exit(2)
        print(json.dumps({args.only_extra: fns[args.only_extra](args.extra_steps)}))
        return

    c = Case("cvx128x11_p16")
    w = c.w
    out = torch.empty((c.P, c.T, c.N, c.n_t), dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    plan = rf_plan(w["probe"], w["medium"], c.o, w["delays"], w["apod"], offsets=c.off)
    plan_s = time.perf_counter() - t0

    def step():
        plan.graph_launch_into(out, c.x, None, c.z, c.R)

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
    graph_ms, graph_n = _lib.profile_read("graph")
    graph_ms /= max(graph_n, 1)
    # the same kernels launched one by one (plan execution), each bracketed by
    # HIP events on the launch stream: the synthesis kernel's duration and
    # the rest of the graph's
    _lib.profile_reset()
    _lib.profile_enable(True)
    eager = torch.empty_like(out)
    for _ in range(2):
        plan.execute_into(eager, c.x, None, c.z, c.R)
    torch.cuda.synchronize()
    _lib.profile_enable(False)
    kern = {k: _lib.profile_read(k) for k in ("synth", "wtable", "finalize", "idft")}
    kern = {k: v[0] / max(v[1], 1) for k, v in kern.items()}
    graph_equals_eager = bool(torch.equal(out, eager))
    # one whole simus_rf call (host planning, upload and the same kernels)
    call = torch.empty_like(out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _lib.rf_into(call, w["probe"], w["medium"], c.o, w["delays"], w["apod"], c.x, None, c.z, c.R, c.off)
    torch.cuda.synchronize()
    call_ms = (time.perf_counter() - t0) * 1e3
    plan.close()

    ms_per_step = wall * 1e3 / args.steps
    value = c.evals() / (ms_per_step * 1e-3)
    M = c.g["nu"] * c.N
    g_terms = float(c.S) * M * c.g["n_bins"]
    # the synthesis kernel inside the timed graph launches: the graph's event
    # time less the other kernels' (measured eagerly; < 0.1 %)
    synth_ms = graph_ms - (kern["wtable"] + kern["finalize"] + kern["idft"])
    alg = alg_slots(c.S, M, c.N, c.T, c.g["n_bins"], c.g["nu"], True)
    alg_fp32 = alg_slots(c.S, M, c.N, c.T, c.g["n_bins"], c.g["nu"], True, CMAC_SLOTS_MFMA_FP32)
    achieved = alg / (synth_ms * 1e-3)
    counters = profile_summary("synth_mt_cvx128x11_p16_counters.txt", MT_SOURCES)
    roof = dict(bound="alu", achieved=achieved / 1e12, peak=VALU_PEAK / 1e12, unit="TOP/s",
                frac=achieved / VALU_PEAK,
                traffic=measured_traffic("synth_mt_cvx128x11_p16_traffic.txt", MT_SOURCES),
                kernel=MT_KERNEL, kernel_ms=synth_ms, kernel_ms_eager=kern["synth"],
                unit_count=dict(g_terms=g_terms, cmac_pairs=float(c.S) * c.N * c.T * c.g["n_bins"]),
                work_per_unit=dict(g_term=G_EVAL_SLOTS + 2.0 * (c.g["nu"] - 1) / c.g["nu"],
                                   cmac_pair=2 * CMAC_SLOTS_MFMA),
                work_def="algorithmic lane issue slots: Green's term by recurrence and table, element "
                         "sum, two complex MACs per (element, scatterer, transmit, bin) on the bf16 "
                         "matrix cores (12 bf16 MACs each: FP32 accuracy from high and low parts); no "
                         "set-up, padding or address arithmetic",
                op_def="lane issue slot: full-rate FP32 VALU 1, transcendental 4, bf16 MFMA MAC "
                       "78.64e12 / 1.25e15 = 0.0629 (dense peaks)",
                frac_fp32_products_model=alg_fp32 / (synth_ms * 1e-3) / VALU_PEAK,
                issue_counters={k: float(counters[k]) for k in ("valu_busy", "mfma_busy", "issue_busy")
                                if k in counters} or None)
    res = {
        "metric": "scatterer*element*freq evals/s", "value": value, "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": c.name, "n_elements": c.N, "n_scatterers": c.S, "n_tx": c.T,
                   "n_phantoms": c.P, "nfft": c.g["nfft"], "n_bins": c.g["n_bins"], "n_t": c.n_t,
                   "nu": c.g["nu"], "launch": "one persistent hipGraph replay per step (plan built once)"},
        "g_terms_per_s": g_terms / (ms_per_step * 1e-3),
        "rf_frames_per_s": c.P * c.T / (ms_per_step * 1e-3),
        "plan_create_s": plan_s, "simus_rf_call_ms": call_ms,
        "simus_rf_call_evals_per_s": c.evals() / (call_ms * 1e-3),
        "graph_equals_eager": graph_equals_eager, "rel_l2_call_vs_graph": _rel(call, out),
        "kernel_ms": {"graph": graph_ms, **kern},
        "roofline": roof,
    }
    if not args.no_extras:
        st = extra_single_transmit(max(args.extra_steps * 5, 10))
        res["extras"] = {
            "single_transmit": st,
            "autotune": extra_autotune(max(args.extra_steps, 5), "pw128_s50k"),
            "autotune_batched": extra_autotune(max(args.extra_steps, 3), "pw128x21_s200k"),
            "batched_transmits": extra_batched_transmits(args.extra_steps),
            "uneven_phantoms": extra_uneven_phantoms(args.extra_steps),
            "forward_adjoint": extra_forward_adjoint(args.extra_steps),
            "two_d": extra_two_d(args.extra_steps, st["ms_per_call"]),
            "large_t": extra_large_t(args.extra_steps),
            "pfield": extra_pfield(args.extra_steps),
        }
    if not args.no_cpu_baseline:
        x, y, z, R = c.host
        res["cpu_baseline"] = cpu_baseline(w, c.g, x, y, z, R, c.off, args.cpu_bin_stride,
                                           args.cpu_scat_stride)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
