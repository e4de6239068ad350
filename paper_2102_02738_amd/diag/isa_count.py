#!/usr/bin/env python3
"""Instruction mix of a kernel's innermost loop in the gfx950 assembly of
this library's sources.

Compiles one source file to device assembly with the library's flags, finds
the named kernel, takes the innermost loop (the backward branch with the
shortest body that contains the most VALU instructions among loops of at
least `--min` instructions) and counts its instructions by class.  The
synthesis kernels' roofline uses these counts: full-rate VALU instructions
issue at one lane-slot each, transcendentals (sin, cos, exp, log, rcp, rsq,
sqrt) at four.

    python paper_2102_02738_amd/diag/isa_count.py kernels.hip \
        '_ZN5simus7k_synthILi256ELi8ELi16ELi1ELb0ELi1ELb1EEEvNS_9SynthArgsE' --terms 16
"""
from __future__ import annotations

import argparse
import collections
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "csrc")
INCLUDE = os.path.join(os.path.dirname(os.path.dirname(HERE)), "include")
TRANS = ("v_sin", "v_cos", "v_exp", "v_log", "v_rcp", "v_rsq", "v_sqrt")


def assembly(source: str) -> str:
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    with tempfile.TemporaryDirectory() as td:
        out = os.path.join(td, "k.s")
        cmd = [hipcc, "-x", "hip", "-O3", "-std=c++17", "--offload-arch=gfx950",
               "--offload-device-only", "-Xclang", "-target-feature", "-Xclang",
               "-packed-fp32-ops", f"-I{INCLUDE}", f"-I{CSRC}", "-S",
               os.path.join(CSRC, source), "-o", out]
        subprocess.run(cmd, check=True, stderr=subprocess.DEVNULL)
        return open(out).read()


def loops(body: list[str]):
    labels = {}
    for k, line in enumerate(body):
        m = re.match(r"^(\.LBB\w+):", line)
        if m:
            labels[m.group(1)] = k
    for k, line in enumerate(body):
        m = re.search(r"s_(?:cbranch_\w+|branch)\s+(\.LBB\w+)", line)
        if m and labels.get(m.group(1), k + 1) < k:
            yield labels[m.group(1)], k


def classify(ops: list[str]) -> collections.Counter:
    c = collections.Counter()
    for x in ops:
        if x.startswith(TRANS):
            c["trans"] += 1
        elif x.startswith("v_mfma"):
            c["mfma"] += 1
        elif x.startswith("v_"):
            c["valu"] += 1
        elif x.startswith("ds_"):
            c["lds"] += 1
        elif x.startswith(("global_", "buffer_", "flat_")):
            c["vmem"] += 1
        elif x.startswith("s_waitcnt"):
            c["waitcnt"] += 1
        elif x.startswith("s_barrier"):
            c["barrier"] += 1
        elif x.startswith("s_"):
            c["salu"] += 1
        else:
            c["other"] += 1
    return c


def innermost(asm: str, kernel: str, min_ops: int):
    """Instructions of the kernel's innermost loop (see the module doc)."""
    i = asm.find(kernel + ":")
    if i < 0:
        raise KeyError(kernel)
    body = asm[i:asm.index(".Lfunc_end", i)].split("\n")
    best = None
    for a, b in loops(body):
        ops = [ln.strip().split()[0] for ln in body[a:b + 1]
               if ln.strip() and not ln.strip().startswith((".", ";", "/"))]
        if len(ops) < min_ops:
            continue
        if best is None or len(ops) < len(best):
            best = ops
    return best


def lds_bytes(asm: str, kernel: str) -> int:
    """The kernel's static LDS (group segment) size from the code object
    metadata that hipcc writes into the assembly."""
    for entry in asm.split("\n  - ")[1:]:
        if re.search(r"^\s+\.name:\s+" + re.escape(kernel) + r"\s*$", entry, re.M):
            m = re.search(r"\.group_segment_fixed_size:\s+(\d+)", entry)
            if m:
                return int(m.group(1))
    raise KeyError(kernel)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("source")
    ap.add_argument("kernel", nargs="+", help="mangled kernel name(s)")
    ap.add_argument("--terms", type=int, default=1, help="Green's terms per loop iteration and lane")
    ap.add_argument("--min", type=int, default=100, help="smallest loop body considered")
    args = ap.parse_args()
    s = assembly(args.source)
    for kernel in args.kernel:
        try:
            ops = innermost(s, kernel, args.min)
        except KeyError:
            sys.exit(f"kernel {kernel} not found in {args.source}")
        if ops is None:
            sys.exit(f"no loop found in {kernel}")
        c = classify(ops)
        slots = c["valu"] + 4 * c["trans"]
        print(f"kernel: {kernel}")
        print(f"source: {args.source}")
        print(f"innermost loop: {len(ops)} instructions, {args.terms} Green's terms per iteration and lane")
        for k in sorted(c):
            print(f"  {k:8s} {c[k]:5d}  ({c[k] / args.terms:.2f} per term)")
        print(f"issue slots per term (valu + 4 trans): {slots / args.terms:.2f}")
        print(f"valu_per_term: {c['valu'] / args.terms:.3f}")
        print(f"trans_per_term: {c['trans'] / args.terms:.3f}")
        print(f"lds_bytes: {lds_bytes(s, kernel)}")
        if c["mfma"]:
            print(f"mfma_per_term: {c['mfma'] / args.terms:.3f}")


if __name__ == "__main__":
    main()
