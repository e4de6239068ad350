"""The issue-cost constants of bench.py's roofline are the instruction mix of
the synthesis kernel the benchmark runs, re-counted here from the gfx950
assembly of the current sources (hipcc cross-compiles without a GPU)."""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_bench_cost_constants_match_isa():
    sys.path.insert(0, ROOT)
    import bench
    out = subprocess.run([sys.executable, os.path.join(ROOT, "paper_2102_02738_amd", "diag", "isa_count.py"),
                          "kernels.hip", bench.SYNTH_KERNEL, bench.SYNTH2D_KERNEL,
                          "--terms", str(bench.SYNTH_TERMS_PER_ITER)],
                         check=True, capture_output=True, text=True).stdout
    valu = [float(v) for v in re.findall(r"valu_per_term: ([0-9.]+)", out)]
    trans = [float(v) for v in re.findall(r"trans_per_term: ([0-9.]+)", out)]
    assert len(valu) == len(trans) == 2, out
    assert valu[0] == pytest.approx(bench.SYNTH_VALU_PER_G, abs=1e-3), out
    assert trans[0] == pytest.approx(bench.SYNTH_TRANS_PER_G, abs=1e-3), out
    assert valu[1] == pytest.approx(bench.SYNTH2D_VALU_PER_G, abs=1e-3), out
    assert trans[1] == pytest.approx(bench.SYNTH2D_TRANS_PER_G, abs=1e-3), out
    # the benchmark's kernel keeps three blocks per CU (LDS in 2 KiB granules
    # of 160 KiB), and one more bin of paired accumulators (1 KiB) would not
    lds = [int(v) for v in re.findall(r"lds_bytes: (\d+)", out)]
    limit = 163840 // 3 // 2048 * 2048
    assert lds[0] <= limit < lds[0] + 1024, (lds, limit)

def test_benchmark_instantiation_is_the_one_counted():
    """pw128_s50k (128 elements, nu = 2, one transmit, y = 0) runs
    k_synth<256, 8, 27, 1, false, 1, true, 1>: block 256, 8 scatterers per
    chunk, 27 bins per tile (the longest that keeps three blocks per CU), 1
    transmit, elevation table, paired lanes."""
    sys.path.insert(0, ROOT)
    import bench
    assert "ILi256ELi8ELi27ELi1ELb0ELi1ELb1ELi1E" in bench.SYNTH_KERNEL
    src = open(os.path.join(ROOT, "paper_2102_02738_amd", "csrc", "kernels.hip")).read()
    assert "#define SIMUS_SC1 8" in src
