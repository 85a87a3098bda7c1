"""bench.py's output contract on a GPU: one JSON line with the fields the
benchmark report needs, in a reduced run (one seed, one timed step, the
extra rows off), so that a change to bench.py that breaks the line shows up
in the GPU tests rather than only in a full benchmark run."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ARGS = ["--steps", "1", "--warmup", "0", "--seeds", "0", "--no-global", "--no-paper-config", "--no-batch",
        "--no-mixed", "--no-diffusion", "--no-1d", "--no-replica", "--no-c2", "--no-tuned", "--no-exact"]


@pytest.mark.gpu
def test_bench_prints_one_json_line_with_roofline_and_cpu_baseline():
    print("bench.py", " ".join(ARGS), flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py")] + ARGS, cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])

    assert isinstance(d["metric"], str) and d["metric"]
    assert d["value"] > 0 and d["unit"] == "ms" and d["higher_is_better"] is False
    assert d["n_gpus"] == 1 and d["steps"] == 1 and d["warmup"] == 0
    assert d["ms_per_step"] > 0 and d["scaling"] in ("weak", "strong")
    assert d["vs_baseline"] is None
    assert d["dtype"] == "f64" and d["data"] == "synthetic"
    assert isinstance(d["config"]["workload"], str) and d["config"]["workload"]
    assert "model" not in d["config"]

    rl = d["roofline"]
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["peak"] == 8000.0
    assert rl["achieved"] > 0 and abs(rl["frac"] - rl["achieved"] / rl["peak"]) < 1e-3
    assert rl["traffic"] is None or rl["traffic"] > 0

    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["unit"] == "ms"
    assert isinstance(cb["cores"], int) and cb["cores"] >= 1
    assert isinstance(cb["sample"], str) and cb["sample"]
    assert cb["cycles_equal_gpu"] is True
