"""bench.py's output contract, on the GPU: one JSON line (strict JSON, no NaN), the metric
and config of the chosen workload, a value consistent with ms_per_step, the stage
roofline object and the CPU oracle baseline. A short run on the 64^3 p=3 workload: 5
steps, a 2 s oracle sample, no legs, adjoint or small-workload run (the default run
headlines the 96^3 p=4 workload the same way)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _reject(c):
    raise ValueError(f"non-finite number {c} in the bench line")


def test_bench_json_line():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "5", "--warmup", "1",
           "--workload", "C3", "--legs", "", "--acc-steps", "5", "--cpu-seconds", "2",
           "--no-adjoint", "--no-small-run"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0], parse_constant=_reject)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 5 and d["warmup"] == 1 and d["dtype"] == "f64"
    dof = 64 ** 3 * 64
    assert d["config"]["workload"] == "deform3d_64cube_p3" and d["config"]["dof"] == dof
    assert abs(d["value"] - dof * 4 / (d["ms_per_step"] * 1e-3)) <= 1e-6 * d["value"]
    rl = d["roofline"]
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["peak"] == 8000.0
    assert abs(rl["frac"] - rl["achieved"] / rl["peak"]) < 1e-12 and 0 < rl["frac"] < 1
    # achieved = algorithmic bytes of a stage over the stage's kernel time
    assert abs(rl["achieved"] - rl["alg_bytes_per_stage"] / (rl["stage_us"] * 1e3)) \
        <= 1e-9 * rl["achieved"]
    assert rl["alg_bytes_per_stage"] == 16 * 8 * dof
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
    # the FP32 and BF16 forms ran the same region
    assert set(d["forms"]) == {"fp32", "bf16"}
    for f in d["forms"].values():
        assert f["after_steps"]["steps"] == 5 and f["after_steps"]["interface_l1_vs_fp64"] >= 0
    # bench refuses more than one GPU with a message
    r2 = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                        capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r2.returncode != 0 and "one GPU" in r2.stderr
