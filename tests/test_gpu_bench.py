"""bench.py's output contract on the GPU: one JSON line with the metric,
the whole-job value, the roofline object of the dominant kernel (achieved
bytes over the measured launch time, against the 8 TB/s HBM peak) and the
step's own access-pattern ceiling beside it.  The main leg alone (the
512^3 x 1000 shot, once), without the CPU leg and the other legs."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.timeout(300)
def test_bench_line_has_the_contract_fields(wave_mod):
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "1", "--warmup", "0", "--no-cpu-baseline",
           "--no-forms", "--no-batched", "--no-gradient", "--no-launch", "--no-paper-shapes"]
    print("case: bench.py main leg only, 1 shot", flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=280, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    rec = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in rec, key
    assert rec["n_gpus"] == 1 and rec["steps"] == 1 and rec["warmup"] == 0
    assert rec["unit"] == "Gpts/s" and rec["dtype"] == "f32" and rec["higher_is_better"] is True
    assert rec["vs_baseline"] is None and rec["cpu_baseline"] is None  # no CPU leg asked for
    assert rec["config"]["workload"].startswith("large_shot")
    # value is 512^3 x 1000 updates over the shot's wall time
    assert abs(rec["value"] - 512 ** 3 * 1000 / (rec["ms_per_step"] * 1e-3) / 1e9) <= 1e-3 * rec["value"]
    rf = rec["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert 0.0 < rf["frac"] < 1.0
    # the kernel time cannot be longer than the shot's wall time per launch
    assert 16 * 512 ** 3 / (rf["achieved"] * 1e9) <= rec["ms_per_step"] * 1e-3 / 1000 * 1.001
    ss = rf["step_stream_measured"]
    assert ss["alternating_gbs"] > 0 and abs(rf["frac_of_step_stream"] - rf["achieved"] / ss["alternating_gbs"]) < 1e-3
    print(f"  bench line: {rec['value']} Gpts/s, roofline frac {rf['frac']}", flush=True)
