"""The bench line's contract, checked on the stored records and on the
one-GPU guard (CPU only: nothing here touches a GPU)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RECORDS = ["bench_c2_512x512x32x1024.json", "bench_c3_256x256x20x256x1024probes.json"]


@pytest.mark.parametrize("name", RECORDS)
def test_stored_record_has_the_contract_fields(name):
    d = json.load(open(os.path.join(ROOT, "profiles", name)))
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["higher_is_better"] is True and d["data"] == "synthetic"
    assert "workload" in d["config"]
    r = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and r["unit"] == "GB/s"
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] >= 1 and c["value"] > 0 and c["sample"]
    # value is the workload's slice-steps (grid points x slices x frames x
    # probes) per second of a timed step
    cfg = d["config"]
    steps = cfg["grid"][0] * cfg["grid"][1] * cfg["slices"] * cfg["frames"] * cfg["probes"]
    assert abs(d["value"] * d["ms_per_step"] / 1e3 / steps - 1.0) < 1e-9


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU only" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
