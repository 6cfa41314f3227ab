"""Host-side checks of the benchmark script (no device): the multi-GPU request is
refused with a message, and the algorithmic byte counts it divides by follow the
per-unit figures of the kernels."""
import json
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parent.parent


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                         timeout=120)
    assert out.returncode != 0
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_committed_counter_summaries_are_well_formed():
    """Every profiles/*_pmc.txt names its kernel, workload, source file and hash, and
    its HBM bytes are the calibrated read + write figures (per dispatch of one kernel,
    or per launch of a stage of several kernels, whose dispatches are summed)."""
    files = sorted((ROOT / "profiles").glob("*_pmc.txt"))
    assert files
    for f in files:
        d = json.loads(f.read_text())
        for key in ("workload", "prec", "kernel", "source", "source_sha256_16", "hbm_bytes_per_launch",
                    "calibration", "command_fetch", "command_write"):
            assert key in d, (f.name, key)
        cal = d["calibration"]
        fk = d["fetch_kib_per_launch"] if "fetch_kib_per_launch" in d else d["fetch_kib_per_dispatch"]
        wk = d["write_kib_per_launch"] if "write_kib_per_launch" in d else d["write_kib_per_dispatch"]
        rd = fk * 1024 * cal["fetch_scale"]
        wr = wk * 1024 * cal["write_scale"]
        assert abs(d["hbm_bytes_per_launch"] - (rd + wr)) <= 2
        assert (ROOT / d["source"]).exists()
        assert f.name == f"{d['kernel']}_{d['workload']}_{d['prec']}_pmc.txt"
