"""Host-side parts of bench.py that need no GPU: the one-GPU contract and the
committed counter summary that the bench reads for `roofline.traffic`."""
import json
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_bench_refuses_several_gpus():
    """The path is one GPU by design: --gpus 2 exits with status 2 and says so
    before touching a device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stdout + r.stderr


def test_counter_summary_covers_the_default_products():
    """The machine-readable block of the committed counter summary parses, carries
    the copy-kernel scale factors, and has an entry (with both counters and the
    algorithmic bytes) for the projection and expansion kernels of the default
    launch choices, the ones the bench's roofline names."""
    text = open(bench.COUNTERS_FILE).read()
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    assert m, "no machine-readable block"
    data = json.loads(m.group(1))
    assert data["fetch_scale_bytes_per_kib"] > 0 and data["write_scale_bytes_per_kib"] > 0
    assert set(data["source_sha256"]) >= {"gemm.hip"}
    for name in (bench.PROJ_KERNELS[14], bench.EXPAND_KERNELS[15]):
        k = data["kernels"][name]
        assert k["fetch_kib"] > 0 and k["write_kib"] > 0
        hbm = k["fetch_kib"] * data["fetch_scale_bytes_per_kib"] + \
            k["write_kib"] * data["write_scale_bytes_per_kib"]
        assert abs(hbm - k["hbm_bytes_per_dispatch"]) <= 1e-6 * hbm + 1
        assert k["algorithmic_bytes"] > 0
