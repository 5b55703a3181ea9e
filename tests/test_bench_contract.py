"""Host-side checks of bench.py's contract (no GPU)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_profile_record_parses():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    for name in ("cgls_cfg2_D6_d12.md", "cgls_batched256.md", "cgls_cfg4_D12_d10.md"):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        assert rec["kernel"].startswith("cgls_rows_kernel<double2")
        assert rec["traffic_bytes_per_launch"] > 0
        assert len(rec["cgls_kernels_sha256"]) == 64

    class P:
        M, entries = 55008, 4 * 18564
    # 48 M + 16 E for the D=6 workload
    assert b.rows_kernel_bytes(P) == 48 * 55008 + 16 * 4 * 18564
