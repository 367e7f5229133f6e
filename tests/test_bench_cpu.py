"""Host-side checks of bench.py's contract that need no GPU: one GPU only, and the traffic summary
it reads resolves for the sources as they stand."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU only" in (r.stdout + r.stderr)
    assert not r.stdout.strip().startswith("{")          # no JSON line


def test_traffic_summary_matches_sources():
    """The PMC traffic lines bench.py reports are valid only while the kernel sources hash to the values
    recorded next to them; a stale summary must be re-taken, not reported."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.measured_traffic("k_fused_E5") is not None
    for name in ("k_sliced_E5", "k_pack_tile"):
        assert bench.measured_traffic(name, profile="sliced_sweep_100bp_E5_pmc.md") is not None, name


def test_trace_summary_matches_sources():
    """The kernel trace summary of the headline kernel names the source hash it was taken at; it must be
    the hash of the sources as they stand."""
    import hashlib
    text = open(os.path.join(ROOT, "profiles", "sliced_sweep_100bp_E5_kernel_trace.md")).read()
    h = hashlib.sha256()
    for src in ("ss_sliced_kernel.h", "ss_sliced_ops.h", "ss_sliced_lo.hip"):
        h.update(open(os.path.join(ROOT, "paper_1910_09020_amd", "csrc", src), "rb").read())
    assert f"sha256_16={h.hexdigest()[:16]}" in text
