"""The benchmark's command-line contract, on the CPU: one GPU only, and the committed
rocprofv3 summaries that its roofline figures read."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_committed_counter_summaries_parse():
    """Each summary carries one traffic line naming the source hash it was taken on and a
    positive byte count; the benchmark reports it only while that hash matches the source
    (a kernel edited since reads null until the counters are taken again)."""
    sys.path.insert(0, ROOT)
    import bench
    profiles = [f for f in os.listdir(os.path.join(ROOT, "profiles")) if f.endswith(".md")]
    checked = 0
    for profile in profiles:
        lines = [l for l in open(os.path.join(ROOT, "profiles", profile)) if l.startswith("traffic-json:")]
        for line in lines:
            rec = json.loads(line.split(":", 1)[1])
            assert len(rec["kernel_source_sha256_16"]) == 16 and rec["traffic_bytes_per_launch"] > 0
            source = rec.get("kernel_source", "dg_kernels.hip")
            prec = rec.get("precision", "fp32_pc")
            t = bench.measured_traffic(profile, source, prec)
            assert t is None or t > 0
            checked += 1
    assert checked >= 1
    assert bench._host()["host_cpus"] >= 1


def test_headline_counters_match_the_current_kernel_source():
    """The headline arm's smoothing step has committed counters for the kernel source as it is:
    the bench's roofline then reports their traffic and the vector units' issue fraction."""
    sys.path.insert(0, ROOT)
    import bench
    t = bench.measured_traffic("cheb_step_heldout32.md", "dg_kernels.hip", "bf16f_pc")
    v = bench.measured_traffic("cheb_step_heldout32.md", "dg_kernels.hip", "bf16f_pc", "valu_busy")
    assert t is not None and t > 0
    assert v is not None and 0 < v <= 1


def test_octree_counters_match_the_current_kernel_source():
    """The octree operator has committed counters for its kernel source as it is, in both arms:
    the octree line's roofline then reports their traffic."""
    sys.path.insert(0, ROOT)
    import bench
    t32 = bench.measured_traffic("octree_step_exchange8.md", "dg_octree.hip", "fp32_pc")
    t64 = bench.measured_traffic("octree_step_exchange8.md", "dg_octree.hip", "fp64")
    assert t32 is not None and t64 is not None and 0 < t32 < t64
