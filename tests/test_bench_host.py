"""Host-side parts of bench.py: the one-GPU contract and the committed
rocprofv3 summaries it reads."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profile_summaries_carry_their_fields():
    """Each summary bench.py reads states the kernel, its average launch
    and the hash of the sources it was taken on (bench reports a summary's
    figures only while that hash matches)."""
    sys.path.insert(0, ROOT)
    import bench
    for name, need in (("resident_kernel_toric2d_L32_minsum.md",
                        ("kernel", "launch_shape", "avg_launch_ns", "avg_timed_launch_ns",
                         "executed_valu_per_check_sweep", "traffic_bytes_per_launch", "fetch_scale",
                         "write_scale", "source_sha256")),
                       ("resident_kernel_toric2d_L32_sumproduct.md",
                        ("kernel", "launch_shape", "avg_launch_ns", "avg_timed_launch_ns",
                         "executed_valu_per_check_sweep", "source_sha256")),
                       ("stream_sweep_toric2d_L32_minsum.md",
                        ("kernel", "avg_launch_ns", "traffic_bytes_per_launch", "source_sha256"))):
        path = os.path.join(ROOT, "profiles", name)
        fields = {}
        for line in open(path):
            if ": " in line:
                k, v = line.strip().split(": ", 1)
                fields[k] = v
        for k in need:
            assert k in fields, (name, k)
        assert float(fields["avg_launch_ns"]) > 0 and len(fields["source_sha256"]) == 64
    # the profile of the dominant kernel names the command that made it
    text = open(os.path.join(ROOT, "profiles", "resident_kernel_toric2d_L32_minsum.md")).read()
    assert "rocprofv3 --kernel-trace --stats" in text and "rocprofv3 --pmc FETCH_SIZE" in text
    # a summary taken on other sources reads as absent, never as stale figures
    assert bench.profile_fields("resident_kernel_toric2d_L32_minsum.md", ("bench.py",)) is None


def test_method_operation_counts():
    """The roofline's operation counts per check-sweep: 19 for normalised
    min-sum on the 2D toric code (its qubit-side clamps cannot bind), 23 with
    the clamps, and 390 for sum-product (3 (d_c - 2) box-plus steps)."""
    sys.path.insert(0, ROOT)
    import bench

    class P:
        q, alpha, clamp = 0.05, 0.75, 1000.0
    assert bench.ops_per_check_sweep("minsum", 4, 2, P) == 19
    P.clamp = 4.0
    assert bench.ops_per_check_sweep("minsum", 4, 2, P) == 23
    assert bench.ops_per_check_sweep("sumproduct", 4, 2, P) == 390
