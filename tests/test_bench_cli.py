"""bench.py's command line on the CPU: more than one GPU is refused with a
message and status 2 before anything touches a device; the copy-probe and
traffic helpers read the committed counter file."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_file_matches_its_kernel_sources():
    """The committed HBM counters are used only while the kernel sources hash
    to the value they were taken for, and only for the item shape they were
    taken with."""
    import pytest
    sys.path.insert(0, ROOT)
    import bench
    with open(bench.TRAFFIC_FILE) as f:
        taken = [ln.split(":", 1)[1].strip() for ln in f if ln.startswith("source_sha256_16:")]
    if taken != [bench.kernel_source_hash()]:
        pytest.skip("the counters predate the kernel sources: retake them")
    shapes, cur = {}, None
    with open(bench.TRAFFIC_FILE) as f:
        for ln in f:
            if ":" not in ln or ln.startswith("#"):
                continue
            k, v = (x.strip() for x in ln.split(":", 1))
            if k == "workload":
                cur = shapes.setdefault(v, [0, 0, 0])
            elif cur is not None and k in ("chunk_groups_per_item", "loads_in_flight",
                                           "words_per_lane"):
                cur[("chunk_groups_per_item", "loads_in_flight", "words_per_lane").index(k)] = int(v)
    assert set(shapes) == {"batched-10000x500", "large-40000x1000"}
    for name, shape in shapes.items():
        assert bench.measured_traffic(name, *shape) is not None
        other = (shape[0], shape[1], 3 - shape[2])  # the other words-per-lane count
        assert bench.measured_traffic(name, *other) is None
