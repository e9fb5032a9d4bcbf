"""bench.py command-line contract that needs no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_measured_traffic_is_reported_only_for_the_profiled_kernels():
    """The roofline's `traffic` comes from the committed counter summary only
    when the kernel sources hash to the summary's hash and the run uses the
    summary's number of cluster blocks per CU; otherwise it is null."""
    import json
    b = _bench_module()
    with open(os.path.join(ROOT, "profiles", "inner_operator_traffic_64x64x32.json")) as fh:
        d = json.load(fh)
    h, cb = b.kernel_source_hash(), d["cluster_blocks"]
    units = d["element_members_per_launch"]
    t = b.traffic_from_profile(h, units, cb)
    if d["kernel_source_hash"] == h:  # the committed summary was taken on these sources
        assert abs(t - d["element"]["bytes_per_launch"]) <= 1.0
    else:  # the kernels changed since: no measured figure until the counters are retaken
        assert t is None
    assert b.traffic_from_profile(h, units, cb + 1 if cb < 4 else cb - 1) is None
    assert b.traffic_from_profile("0" * 16, units, cb) is None
