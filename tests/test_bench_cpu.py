"""bench.py host logic (CPU, no GPU): the one-GPU refusal and the recorded HBM traffic."""
import hashlib
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_recorded_traffic_follows_the_kernel_sources():
    """traffic is the profile's figure while the recorded source hash matches, else None."""
    bench = load_bench()
    path = os.path.join(ROOT, "profiles", "k_particles_c2_hbm_traffic.txt")
    fields = dict(line.split(": ", 1) for line in open(path).read().splitlines()
                  if line.startswith(("kernel_source_sha256:", "sources:",
                                      "traffic_bytes_per_launch:")))
    h = hashlib.sha256()
    for src in fields["sources"].split():
        h.update(open(os.path.join(ROOT, src), "rb").read())
    current = h.hexdigest() == fields["kernel_source_sha256"].strip()
    got = bench.measured_traffic()
    if current:
        assert got == float(fields["traffic_bytes_per_launch"])
        # the recorded traffic is at least the algorithmic bytes per particle of c2
        assert got >= bench.PARTICLE_BYTES_FP32 * 16777216
    else:
        assert got is None
