"""Host logic of bench.py that runs without a GPU: the algorithmic-byte count behind the
roofline figure, the source-hash gate on the committed traffic summary, and the refusal of
runs on more than one GPU."""
import hashlib
import os
import subprocess
import sys

import bench


def test_algorithmic_bytes_closed_form():
    # 8 B per expanded vertex (seeds of every sample + reached), 8 B per scanned edge,
    # 16 B per reached vertex (the 64-bit counter's read and write)
    st = {"samples": 10, "reached": 1000, "edges_scanned": 25000, "live_edges": 1100}
    assert bench.algorithmic_bytes(st, 7) == 8 * (10 * 7 + 1000) + 8 * 25000 + 16 * 1000
    assert bench.algorithmic_bytes({"samples": 0, "reached": 0, "edges_scanned": 0}, 3) == 0


def test_traffic_only_for_the_kernel_source_it_was_taken_on(tmp_path):
    src = tmp_path / "kernel.hip"
    src.write_bytes(b"__global__ void k() {}\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "prof.txt"
    prof.write_text("# counters\n"
                    f"kernel_source_sha256: {digest}  (when the counters were taken)\n"
                    "traffic_bytes_per_launch: 12345\n")
    assert bench.traffic_from_profile(str(prof), str(src)) == 12345.0
    src.write_bytes(b"__global__ void k() { /* changed */ }\n")
    assert bench.traffic_from_profile(str(prof), str(src)) is None
    assert bench.traffic_from_profile(str(tmp_path / "missing.txt"), str(src)) is None


def test_committed_profile_names_a_source_hash_and_traffic():
    root = os.path.dirname(os.path.abspath(bench.__file__))
    fields = {}
    with open(os.path.join(root, "profiles", "decrease_kernel_rmat22_pmc.txt")) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.split()[0]
    assert len(fields["kernel_source_sha256"]) == 64
    assert float(fields["traffic_bytes_per_launch"]) > float(fields["algorithmic_bytes_per_launch"])
    # the committed counters belong to the committed kernel source, so the bench line carries
    # them (a kernel change needs new counters before it is committed)
    src = os.path.join(root, "paper_2302_13529_amd", "csrc", "decrease.hip")
    assert fields["kernel_source_sha256"] == hashlib.sha256(open(src, "rb").read()).hexdigest()


def test_more_than_one_gpu_is_refused():
    root = os.path.dirname(os.path.abspath(bench.__file__))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
