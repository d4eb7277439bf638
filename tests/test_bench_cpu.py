"""Host-side logic of bench.py (no GPU): the algorithmic byte model of the
K = 2 evaluation kernel, the source-hash gate on the counter traffic, and the
--gpus guard."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1909_11469_amd", "csrc", "bp_kernels.hip")
COUNTERS = os.path.join(ROOT, "profiles", "k_eval_logodds_rnbp_ising1000_counters.txt")


def test_eval_kernel_bytes_1000x1000():
    # 1000 x 1000 grid: N = 10^6, E = 2 * 1,998,000 directed messages
    # (the grid's reverse slots are read as 16-bit offsets: 18 B per message)
    N, E = 1000 * 1000, 2 * 2 * 1000 * 999
    assert bench.eval_kernel_bytes(N, E) == 18 * 3996000 + 8 * 1000000 == 79928000
    assert bench.eval_kernel_bytes(N, E, two_outputs=False) == 14 * 3996000 + 8 * 1000000
    # with 4-byte reverse indices (graphs whose offsets do not fit 16 bits)
    assert bench.eval_kernel_bytes(N, E, rev_bytes=4) == 20 * 3996000 + 8 * 1000000


def test_iteration_bytes_matches_workload_definition():
    # 28.0 B per directed message at 1000 x 1000 (111.9 MB), 298.5 MB for the
    # 500 x 500 K = 32 Potts grid, 32.8 MB for the 200k-node ER graph
    N, E = 1000 * 1000, 3996000
    assert bench.iteration_bytes(N, E) == 111896004
    assert abs(bench.iteration_bytes(N, E) / E - 28.0) < 0.01
    assert bench.iteration_bytes(250000, 998000, 32, 32) == 298468004
    assert bench.iteration_bytes(200000, 1200000) == 32800004


def test_host_cpu_reports_cores():
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and h["logical_cpus"] >= h["nproc"]


def test_committed_counter_summary():
    # the summary's algorithmic bytes follow the byte model; its traffic is
    # reported exactly when it was taken on the kernel source as it stands
    kv = dict(l.strip().split("=", 1) for l in open(COUNTERS) if "=" in l and not l.startswith("#"))
    assert int(kv["algorithmic_bytes_per_launch"]) == bench.eval_kernel_bytes(10 ** 6, 3996000)
    same = kv["kernel_source_sha256"] == hashlib.sha256(open(SRC, "rb").read()).hexdigest()
    want = float(kv["traffic_bytes_per_launch"]) if same else None
    assert bench.counter_traffic(COUNTERS, SRC) == want


def test_counter_traffic_null_when_source_changed(tmp_path):
    src = tmp_path / "k.hip"
    src.write_bytes(b"// another kernel\n")
    assert bench.counter_traffic(COUNTERS, str(src)) is None
    assert bench.counter_traffic(str(tmp_path / "missing.txt"), SRC) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
