"""bench.py on the CPU: the one-GPU contract and the consistency of the
measured-traffic table with the committed rocprofv3 summaries (no GPU)."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_kernel_sources_exist():
    for kernel, (srcs, bound) in bench.KERNELS.items():
        assert bound in ("alu", "hbm"), kernel
        for s in srcs:
            assert os.path.exists(os.path.join(ROOT, "paper_cs_0609090_amd", "csrc", s)), (kernel, s)


@pytest.mark.parametrize("entry", bench.MEASURED_TRAFFIC, ids=lambda e: f"{e['kernel']}-{e['workload'][0]}-"
                                                                         f"{e['workload'][1]}")
def test_measured_traffic_matches_its_profile(entry):
    """Each entry names a committed summary whose combined source hash is the
    entry's hash and whose scaled FETCH + WRITE total is the entry's bytes;
    the hash is that of the current sources (a stale entry would report a
    figure for code it was not measured on)."""
    assert entry["kernel"] in bench.KERNELS
    msg, sched, frames, iters = entry["workload"]
    assert msg in ("int8", "1bit", "fp32") and sched in ("single_scan", "two_scan")
    path = os.path.join(ROOT, entry["profile"])
    text = open(path).read()
    m = re.search(r"Combined .*?: ([0-9a-f]{16})\.", text)
    assert m and m.group(1) == entry["hash"], path
    t = re.search(r"HBM traffic per call \(scaled\): .*? = ([0-9.]+) MB = ", text)
    assert t and abs(float(t.group(1)) * 1e6 - entry["bytes"]) < 0.051e6, path
    assert bench.source_hash(bench.KERNELS[entry["kernel"]][0]) == entry["hash"], "profile is stale"
    # the profiled command runs this workload (int8 and single-scan are bench.py's defaults)
    cmd = next(line for line in text.splitlines() if line.startswith("rocprofv3 --kernel-trace"))
    assert (f"--msg {msg}" in cmd) if msg != "int8" else ("--msg" not in cmd or "--msg int8" in cmd)
    assert ("--sched two_scan" in cmd) == (sched == "two_scan")


def test_cpu_baseline_fields():
    """The CPU baseline reports the threads it used, the host's CPU count,
    the single-thread rate and the oracle's single-scan / two-scan ratio
    on the same frames."""
    from paper_cs_0609090_amd import workloads as W
    code = W.code_c0_peg1008()
    q = W.quantize_llr(W.awgn_llr(code.N, 8, 1.0, code.design_rate, key=(0xC2, 0xBE)))
    cb = bench.cpu_baseline(code, q, 8, 8)
    threads, host = bench.host_threads()
    assert cb["kind"] == "oracle" and cb["cores"] == threads and cb["host_cpus"] == host
    assert 1 <= threads <= 16
    assert cb["value"] > 0 and cb["single_thread"]["coded_gbps"] > 0
    assert cb["two_scan_single_thread"]["coded_gbps"] > 0
    w1, w2 = cb["single_thread"]["wall_s"], cb["two_scan_single_thread"]["wall_s"]
    r = w2 / w1  # from the rounded walls: allow for the rounding
    assert abs(cb["single_scan_over_two_scan"] - r) <= 0.002 + r * 1e-3 * (1 / w1 + 1 / w2)
