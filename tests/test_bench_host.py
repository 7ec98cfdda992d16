"""Host logic of bench.py that needs no GPU: the one-GPU refusal, the
roofline's algorithmic FLOP/byte accounting, the traffic summary lookup and
the reuse of staged inputs."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2108_12430_amd import synth  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_fused_kernel_accounting():
    """Per launch: 2 x MACs of the nine layers for each of the 179 windows
    (per window, worked out layer by layer: 131,203,072 MACs at W = 32768),
    and bytes = each window's 21 x 32768 BF16 input read once, 4-byte strain
    in and clean out for every new sample, and the snapshot update the launch
    performs: each new channel sample read in FP32 and written to the FP32
    ring and its BF16 shadow."""
    dc_s, bb_s = bench.make_mix()
    macs = (8 * 16384 * 21 * 7 + 16 * 8192 * 8 * 7 + 32 * 4096 * 16 * 7 + 64 * 2048 * 32 * 7    # convs
            + 64 * 2048 * 32 * 7 + 32 * 4096 * 16 * 7 + 16 * 8192 * 8 * 7 + 8 * 16384 * 8 * 7  # transposed
            + 1 * 32768 * 8 * 7)                                                                  # output
    assert macs == 131_203_072
    flops, by = bench.algorithmic("dc_fused_bf16", "bf16", synth.deepclean_layers(), dc_s, bb_s)
    assert flops == 2.0 * macs * bench.N_DC
    assert by == bench.N_DC * 21 * 32768 * 2 + 8 * int(dc_s.sum()) + 21 * int(dc_s.sum()) * (4 + 4 + 2)


def test_traffic_lookup_follows_the_kernel_source():
    """Each committed traffic figure is used only while its own kernel
    source's hash matches the one recorded with the counters."""
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic_serving_mix_bf16.json")))
    assert "dc_fused_bf16" in d["kernels"]
    for name, k in d["kernels"].items():
        src = open(os.path.join(ROOT, k["source"]), "rb").read()
        got = bench.traffic_for(name)
        if hashlib.sha256(src).hexdigest() == k["source_sha256"]:
            assert got == k["bytes_per_launch"], name
        else:
            assert got is None, name
    assert bench.traffic_for("no_such_kernel") is None


def test_staged_inputs_are_reused_in_turn():
    c = bench.Cycle([10, 11, 12])
    assert [c[k] for k in range(7)] == [10, 11, 12, 10, 11, 12, 10]


def test_mix_shape():
    dc_s, bb_s = bench.make_mix()
    assert len(dc_s) == 179 and len(bb_s) == 77
    assert set(np.unique(dc_s)) <= {256, 512, 1024}
    assert set(np.unique(bb_s)) <= {128, 256, 512}


def test_cpu_baseline_uses_one_process_per_core():
    """The oracle baseline runs in single-threaded worker processes and
    records how many it used, the host's core count and CPU model."""
    dc_s, bb_s = bench.make_mix()
    r = bench.cpu_baseline(dc_s, bb_s, budget_s=0.3, max_procs=2)
    assert r["kind"] == "oracle" and r["cores"] == min(2, r["host"]["affinity"])
    assert r["value"] > 0 and r["single_core"]["value"] > 0
    assert set(r["host"]) == {"nproc", "affinity", "model"}
