#!/usr/bin/env python3
"""Streaming-inference benchmark on one MI355X.

Workload: the multi-stream serving mix run closed-loop (every stream always
has its next request pending): 179 DeepClean streams (21 witness channels,
8-s windows of 32768 samples at 4096 Hz) and 77 BBHnet streams (2 detectors,
1-s windows of 2048 samples at 2048 Hz); each stream's request carries 1/16,
1/8 or 1/4 s of new samples (seeded per stream).  One step = one request of
every stream: ingest of the requests' new samples into the snapshot rings
(one batched snapshot_update per model group), the DeepClean forward of all
179 windows with the causal slice and noise subtraction, and the BBHnet
forward of all 77 windows (on a second HIP stream, overlapping the DeepClean
forward).  At most two steps are in flight.

Reported: streamed samples/s (sum of new samples over completed requests per
second, the BF16 batched path, every step's inputs already resident in HBM
when the timed loop starts) with per-update latency p50/p99 from arrival to
observed completion in the same timed loop (a saturated source: a stream's
next request arrives when its previous one is issued); the same step with
its requests in pinned host memory, the host-to-device copy of the new
samples and the copy of the results back inside the timed loop
(PCIe-inclusive, with its own latency); the same workload on the FP32 plain
path (one stream at a time, FP32 direct convolution); the dominant kernel's
roofline figures from HIP events; and the FP64 CPU oracle (one
single-threaded process per host core) on a bounded sample of the same
requests.  Further legs, each outside
`value` and skippable:
the receptive-field band only (GW_CAUSAL), the output aggregation variants
(0.75-s aggregation latency, depth-4 overlap averaging) and FP16 DeepClean,
64 end-to-end ensemble streams, dense BBHnet batches, a 1-s FP32 DeepClean
window, the retraining step, and PCIe-inclusive serving through serve.py.
"""
from __future__ import annotations

import argparse
import collections
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_CUS = 256  # MI355X compute units
ROOF_STEPS = 40  # steps whose launches the roofline pass times


class Cycle(list):
    """A list indexed modulo its length (staged inputs reused in turn)."""

    def __getitem__(self, k):
        return list.__getitem__(self, k % len(self))
METRIC = "streamed samples/sec + p99 per-update latency, BF16 batched vs FP32 plain"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_PEAK_TFLOPS = 157.3

N_DC, N_BB = 179, 77
DC_C, DC_W, DC_FS = 21, 32768, 4096
BB_C, BB_W, BB_FS = 2, 2048, 2048


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_mix(seed=6):
    rng = np.random.default_rng(seed)
    frac = np.array([1 / 16, 1 / 8, 1 / 4])
    dc_s = (rng.choice(frac, N_DC) * DC_FS).astype(np.int64)
    bb_s = (rng.choice(frac, N_BB) * BB_FS).astype(np.int64)
    return dc_s, bb_s


def layer_shapes(layers, W):
    out, L = [], W
    for (typ, ci, co, k, s, p, op, bn) in layers:
        Lo = (L + 2 * p - k) // s + 1 if typ == "conv" else (L - 1) * s - 2 * p + k + op
        out.append((typ, ci, co, k, L, Lo))
        L = Lo
    return out


def algorithmic(name, precision, layers, dc_s, bb_s):
    """(flops, bytes) per launch of a named kernel in one step."""
    esz = 2 if precision == "bf16" else 4
    kind, _, tag = name.partition(".")
    if kind.startswith("dc_conv"):
        l = int(tag[1:])
        typ, ci, co, k, Li, Lo = layer_shapes(layers, DC_W)[l]
        n = N_DC
        macs = n * co * Lo * ci * k if typ == "conv" else n * ci * Li * co * k
        by = n * ci * Li * esz + co * ci * k * esz
        if l == len(layers) - 1:
            by += 2 * 4 * int(dc_s.sum())          # strain in, clean out
        else:
            by += n * co * Lo * esz
        return 2.0 * macs, float(by)
    if kind == "dc_fused_bf16":
        # whole network per window: input read once from the BF16 ring
        # shadow, strain read and clean written once; activations stay on chip
        n = N_DC
        macs = 0
        for (typ, ci, co, k, Li, Lo) in layer_shapes(layers, DC_W):
            macs += co * Lo * ci * k if typ == "conv" else ci * Li * co * k
        by = n * DC_C * DC_W * 2 + 2 * 4 * int(dc_s.sum())
        # the step's launch also performs the snapshot update: the new
        # samples read in FP32, written to the ring (FP32) and its BF16 shadow
        by += DC_C * int(dc_s.sum()) * (4 + 4 + 2)
        return 2.0 * macs * n, float(by)
    if kind.startswith("bbh_conv"):
        st = int(tag[1:])
        n, L = N_BB, BB_W
        chans = [(2, 32), (32, 64), (64, 128)]
        for i in range(st):
            L //= 2
        ci, co = chans[st]
        Lo = L // 2
        if "conva" in kind:
            macs = n * co * Lo * ci * 7
            by = n * ci * L * esz + n * co * Lo * esz + co * ci * 7 * esz
        else:
            macs = n * co * Lo * co * 7 + n * co * Lo * ci
            by = n * co * Lo * esz * 2 + n * ci * L * esz + co * co * 7 * esz
        return 2.0 * macs, float(by)
    if kind == "snapshot":
        cs = DC_C * int(dc_s.sum()) + BB_C * int(bb_s.sum())
        return 0.0, float(cs * (4 + 4 + 2))
    if kind == "gather":
        return 0.0, float(N_BB * BB_C * BB_W * 8)
    return 0.0, 0.0


def _oracle_requests(dc_s, bb_s, first, budget_s, interleave=True):
    """Run oracle requests of the serving mix (DeepClean and BBHnet streams
    interleaved 179:77, starting at request `first`) for about budget_s
    seconds on the calling thread; returns (samples, DeepClean requests,
    BBHnet requests, seconds).  Each request recomputes its stream's full
    window (plain definition), then the causal slice and subtraction for
    DeepClean streams."""
    from oracle import ref
    from paper_2108_12430_amd import synth
    dcp = synth.deepclean_params(0)
    bbp = synth.bbhnet_params(0)
    wit, strain = synth.witness_stream(11, DC_W + 1024)
    bbx = synth.gaussian(12, (BB_C, BB_W + 512))
    samples = n_dc = n_bb = 0
    t0 = time.perf_counter()
    i = first
    while time.perf_counter() - t0 < budget_s or n_dc == 0 or n_bb == 0:
        is_dc = ((i + 1) * N_DC // (N_DC + N_BB) > i * N_DC // (N_DC + N_BB)) if interleave else (i % 2 == 0)
        if is_dc:
            s = int(dc_s[i % N_DC])
            x = ref.snapshot_after(wit, DC_W + s, DC_W)[None]
            ref.causal_clean(ref.deepclean_forward(dcp, x), strain[None, DC_W: DC_W + s])
            n_dc += 1
        else:
            s = int(bb_s[i % N_BB])
            ref.bbhnet_forward(bbp, ref.snapshot_after(bbx, BB_W + s, BB_W)[None])
            n_bb += 1
        samples += s
        i += 1
    return samples, n_dc, n_bb, time.perf_counter() - t0


def _oracle_worker(args):
    """One single-threaded oracle process (BLAS limited to one thread)."""
    from threadpoolctl import threadpool_limits
    dc_s, bb_s, first, budget_s = args
    with threadpool_limits(limits=1):
        return _oracle_requests(dc_s, bb_s, first, budget_s)


def host_cpu():
    """Host core count and CPU model (recorded with the CPU baseline)."""
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": aff, "model": model}


def cpu_baseline(dc_s, bb_s, budget_s=12.0, max_procs=16):
    """The FP64 oracle on the host's cores: one single-threaded process per
    core (at most max_procs, the CPU share of one GPU on the benchmark
    machines), each running its own slice of the serving mix's requests for
    about budget_s seconds; plus the same requests on one core.  Call it
    before the process touches the GPU (the workers are started with
    'spawn')."""
    import multiprocessing as mp
    cpu = host_cpu()
    nproc = max(1, min(max_procs, cpu["affinity"]))
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ.setdefault(v, "1")
    ctx = mp.get_context("spawn")
    with ctx.Pool(nproc) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_worker, [(dc_s, bb_s, 97 * w, budget_s) for w in range(nproc)])
        wall = time.perf_counter() - t0
    samples = sum(r[0] for r in res)
    n_dc = sum(r[1] for r in res)
    n_bb = sum(r[2] for r in res)
    # one core: the same request mix in this process, BLAS on one thread
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        s1, d1n, b1n, d1 = _oracle_requests(dc_s, bb_s, 0, budget_s / 2)
    return {"value": samples / wall, "unit": "samples/s", "cores": nproc, "kind": "oracle",
            "sample": f"{n_dc} DeepClean + {n_bb} BBHnet requests of the same mix (FP64 numpy oracle, full-window "
                      f"recompute per request) in {nproc} single-threaded processes, {wall:.1f} s wall",
            "host": cpu,
            "single_core": {"value": s1 / d1, "unit": "samples/s",
                            "sample": f"{d1n} DeepClean + {b1n} BBHnet requests, {d1:.1f} s, one process, 1 thread"}}


def traffic_for(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the summary is missing or the kernel source has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_serving_mix_bf16.json")
    try:
        k = json.load(open(path))["kernels"][kernel]
        src = open(os.path.join(ROOT, k["source"]), "rb").read()
    except (OSError, ValueError, KeyError, TypeError):
        return None
    if hashlib.sha256(src).hexdigest() != k.get("source_sha256"):
        return None
    return float(k["bytes_per_launch"])


def train_bench(dev, steps=5, warmup=2, B=32, W=DC_W, recompute=True, precision="fp32"):
    """One DeepClean training step = batch-statistics forward, band-passed
    MSE (55-65 Hz), hand-written backward (FP32 activations, statistics and
    gradients; precision "bf16" runs the convolutions on BF16 matrix cores);
    the optimizer update is outside the library and not timed."""
    import torch

    from paper_2108_12430_amd import gwstream as gs
    from paper_2108_12430_amd import synth
    params = torch.from_numpy(synth.deepclean_params(0)).to(dev)
    m = gs.DeepClean(params, synth.deepclean_layers())
    wit, strain = synth.witness_stream(4, 4 * W)
    x = torch.from_numpy(np.ascontiguousarray(np.tile(wit.reshape(DC_C, 4, W).transpose(1, 0, 2), (B // 4, 1, 1))))
    x = x.to(dev)
    st = torch.from_numpy(np.ascontiguousarray(np.tile(strain.reshape(4, W), (B // 4, 1)))).to(dev)
    flags = gs.TRAIN | (gs.RECOMPUTE if recompute else 0)
    prec = gs.BF16 if precision == "bf16" else gs.FP32
    noise = torch.empty((B, W), device=dev)
    ws = torch.empty(m.workspace_bytes(B, W, prec, flags), dtype=torch.uint8, device=dev)
    scratch = torch.empty(m.backward_scratch_bytes(B, W, flags), dtype=torch.uint8, device=dev)
    dp = torch.empty_like(params)

    def one():
        m.forward(x=x, noise=noise, flags=flags, ws=ws, precision=prec)
        loss, dn = gs.bandpass_mse(st, noise, float(DC_FS), 55.0, 65.0)
        m.backward(x, dn, ws, dp, flags=flags, scratch=scratch, precision=prec)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return {"batch": B, "window": W, "ms_per_step": 1e3 * dt, "samples_per_s": B * W / dt,
            "conv_dtype": precision, "recompute": recompute, "workspace_MB": (ws.numel() + scratch.numel()) / 1e6}


def bbhnet_flops(L=BB_W):
    """Algorithmic FLOPs of one BBHnet window (three residual stages)."""
    macs = 0
    for ci, co in ((BB_C, 32), (32, 64), (64, 128)):
        L //= 2
        macs += co * L * ci * 7 + co * L * co * 7 + co * L * ci   # conv_a, conv_b, 1x1 shortcut
    return 2.0 * (macs + 128)


def bbhnet_batch_bench(dev, batches=(64, 256, 1024), iters=100, warm_s=0.2):
    """BBHnet BF16 forward on dense batches of 2 x 2048 windows: at least
    warm_s seconds of the same launches first (steady clocks), then iters
    launches timed with HIP events on the launch stream."""
    import torch

    from paper_2108_12430_amd import gwstream as gs
    from paper_2108_12430_amd import synth
    bb = gs.BBHnet(torch.from_numpy(synth.bbhnet_params(0)).to(dev), synth.bbhnet_stages())
    out = []
    for B in batches:
        x = torch.from_numpy(synth.bbh_windows(3 + B, B)[0]).to(dev)
        logits = torch.empty(B, device=dev)
        ws = torch.empty(bb.workspace_bytes(B, BB_W, gs.BF16), dtype=torch.uint8, device=dev)
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < warm_s:
            for _ in range(10):
                bb.forward(x=x, logits=logits, precision=gs.BF16, ws=ws)
            torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(iters):
            bb.forward(x=x, logits=logits, precision=gs.BF16, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        dt = e0.elapsed_time(e1) * 1e-3 / iters
        tf = B * bbhnet_flops() / dt / 1e12
        out.append({"batch": B, "ms": 1e3 * dt, "windows_per_s": B / dt, "samples_per_s": B * BB_W / dt,
                    "tflops": tf, "frac_of_bf16_peak": tf / BF16_PEAK_TFLOPS})
    return out


def d0_latency(dev, reps=50):
    """One 1-s window (21 x 4096) through DeepClean, FP32, batch 1:
    synchronous call latency."""
    import torch

    from paper_2108_12430_amd import gwstream as gs
    from paper_2108_12430_amd import synth
    m = gs.DeepClean(torch.from_numpy(synth.deepclean_params(0)).to(dev), synth.deepclean_layers())
    x = torch.from_numpy(synth.witness_stream(1, 4096)[0][None]).to(dev)
    noise = torch.empty((1, 4096), device=dev)
    ws = torch.empty(m.workspace_bytes(1, 4096, gs.FP32), dtype=torch.uint8, device=dev)
    lat = []
    for i in range(reps + 5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.forward(x=x, noise=noise, precision=gs.FP32, ws=ws)
        torch.cuda.synchronize()
        if i >= 5:
            lat.append(1e3 * (time.perf_counter() - t0))
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "config": "DeepClean FP32, 21 x 4096 (1 s at 4096 Hz), batch 1"}


def serve_bench(dc, bb, prec, dc_s, bb_s, rates, seconds, log_fn, phases=(1, 2, 4, 8)):
    """Serving loop (continuous batching; clients receive their new samples
    straight into pinned staging memory handed out by the server, so the
    copy to the device is PCIe-inclusive) on the same 256-stream mix.

    Closed loop: every stream keeps one update outstanding and sends the next
    as soon as its previous result is back.  The loop is event driven: it
    receives the next updates of the streams whose results came back, in
    batches of up to N/P (N streams, P the batch divisor), launches a step per
    batch and polls for completed steps after each, so results are taken as
    they finish and one batch's host work overlaps the others' device work.
    A batch's receives (the copies of the clients' new samples into the
    handed-out buffers) are one native batched copy spread over host threads
    (gw_host_copy_batch, outside the interpreter lock).  Larger P: smaller,
    more frequent steps, lower latency.  Open loop: Poisson arrivals at the
    given aggregate update rates.  Latency runs from a request's arrival (its
    samples complete in memory) to its result on the host."""
    import torch

    from paper_2108_12430_amd.serve import HipExecutor, Server
    from paper_2108_12430_amd import synth

    rng = np.random.default_rng(6)
    src = synth.gaussian(8, (DC_C, 1 << 18))
    src_s = synth.gaussian(9, (1 << 18,))
    specs = [("dc", DC_C, DC_W, int(s)) for s in dc_s] + [("bbh", BB_C, BB_W, int(s)) for s in bb_s]
    ring = lambda c, w: ((c * w * 4 + 255) // 256 + (c * w * 2 + 255) // 256) * 256
    arena = N_DC * ring(DC_C, DC_W) + N_BB * ring(BB_C, BB_W) + (64 << 20)
    out = {}

    # each stream's source blocks (what its receive delivers), 8 per stream
    # used in turn
    NPRE = 8
    pre = []
    for i, (model, C, W, s) in enumerate(specs):
        blocks = []
        for k in range(NPRE):
            o = (i * 7919 + k * s) % ((1 << 18) - 1024)
            blocks.append((np.ascontiguousarray(src[:C, o:o + s]),
                           np.ascontiguousarray(src_s[o:o + s]) if model == "dc" else None))
        pre.append(blocks)

    # the blocks' host addresses, for batched receives
    pre_addr = [[(x.__array_interface__["data"][0], None if st is None else st.__array_interface__["data"][0])
                 for x, st in blocks] for blocks in pre]

    def fill(r, i, k):
        x, st = pre[i][k % NPRE]
        np.copyto(r.samples, x)
        if st is not None:
            np.copyto(r.strain, st)

    def receive(srv, sid, i, k, t_arrival=None):
        """Client i's k-th update, received into a handed-out buffer."""
        r = srv.reserve(sid, specs[i][3])
        fill(r, i, k)
        return srv.commit(r, t_arrival)

    def receive_batch(srv, batch):
        for sid, i, k in batch:
            receive(srv, sid, i, k)

    def run(arrivals, nphase=2):
        ex = HipExecutor({"dc": dc, "bbh": bb}, arena_bytes=arena, max_slots=len(specs),
                         max_items=len(specs), precision=prec)
        srv = Server(ex, max_inflight=nphase + 1)
        sids = [srv.open_stream(m, C, W) for (m, C, W, s) in specs]
        index = {sid: i for i, sid in enumerate(sids)}
        # warm-up: a few requests per stream (staging pages, workspaces)
        for k in range(3):
            for i, sid in enumerate(sids):
                receive(srv, sid, i, k)
            srv.drain()
        srv.completed.clear()
        torch.cuda.synchronize()
        # requests form no reference cycles; the cyclic collector's full passes
        # (tens of ms over the live objects) are kept out of the timed loop
        gc.collect()
        gc.freeze()
        gc.disable()
        t0 = time.perf_counter()
        nsamp = 0
        if arrivals is None:
            cnt = [3] * len(specs)
            todo = collections.deque(range(len(specs)))  # streams whose next update is due
            per_step = (len(specs) + nphase - 1) // nphase
            seen = 0
            stop = False

            def retire():
                nonlocal seen, nsamp
                srv.poll()
                done = srv.completed
                for r in done[seen:]:
                    i = index[r.stream]
                    nsamp += specs[i][3]
                    todo.append(i)
                seen = len(done)

            while True:
                n = 0
                while todo and n < per_step and not stop:
                    # receive a batch: reserve, one native batched copy over
                    # the host threads, then commit (arrival = data complete)
                    idx = [todo.popleft() for _ in range(min(per_step - n, len(todo)))]
                    rs = [srv.reserve(sids[i], specs[i][3]) for i in idx]
                    srv.receive(rs, [pre_addr[i][cnt[i] % NPRE] for i in idx])
                    for r, i in zip(rs, idx):
                        srv.commit(r)
                        cnt[i] += 1
                    n += len(idx)
                    retire()
                if srv.pending():
                    srv.step()
                retire()
                stop = stop or time.perf_counter() - t0 >= seconds
                if not todo or stop:
                    if not srv.inflight and not srv.pending():
                        break
                    srv.wait()
                    retire()
        else:
            idx = 0
            cnt = [3] * len(specs)
            while idx < len(arrivals) or srv.pending() or srv.inflight:
                now = time.perf_counter() - t0
                while idx < len(arrivals) and arrivals[idx][0] <= now:
                    ta, i = arrivals[idx]
                    receive(srv, sids[i], i, cnt[i], t_arrival=t0 + ta)
                    cnt[i] += 1
                    nsamp += specs[i][3]
                    idx += 1
                if srv.pending():
                    srv.step()
                else:
                    srv.poll()
        dt = time.perf_counter() - t0
        gc.enable()
        gc.unfreeze()
        st_ = srv.latency_stats()
        st_["samples_per_s"] = nsamp / dt
        st_["steps"] = srv.steps
        return st_

    out["closed_loop"] = []
    for P in phases:
        res = run(None, P)
        res["phases"] = P
        out["closed_loop"].append(res)
        log_fn(f"bench: serving closed loop, {P} phase groups: {res}")
    strides = np.array([s for *_, s in specs], np.float64)
    w = 1.0 / strides
    out["open_loop"] = []
    for lam in rates:
        per = lam * w / w.sum()   # per-stream Poisson rates proportional to 1/stride
        span = max(seconds, 1e4 / lam)  # at least 10^4 updates per rate
        arr = []
        for i, r in enumerate(per):
            t = rng.exponential(1.0 / r)
            while t < span:
                arr.append((t, i))
                t += rng.exponential(1.0 / r)
        arr.sort()
        res = run(arr)
        res["rate"] = lam
        out["open_loop"].append(res)
        log_fn(f"bench: serving open loop {lam}/s: {res}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", choices=["bf16", "fp32"], default="bf16")
    ap.add_argument("--lat-steps", type=int, default=300)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-rates", default="1000,2000,5000,10000,20000")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--no-train", action="store_true")
    ap.add_argument("--no-band", action="store_true")
    ap.add_argument("--no-agg", action="store_true", help="skip the output aggregation variants")
    ap.add_argument("--no-ens", action="store_true", help="skip the end-to-end ensemble leg")
    ap.add_argument("--serial-groups", action="store_true",
                    help="run the two model groups one after the other on one stream (the schedule the roofline "
                         "pass times; for profiling the kernels on their own)")
    ap.add_argument("--no-extra", action="store_true", help="skip the BBHnet batch and 1-s window legs")
    ap.add_argument("--dc-cus", type=int, default=0,
                    help="CU budget of the fused DeepClean kernel (0: all CUs); CUs left over run the BBHnet "
                         "group's kernels beside it")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--train-only", action="store_true",
                    help="time only the training step (FP32 and BF16-conv; --steps/--warmup apply), for profiling")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving-loop leg (closed and open loop), for profiling")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    cpu = None
    if not args.no_cpu and not args.train_only and not args.serve_only:
        # before anything touches the GPU: the oracle workers are new processes
        dc_s0, bb_s0 = make_mix()
        cpu = cpu_baseline(dc_s0, bb_s0)
        log(f"bench: cpu oracle {cpu['value']:.4g} samples/s in {cpu['cores']} single-threaded processes "
            f"(one core: {cpu['single_core']['value']:.4g}); host {cpu['host']}")

    import torch

    if args.train_only:
        dev = torch.device("cuda:0")
        out = {}
        for prec in ("fp32", "bf16"):
            out[prec] = train_bench(dev, steps=args.steps, warmup=args.warmup, precision=prec)
            log(f"bench: training {prec}: {out[prec]['ms_per_step']:.3f} ms/step")
        print(json.dumps({"training": out}))
        return

    from paper_2108_12430_amd import gwstream as gs
    from paper_2108_12430_amd import synth

    dev = torch.device("cuda:0")
    dc_s, bb_s = make_mix()
    layers = synth.deepclean_layers()
    stages = synth.bbhnet_stages()
    dc = gs.DeepClean(torch.from_numpy(synth.deepclean_params(0)).to(dev), layers)
    bb = gs.BBHnet(torch.from_numpy(synth.bbhnet_params(0)).to(dev), stages)
    dc.set_cu_budget(args.dc_cus)
    prec = gs.BF16 if args.precision == "bf16" else gs.FP32
    try:
        dc.workspace_bytes(1, DC_W, prec)
        probe = torch.zeros((1, DC_C, 64), device=dev)
        dc.forward(x=probe, noise=torch.empty((1, 64), device=dev), precision=prec)
    except gs.GwError as e:
        if e.code != gs.GW_EUNSUPPORTED:
            raise
        log(f"bench: {args.precision} path unavailable ({e}); measuring fp32")
        args.precision, prec = "fp32", gs.FP32
    if args.serve_only:
        rates = [float(r) for r in args.serve_rates.split(",") if r]
        print(json.dumps({"serving": serve_bench(dc, bb, prec, dc_s, bb_s, rates, args.serve_seconds, log)}))
        return

    # pool with every stream admitted
    ring = lambda c, w: ((c * w * 4 + 255) // 256 + (c * w * 2 + 255) // 256) * 256
    arena = N_DC * ring(DC_C, DC_W) + N_BB * ring(BB_C, BB_W) + (64 << 20)
    pool = gs.Pool(arena, max_slots=N_DC + N_BB, max_items=N_DC + N_BB)
    dc_slots = [pool.open(DC_C, DC_W) for _ in range(N_DC)]
    bb_slots = [pool.open(BB_C, BB_W) for _ in range(N_BB)]
    slots = dc_slots + bb_slots
    strides = np.concatenate([dc_s, bb_s])
    offsets = np.zeros(len(slots), np.int64)
    o = 0
    for i, s in enumerate(strides):
        offsets[i] = o
        o += (DC_C if i < N_DC else BB_C) * int(s)
    per_step_floats = o
    dc_strain_len = int(dc_s.sum())
    step_samples = int(strides.sum())
    log(f"bench: {len(slots)} streams admitted, {step_samples} new samples per step, precision {args.precision}")

    # synthetic sources (coloured-noise witnesses with mains lines; whitened detector noise)
    nsrc = 1 << 20
    wit, strain = synth.witness_stream(2, nsrc)
    wit_t = torch.from_numpy(wit).to(dev)
    strain_t = torch.from_numpy(strain).to(dev)
    bbx_t = torch.from_numpy(synth.gaussian(3, (BB_C, nsrc))).to(dev)
    # distinct staged inputs: one set per step up to 128, then reused in turn
    # (the rings still advance every step)
    n_steps_total = min(args.warmup + args.steps + args.lat_steps + 4, 128)
    pos = (np.arange(len(slots)) * 104729) % (nsrc // 2)
    staged, staged_strain = [], []
    for k in range(n_steps_total):
        blocks, sblocks = [], []
        for i, s in enumerate(strides):
            p = int(pos[i]) % (nsrc - 2048)
            if i < N_DC:
                blocks.append(wit_t[:, p:p + s].reshape(-1))
                sblocks.append(strain_t[p:p + s])
            else:
                blocks.append(bbx_t[:, p:p + s].reshape(-1))
            pos[i] += s
        staged.append(torch.cat(blocks).contiguous())
        staged_strain.append(torch.cat(sblocks).contiguous())
    staged, staged_strain = Cycle(staged), Cycle(staged_strain)
    assert staged[0].numel() == per_step_floats
    clean = torch.empty(dc_strain_len, device=dev)
    logits = torch.empty(N_BB, device=dev)
    ws_dc = torch.empty(dc.workspace_bytes(N_DC, DC_W, prec), dtype=torch.uint8, device=dev)
    ws_bb = torch.empty(bb.workspace_bytes(N_BB, BB_W, prec), dtype=torch.uint8, device=dev)
    dc_sl = np.array(dc_slots, np.int32)
    bb_sl = np.array(bb_slots, np.int32)
    torch.cuda.synchronize()
    log(f"bench: staged {n_steps_total} sets of step inputs in HBM")

    # the two model groups share no state: each runs its own ingest and
    # forward on its own HIP stream (default priorities), so neither waits
    # for the other; a timed loop ends with a device-wide synchronisation,
    # i.e. when both groups have finished every step
    s_main, s_bb = torch.cuda.current_stream(), torch.cuda.Stream()
    dc_str, bb_str = strides[:N_DC], strides[N_DC:]
    dc_off, bb_off = offsets[:N_DC], offsets[N_DC:]

    def bbh_group(k, st=None):
        st = s_bb if st is None else st
        pool.update(bb_sl, bb_str, staged[k], bb_off, stream=st)
        bb.forward(pool=pool, slots=bb_sl, W=BB_W, logits=logits, precision=prec, ws=ws_bb, stream=st)

    def run_models(k, flags, delays=None, dc_prec=None, bb_stream=None):
        # the DeepClean streams' update and forward in one call (one launch on
        # the fused BF16 path; the two calls otherwise); a request's new
        # samples are also its clean stride
        dc.update_forward(pool=pool, slots=dc_sl, strides=dc_s, samples=staged[k], offsets=dc_off, W=DC_W,
                          strain=staged_strain[k], clean=clean, precision=prec if dc_prec is None else dc_prec,
                          ws=ws_dc, flags=flags, delays=delays, stream=s_main)
        bbh_group(k, bb_stream)

    def step(k):
        run_models(k, 0, bb_stream=s_main if args.serial_groups else None)

    # ---- the whole step with its host copies (ingest_inclusive) ----------
    # Each step's requests are in pinned host memory, as a server's receive
    # buffers would hold them: one packed block per step with every stream's
    # new samples followed by the DeepClean streams' strain (NH distinct
    # blocks, reused in turn).  All host-device copies run in order on one
    # copy stream: step k's block goes into device staging buffer k mod 2 once
    # step k - 2 (that buffer's last reader) has finished, then step k - 1's
    # results (clean strain, logits) come back to pinned host memory once its
    # kernels have finished.  Step k's input copy thus overlaps step k - 1's
    # kernels, and a result copy never waits behind an input copy that has
    # not started.  Each model group waits for its step's input copy, updates
    # its rings from the staging buffer and runs its forward on its own
    # stream.  A step is complete when its results are in host memory; the
    # host keeps at most two steps in flight and observes completions by
    # polling their events.
    NH = min(16, n_steps_total)
    in_floats = per_step_floats + dc_strain_len
    host_in = []
    for j in range(NH):
        h = torch.empty(in_floats, dtype=torch.float32, pin_memory=True)
        h[:per_step_floats].copy_(staged[j])
        h[per_step_floats:].copy_(staged_strain[j])
        host_in.append(h)
    dev_in = [torch.empty(in_floats, device=dev) for _ in range(2)]
    dev_clean = [torch.empty(dc_strain_len, device=dev) for _ in range(2)]
    dev_logits = [torch.empty(N_BB, device=dev) for _ in range(2)]
    host_clean = [torch.empty(dc_strain_len, dtype=torch.float32, pin_memory=True) for _ in range(2)]
    host_logits = [torch.empty(N_BB, dtype=torch.float32, pin_memory=True) for _ in range(2)]
    s_cp = torch.cuda.Stream()
    ev_in = [torch.cuda.Event() for _ in range(2)]
    ev_dc = [torch.cuda.Event() for _ in range(2)]
    ev_bb = [torch.cuda.Event() for _ in range(2)]
    ev_res = [torch.cuda.Event() for _ in range(2)]
    torch.cuda.synchronize()

    def results_back(k):
        """Enqueue the copy of step k's results to the host (copy stream)."""
        b = k & 1
        s_cp.wait_event(ev_dc[b])
        s_cp.wait_event(ev_bb[b])
        with torch.cuda.stream(s_cp):
            host_clean[b].copy_(dev_clean[b], non_blocking=True)
            host_logits[b].copy_(dev_logits[b], non_blocking=True)
            ev_res[b].record(s_cp)

    def issue(k):
        b = k & 1
        db = dev_in[b]
        st_bb = s_main if args.serial_groups else s_bb
        # staging buffer b was last read by step k - 2, whose results were
        # copied back (after its kernels) earlier on this stream
        with torch.cuda.stream(s_cp):
            db.copy_(host_in[k % NH], non_blocking=True)
            ev_in[b].record(s_cp)
        if k >= 1:
            results_back(k - 1)
        s_main.wait_event(ev_in[b])
        # the update and the forward as two calls: in this copy-bound loop the
        # one-launch form (run_models) measured slower
        pool.update(dc_sl, dc_str, db, dc_off, stream=s_main)
        dc.forward(pool=pool, slots=dc_sl, W=DC_W, strides=dc_s, strain=db[per_step_floats:], clean=dev_clean[b],
                   precision=prec, ws=ws_dc, stream=s_main)
        ev_dc[b].record(s_main)
        if st_bb is not s_main:
            st_bb.wait_event(ev_in[b])
        pool.update(bb_sl, bb_str, db, bb_off, stream=st_bb)
        bb.forward(pool=pool, slots=bb_sl, W=BB_W, logits=dev_logits[b], precision=prec, ws=ws_bb, stream=st_bb)
        ev_bb[b].record(st_bb)

    def run_ingest(nsteps, k0):
        """Issue nsteps steps from k0 with at most two in flight; returns
        (wall seconds, per-step latency in ms from arrival to observed
        completion)."""
        t_issue = np.zeros(nsteps)
        t_done = np.zeros(nsteps)
        done = 0  # steps whose completion has been observed

        def observe(upto, block):
            # note the completion of steps done .. upto - 1 (their result
            # copies are enqueued once the next step has been issued)
            nonlocal done
            while done < upto:
                ev = ev_res[(k0 + done) & 1]
                if block:
                    while not ev.query():
                        pass
                elif not ev.query():
                    return
                t_done[done] = time.perf_counter()
                done += 1

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(nsteps):
            # results of steps up to i - 2 have been enqueued; wait for step
            # i - 2, so that steps i - 1 and i are the two in flight
            observe(i - 1, block=True)
            t_issue[i] = time.perf_counter()
            issue(k0 + i)
        results_back(k0 + nsteps - 1)
        observe(nsteps, block=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # saturated source: a stream's request for step i arrives when its
        # request for step i - 1 is issued
        t_arr = np.concatenate([[t_issue[0]], t_issue[:-1]])
        return wall, 1e3 * (t_done - t_arr)

    k = 0
    run_ingest(args.warmup, k)
    k += args.warmup
    log("bench: warmup done")
    # the host loop allocates small Python objects per call; a full cyclic
    # collection over the live objects would stall it for tens of ms, so
    # the timed loops run with the collector frozen (the calls create no
    # reference cycles)
    gc.collect()
    gc.freeze()
    gc.disable()
    dti, lati = run_ingest(args.steps, k)
    k += args.steps
    ingest = {"value": step_samples * args.steps / dti, "unit": "samples/s", "ms_per_step": 1e3 * dti / args.steps,
              "latency_ms": {"p50": float(np.percentile(lati, 50)), "p99": float(np.percentile(lati, 99)),
                             "max": float(lati.max())},
              "note": "the same step with its requests in pinned host memory: the host-to-device copy of the new "
                      "samples and strain, and the copy of the clean strain and logits back to the host, inside "
                      "the timed loop (PCIe-inclusive); latency from a request's arrival in host memory to the host "
                      "observing its results' copy"}
    log(f"bench: ingest-inclusive {ingest['ms_per_step']:.3f} ms/step, {ingest['value']:.4g} samples/s; "
        f"latency p50 {ingest['latency_ms']['p50']:.3f} ms p99 {ingest['latency_ms']['p99']:.3f} ms")

    # value: the same steps with every step's inputs already resident in HBM
    # when the timed loop starts (no host-device copies), at most two in
    # flight; a step is complete when both model groups' kernels are done
    ev_done = [(torch.cuda.Event(), torch.cuda.Event()) for _ in range(2)]

    def run_resident(nsteps, k0):
        t_issue = np.zeros(nsteps)
        t_done = np.zeros(nsteps)
        done = 0

        def observe(upto):
            nonlocal done
            while done < upto:
                e1, e2 = ev_done[(k0 + done) & 1]
                while not (e1.query() and e2.query()):
                    pass
                t_done[done] = time.perf_counter()
                done += 1

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(nsteps):
            observe(i - 1)  # steps i - 1 and i in flight
            t_issue[i] = time.perf_counter()
            step(k0 + i)
            e1, e2 = ev_done[(k0 + i) & 1]
            e1.record(s_main)
            e2.record(s_main if args.serial_groups else s_bb)
        observe(nsteps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        t_arr = np.concatenate([[t_issue[0]], t_issue[:-1]])
        return wall, 1e3 * (t_done - t_arr)

    run_resident(args.warmup, k)
    k += args.warmup
    dt, lat = run_resident(args.steps, k)
    k += args.steps
    gc.enable()
    gc.unfreeze()
    ms_per_step = 1e3 * dt / args.steps
    value = step_samples * args.steps / dt
    log(f"bench: {ms_per_step:.3f} ms/step, {value:.4g} samples/s (inputs resident in HBM); "
        f"latency p50 {np.percentile(lat, 50):.3f} ms p99 {np.percentile(lat, 99):.3f} ms")

    if args.copy_calibration:
        # a plain copy of known size, so hardware byte counters can be scaled
        nb = args.copy_calibration << 20
        a = torch.empty(nb // 4, dtype=torch.float32, device=dev).fill_(1.0)
        c = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        log(f"bench: copy calibration {args.copy_calibration} MiB x 3")
        del a, c

    # fully-online output only (GW_CAUSAL): the DeepClean streams compute just
    # the band of each window that their newest samples depend on
    def step_band(k):
        run_models(k, gs.CAUSAL)

    band = None
    if not args.no_band:
        kb = 0
        for _ in range(args.warmup):
            step_band(kb % n_steps_total)
            kb += 1
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step_band(kb % n_steps_total)
            kb += 1
        torch.cuda.synchronize()
        dtb = time.perf_counter() - t0
        latb = []
        for _ in range(args.lat_steps):
            t1 = time.perf_counter()
            step_band(kb % n_steps_total)
            torch.cuda.synchronize()
            latb.append(1e3 * (time.perf_counter() - t1))
            kb += 1
        latb = np.array(latb) if latb else np.zeros(1)
        band = {"value": step_samples * args.steps / dtb, "unit": "samples/s", "ms_per_step": 1e3 * dtb / args.steps,
                "sync_step_p50_ms": float(np.percentile(latb, 50)), "sync_step_p99_ms": float(np.percentile(latb, 99)),
                "inputs": "resident in HBM",
                "note": "DeepClean computes only the receptive-field band of each window its newest samples need; "
                        "clean output bitwise equal to the full-window recompute"}
        log(f"bench: causal band {band['value']:.4g} samples/s, {band['ms_per_step']:.3f} ms/step, "
            f"synchronous step p99 {band['sync_step_p99_ms']:.3f} ms")

    # output aggregation variants (App. B): a 0.75-s aggregation latency on
    # every DeepClean stream (causal band reaching back s + delay), and the
    # average of each output over the 4 latest overlapping predictions (full
    # noise windows, then deepclean_overlap_average with per-stream state)
    agg = precision_leg = None
    if not args.no_agg and prec == gs.BF16:
        delay = int(0.75 * 4096)
        dls = np.full(N_DC, delay, np.int32)
        depth = 4
        noise_full = torch.empty((N_DC, DC_W), device=dev)
        ws_full = torch.empty(dc.workspace_bytes(N_DC, DC_W, prec), dtype=torch.uint8, device=dev)
        state = torch.zeros(dc.overlap_state_floats(dc_s, depth), device=dev)
        cnt = [0]

        def step_delay(k):
            run_models(k, gs.CAUSAL, dls)

        def step_avg(k):
            dc.update_forward(pool=pool, slots=dc_sl, strides=dc_s, samples=staged[k], offsets=dc_off, W=DC_W,
                              noise=noise_full, precision=prec, ws=ws_full, stream=s_main)
            dc.overlap_average(noise=noise_full, strides=dc_s, depth=depth, counts=[cnt[0]] * N_DC, state=state,
                               strain=staged_strain[k], clean=clean)
            cnt[0] += 1
            bbh_group(k)

        def step_f16(k):
            run_models(k, 0, dc_prec=gs.FP16)

        # the same outputs over per-stream activation caches: each update
        # recomputes only every layer's dirty bands and yields the full noise
        # window (the first call per stream, in the warmup, computes it all)
        caches = [dc.new_cache(DC_W) for _ in range(N_DC)]
        for sl_, c_ in zip(dc_slots, caches):
            pool.attach_cache(sl_, c_)
        state_c = torch.zeros_like(state)
        cnt_c = [0]

        def step_cavg(k):
            pool.update(dc_sl, dc_str, staged[k], dc_off, stream=s_main)
            dc.forward_cached(pool=pool, slots=dc_sl, W=DC_W, noise=noise_full, stream=s_main)
            dc.overlap_average(noise=noise_full, strides=dc_s, depth=depth, counts=[cnt_c[0]] * N_DC, state=state_c,
                               strain=staged_strain[k], clean=clean)
            cnt_c[0] += 1
            bbh_group(k)

        def step_cdelay(k):
            pool.update(dc_sl, dc_str, staged[k], dc_off, stream=s_main)
            dc.forward_cached(pool=pool, slots=dc_sl, W=DC_W, strides=dc_s, strain=staged_strain[k], clean=clean,
                              delays=dls, stream=s_main)
            bbh_group(k)

        agg = {}
        for name, fn in (("delay_0.75s_band", step_delay), ("overlap_average_depth4", step_avg),
                         ("deepclean_fp16", step_f16), ("overlap_average_depth4_cached", step_cavg),
                         ("delay_0.75s_cached", step_cdelay)):
            ka = 0
            for _ in range(args.warmup):
                fn(ka % n_steps_total)
                ka += 1
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fn(ka % n_steps_total)
                ka += 1
            torch.cuda.synchronize()
            dta = time.perf_counter() - t0
            agg[name] = {"value": step_samples * args.steps / dta, "unit": "samples/s",
                         "ms_per_step": 1e3 * dta / args.steps}
            log(f"bench: variant {name}: {agg[name]['value']:.4g} samples/s, "
                f"{agg[name]['ms_per_step']:.3f} ms/step")
        gs.profile_begin()
        for _ in range(5):
            step_cavg(ka % n_steps_total)
            ka += 1
        prof_c = gs.profile_end()
        agg["cache_kernels_ms_per_step"] = {k2: round(v[1] / 5, 4) for k2, v in sorted(prof_c.items())
                                            if k2.startswith("cache_")}
        gs.profile_begin()
        for _ in range(5):
            step_avg(ka % n_steps_total)
            ka += 1
        prof_a = gs.profile_end()
        if "overlap_average" in prof_a:
            c_, t_ = prof_a["overlap_average"]
            # per launch: read the windows' last depth*s samples, read+write the
            # state, read strain, write clean
            by = 4.0 * float(np.sum(dc_s)) * (depth + 2 * depth + 2)
            agg["overlap_average_kernel"] = {"avg_us": 1e3 * t_ / c_, "algorithmic_bytes": by,
                                             "achieved_GBs": by / (t_ / c_ * 1e-3) / 1e9}
        agg["note"] = ("delay: clean = strain - noise[W-s-d, W-d) with d = 3072 samples (0.75 s), causal band; "
                       "average: full noise windows, then the mean over the 4 latest predictions of each sample; "
                       "_cached: the same outputs from per-stream activation caches (every layer recomputes only "
                       "its dirty bands per update; full noise window bitwise equal to recomputing it)")
        precision_leg = {"deepclean_fp16": agg.pop("deepclean_fp16"),
                         "note": "the main step with FP16 operands in the fused DeepClean kernel (BBHnet BF16)"}
        for sl_ in dc_slots:
            pool.attach_cache(sl_, None)
        del noise_full, ws_full, state, state_c, caches

    # end-to-end ensemble (main text, second offline workflow): per request,
    # both detectors' witness rings, DeepClean-H1 and -L1 with the clean
    # output, decimation to 2048 Hz into the BBHnet ring, BBHnet logits
    ens = None
    if not args.no_ens and prec == gs.BF16:
        from paper_2108_12430_amd import ensemble
        n_e, s_e = 64, 256
        dc_l1 = gs.DeepClean(torch.from_numpy(synth.deepclean_params(1)).to(dev), layers)
        dc.set_cu_budget(0)  # one stream: nothing runs beside the DeepClean kernels
        e = ensemble.Ensemble(dc, dc_l1, bb, n_e, W_dc=DC_W, W_bb=BB_W, stride=s_e, precision=prec, pipeline=True)
        g = torch.Generator(device="cpu").manual_seed(11)
        e.prefill(torch.randn((2, n_e, DC_C, DC_W), generator=g).to(dev))
        wits = [torch.randn((2, n_e, DC_C, s_e), generator=g).to(dev) for _ in range(8)]
        sts = [torch.randn((2, n_e, s_e), generator=g).to(dev) for _ in range(8)]
        for k in range(args.warmup):
            e.step(wits[k % 8], sts[k % 8])
        torch.cuda.synchronize()
        gc.collect()
        gc.freeze()
        gc.disable()
        t0 = time.perf_counter()
        for k in range(args.steps):
            e.step(wits[k % 8], sts[k % 8])
        torch.cuda.synchronize()
        dte = time.perf_counter() - t0
        gc.enable()
        gc.unfreeze()
        ms_e = 1e3 * dte / args.steps
        ens = {"streams": n_e, "stride": s_e, "ms_per_step": ms_e, "pipelined": True,
               "strain_samples_per_s": 2 * n_e * s_e / (ms_e * 1e-3),
               "data_seconds_per_s": n_e * s_e / 4096 / (ms_e * 1e-3),
               "config": f"{n_e} ensemble streams: 2 x (21 x {DC_W}) witness snapshots at 4096 Hz, "
                         f"BBHnet 2 x {BB_W} at 2048 Hz, {s_e} new samples per request"}
        log(f"bench: ensemble {ms_e:.3f} ms/step, {ens['data_seconds_per_s']:.1f} s of data per s")
        del e, dc_l1, wits, sts
        dc.set_cu_budget(args.dc_cus)

    roof = None
    if not args.no_roofline:
        # each kernel timed on its own: the step's two groups one after the
        # other on one stream (in the timed loop they overlap, and a launch's
        # duration there includes the other group's kernels on its CUs)
        def step_serial(k):
            run_models(k, 0, bb_stream=s_main)

        kp = 0
        for _ in range(args.warmup):
            step_serial(kp % n_steps_total)
            kp += 1
        gs.profile_begin()
        for _ in range(ROOF_STEPS):
            step_serial(kp % n_steps_total)
            kp += 1
        prof = gs.profile_end()
        name, (cnt, tot) = max(prof.items(), key=lambda kv: kv[1][1])
        avg_s = tot / cnt / 1e3
        flops, by = algorithmic(name, args.precision, layers, dc_s, bb_s)
        if args.precision == "fp32":
            roof = {"bound": "alu", "achieved": flops / avg_s / 1e12, "peak": FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s"}
        elif flops / max(by, 1.0) > BF16_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9):
            roof = {"bound": "mfma", "achieved": flops / avg_s / 1e12, "peak": BF16_PEAK_TFLOPS,
                    "unit": "TFLOP/s"}
        else:
            roof = {"bound": "hbm", "achieved": by / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        roof["frac"] = roof["achieved"] / roof["peak"]
        roof["traffic"] = traffic_for(name)
        roof["kernel"] = name
        roof["avg_us"] = avg_s * 1e6
        if name == "dc_fused_bf16":
            # the step runs the fused kernel on its CU budget, beside BBHnet
            roof["cus"] = min(args.dc_cus, N_CUS) if args.dc_cus > 0 else N_CUS
        roof["algorithmic_flops"] = flops
        roof["algorithmic_bytes"] = by
        step_ms = sum(v[1] for v in prof.values()) / ROOF_STEPS
        roof["kernels_ms_per_step"] = {k2: round(v[1] / ROOF_STEPS, 4) for k2, v in sorted(prof.items())}
        log(f"bench: dominant kernel {name} avg {avg_s * 1e6:.1f} us; kernel sum {step_ms:.3f} ms/step")

    plain = None
    if not args.no_plain:
        ws1 = torch.empty(dc.workspace_bytes(1, DC_W, gs.FP32), dtype=torch.uint8, device=dev)
        wsb1 = torch.empty(bb.workspace_bytes(1, BB_W, gs.FP32), dtype=torch.uint8, device=dev)
        lat_plain, times = [], []
        for _ in range(args.plain_steps):
            kk = k % n_steps_total
            ev0 = torch.cuda.Event(enable_timing=True)
            evs = []
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ev0.record()
            # the step's requests from pinned host memory, then one stream at a time
            din = dev_in[0]
            din.copy_(host_in[kk % NH], non_blocking=True)
            for i, sl in enumerate(slots):
                pool.update([sl], [strides[i]], din, [offsets[i]])
                if i < N_DC:
                    so = per_step_floats + int(dc_s[:i].sum())
                    dc.forward(pool=pool, slots=[sl], W=DC_W, strides=[dc_s[i]],
                               strain=din[so:so + int(dc_s[i])], clean=clean[so - per_step_floats:so - per_step_floats + int(dc_s[i])],
                               precision=gs.FP32, ws=ws1)
                else:
                    bb.forward(pool=pool, slots=[sl], W=BB_W, logits=logits[i - N_DC:i - N_DC + 1],
                               precision=gs.FP32, ws=wsb1)
                e = torch.cuda.Event(enable_timing=True)
                e.record()
                evs.append(e)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
            lat_plain += [ev0.elapsed_time(e) for e in evs]
            k += 1
        tp = float(np.mean(times))
        plain = {"value": step_samples / tp, "unit": "samples/s", "ms_per_step": 1e3 * tp,
                 "p50_ms": float(np.percentile(lat_plain, 50)), "p99_ms": float(np.percentile(lat_plain, 99)),
                 "dtype": "f32", "batching": "one stream per launch"}
        log(f"bench: fp32 plain {plain['value']:.4g} samples/s, p99 {plain['p99_ms']:.3f} ms")

    training = None
    if not args.no_train:
        training = {"fp32": train_bench(dev), "bf16_conv": train_bench(dev, precision="bf16")}
        log(f"bench: training step {training}")

    bbh_batches = d0 = None
    if not args.no_extra:
        bbh_batches = bbhnet_batch_bench(dev)
        log(f"bench: bbhnet batches {bbh_batches}")
        d0 = d0_latency(dev)
        log(f"bench: deepclean 1-s window fp32 latency {d0}")

    serving = None
    if not args.no_serve:
        rates = [float(r) for r in args.serve_rates.split(",") if r]
        serving = serve_bench(dc, bb, prec, dc_s, bb_s, rates, args.serve_seconds, log)

    out = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.precision if args.precision == "bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": "closed-loop serving mix: 179 DeepClean streams (21 ch x 32768, 4096 Hz) + "
                               "77 BBHnet streams (2 ch x 2048, 2048 Hz), strides 1/16-1/4 s",
                   "streams": N_DC + N_BB, "samples_per_step": step_samples, "deepclean_cus": args.dc_cus,
                   "channel_samples_per_step": int(DC_C * dc_s.sum() + BB_C * bb_s.sum())},
        "channel_samples_per_s": value * (DC_C * dc_s.sum() + BB_C * bb_s.sum()) / step_samples,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max()),
                       "definition": "host time from a request's arrival (its samples resident in HBM) to the host "
                                     "observing its step's completion events, over the timed steps; saturated "
                                     "source (a stream's next request arrives when its previous one is issued), "
                                     "two steps in flight"},
        "ingest_inclusive": ingest,
        "bbhnet_batches": bbh_batches, "deepclean_1s_fp32": d0,
        "fp32_plain": plain, "causal_band": band, "aggregation": agg, "precision": precision_leg, "ensemble": ens, "serving": serving, "training": training, "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
