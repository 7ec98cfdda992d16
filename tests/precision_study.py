"""Operand-precision study of the DeepClean and BBHnet forwards on the CPU.

The paper served DeepClean in FP16 under TensorRT (App. B.4); gfx950 also has
FP8 matrix cores (OCP e4m3 and e5m2).  This study measures what rounding the
convolution operands to each 16- or 8-bit format does to the outputs, with
the FP64 oracle's layer definitions and everything else exact: for every
convolution the input activations and the weights are rounded to the format
(round to nearest even, saturating at the format's largest finite value),
the products are summed in float64, and the bias, normalisation and tanh
(or ReLU) stay exact, as in the kernels' FP32 epilogues.  FP8 operands are
optionally scaled per tensor by a power of two that maps the tensor's
largest magnitude to just below the format's maximum (undone after the
sum).  The error of an output tensor is normwise: max |y - y_ref| / max
|y_ref| (the measure every parity test uses).

    python tests/precision_study.py      # prints the tables

Test infrastructure: uses the oracle's definitions, never the device path.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import ref  # noqa: E402
from paper_2108_12430_amd import synth  # noqa: E402

FORMATS = {
    "bf16": (torch.bfloat16, None),
    "fp16": (torch.float16, 65504.0),
    "e4m3": (torch.float8_e4m3fn, 448.0),
    "e5m2": (torch.float8_e5m2, 57344.0),
}


def round_to(x, fmt, scaled=False):
    """Round float64 values to `fmt` (nearest even, saturating) and back.
    scaled: multiply by 2^k first, k the largest integer with
    max|x| 2^k <= the format's maximum, and divide afterwards."""
    if fmt is None:
        return np.asarray(x, np.float64)
    dt, vmax = FORMATS[fmt]
    x = np.asarray(x, np.float64)
    k = 0
    if scaled and vmax is not None:
        amax = float(np.max(np.abs(x)))
        if amax > 0:
            k = int(np.floor(np.log2(vmax / amax)))
    y = x * 2.0 ** k
    if vmax is not None:
        y = np.clip(y, -vmax, vmax)
    y = torch.from_numpy(y).to(torch.float32).to(dt).to(torch.float64).numpy()
    return y / 2.0 ** k


def rel(y, yref):
    return float(np.max(np.abs(y - yref)) / np.max(np.abs(yref)))


def deepclean_rounded(params, x, fmts, scaled=False, layers=ref.DEEPCLEAN_LAYERS):
    """Inference forward with the operands of layer l rounded to fmts[l]
    (None: exact)."""
    ps = ref.unpack_deepclean(params, layers)
    a = np.asarray(x, np.float64)
    for l, ((typ, ci, co, k, s, pad, op, bn), d) in enumerate(zip(layers, ps)):
        f = fmts[l]
        w = round_to(d["w"], f, scaled)
        ar = round_to(a, f, scaled)
        if typ == "conv":
            z = ref.conv1d(ar, w, d["b"], s, pad)
        else:
            z = ref.conv_transpose1d(ar, w, d["b"], s, pad, op)
        a = np.tanh(ref.batchnorm_infer(z, d["gamma"], d["beta"], d["mean"], d["var"])) if bn else z
    return a[:, 0, :]


def bbhnet_rounded(params, x, fmt, scaled=False, stages=ref.BBHNET_STAGES):
    """BBHnet forward with every convolution's operands rounded to fmt."""
    ps, head = ref.unpack_bbhnet(params, stages)
    a = np.asarray(x, np.float64)
    for d in ps:
        ar = round_to(a, fmt, scaled)
        h = np.maximum(ref.conv1d(ar, round_to(d["wa"], fmt, scaled), d["ba"], 2, 3), 0.0)
        h = ref.conv1d(round_to(h, fmt, scaled), round_to(d["wb"], fmt, scaled), d["bb"], 1, 3)
        sc = ref.conv1d(ar, round_to(d["ws"], fmt, scaled), d["bs"], 2, 0)
        a = np.maximum(h + sc, 0.0)
    return a.mean(axis=2) @ head["w"][0] + head["b"][0]


def deepclean_table(W=32768, batch=2, seed=21):
    """Whole-network error per format, and per layer (only that layer's
    operands rounded) for the FP8 formats."""
    params = synth.deepclean_params(0)
    wit, _ = synth.witness_stream(seed, batch * W)
    x = np.ascontiguousarray(wit.reshape(21, batch, W).transpose(1, 0, 2))
    yref = ref.deepclean_forward(params, x)
    L = len(ref.DEEPCLEAN_LAYERS)
    out = {"whole": {}, "per_layer": {}}
    for f in FORMATS:
        out["whole"][f] = rel(deepclean_rounded(params, x, [f] * L), yref)
    for f in ("e4m3", "e5m2"):
        out["whole"][f + "_scaled"] = rel(deepclean_rounded(params, x, [f] * L, scaled=True), yref)
        out["per_layer"][f + "_scaled"] = [
            rel(deepclean_rounded(params, x, [f if j == l else None for j in range(L)], scaled=True), yref)
            for l in range(L)]
    return out


def mixed_fp8(W=32768, batch=2, seed=21, bound=2e-2, fp8="e4m3"):
    """Greedy mixed precision: starting from BF16 on every layer, move layers
    to scaled FP8 in order of their single-layer FP8 error while the whole
    network stays within `bound`.  Returns (layers in FP8, error)."""
    params = synth.deepclean_params(0)
    wit, _ = synth.witness_stream(seed, batch * W)
    x = np.ascontiguousarray(wit.reshape(21, batch, W).transpose(1, 0, 2))
    yref = ref.deepclean_forward(params, x)
    L = len(ref.DEEPCLEAN_LAYERS)
    single = [rel(deepclean_rounded(params, x, [fp8 if j == l else None for j in range(L)], scaled=True), yref)
              for l in range(L)]
    chosen = []
    err = rel(deepclean_rounded(params, x, ["bf16"] * L), yref)
    for l in np.argsort(single):
        trial = chosen + [int(l)]
        # mixed: FP8 (scaled) on the chosen layers, BF16 elsewhere
        ps = ref.unpack_deepclean(params)
        a = np.asarray(x, np.float64)
        for j, ((typ, ci, co, k, s, pad, op, bn), d) in enumerate(zip(ref.DEEPCLEAN_LAYERS, ps)):
            f, sc = (fp8, True) if j in trial else ("bf16", False)
            w, ar = round_to(d["w"], f, sc), round_to(a, f, sc)
            z = ref.conv1d(ar, w, d["b"], s, pad) if typ == "conv" else ref.conv_transpose1d(ar, w, d["b"], s, pad, op)
            a = np.tanh(ref.batchnorm_infer(z, d["gamma"], d["beta"], d["mean"], d["var"])) if bn else z
        e = rel(a[:, 0, :], yref)
        if e > bound:
            break
        chosen, err = trial, e
    return sorted(chosen), err


def bbhnet_table(batch=64, seed=23):
    params = synth.bbhnet_params(0)
    x, _ = synth.bbh_windows(seed, batch)
    yref = ref.bbhnet_forward(params, x)
    out = {}
    for f in FORMATS:
        out[f] = rel(bbhnet_rounded(params, x, f), yref)
    for f in ("e4m3", "e5m2"):
        out[f + "_scaled"] = rel(bbhnet_rounded(params, x, f, scaled=True), yref)
    return out


if __name__ == "__main__":
    t = deepclean_table()
    print("DeepClean, 2 windows of 21 x 32768, normwise error of the noise output")
    for k, v in t["whole"].items():
        print(f"  all layers {k:12s} {v:.2e}")
    for k, v in t["per_layer"].items():
        print(f"  one layer  {k:12s} " + " ".join(f"L{l}:{e:.1e}" for l, e in enumerate(v)))
    ch, e = mixed_fp8()
    print(f"  greedy mixed (scaled e4m3 on layers {ch}, BF16 elsewhere): {e:.2e}")
    b = bbhnet_table()
    print("BBHnet, 64 windows of 2 x 2048, normwise error of the logits")
    for k, v in b.items():
        print(f"  {k:12s} {v:.2e}")
