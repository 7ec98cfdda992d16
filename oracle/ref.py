"""FP64 CPU oracle for the streaming 1-D CNN hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
calls this module; only the tests, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the device path: the two meet only
in the seeded input generators, which hold none of the arithmetic below.

Everything here is the plain definition written out in float64 with numpy,
with no blocking, fusion or reordering beyond the definitions:

* the stateful "snapshotter" model (App. B.1): each request carries floor(f_s/r)
  strictly new samples that update the held snapshot, i.e. after n requests the
  snapshot is the last W samples of the stream so far (zero before the start);
* the static models fed by that snapshot: a DeepClean-shaped 1-D convolutional
  autoencoder (main text, DeepClean paragraph) and a BBHnet-shaped 1-D CNN
  classifier (main text, BBHnet paragraph);
* causal ("fully-online") output selection: each prediction keeps only its
  most recent floor(f_s/r) samples (App. B.2), and the cleaned strain is strain
  minus the predicted noise (App. B.4, client pipeline);
* the training-step gradient used for DeepClean retraining (main text,
  retraining paragraph) with a band-passed mean-squared-error loss.

Layer shapes are not given in the paper; the readings used are listed in the
design notes of the repository (Conv1d/ConvTranspose1d are cross-correlations
with PyTorch's weight layouts; transposed layers use output_padding 1 so the
length doubles; BatchNorm eps = 1e-5).

Every function is pinned by the CPU tests against brute-force loops, library
routines (numpy.correlate/convolve, torch CPU ops in float64), closed forms,
invariants or finite differences.
"""
from __future__ import annotations

import numpy as np

BN_EPS = 1e-5

# (type, C_in, C_out, k, stride, pad, out_pad, bn_tanh): DeepClean-shaped net,
# four strided encoder convs, four transposed decoder convs, one linear output conv.
DEEPCLEAN_LAYERS = (
    [("conv", ci, co, 7, 2, 3, 0, True) for ci, co in ((21, 8), (8, 16), (16, 32), (32, 64))]
    + [("convT", ci, co, 7, 2, 3, 1, True) for ci, co in ((64, 32), (32, 16), (16, 8), (8, 8))]
    + [("conv", 8, 1, 7, 1, 3, 0, False)]
)

BBHNET_STAGES = ((2, 32), (32, 64), (64, 128))


# ---------------------------------------------------------------------------
# Elementary operations (definitions)
# ---------------------------------------------------------------------------

def conv1d(x, w, b, stride, pad):
    """y[b,o,t] = bias[o] + sum_{i,j} w[o,i,j] * xz[b,i,stride*t - pad + j],
    xz = x with zeros outside [0, L); L_out = floor((L + 2 pad - k)/stride) + 1.
    x: [B][C_in][L], w: [C_out][C_in][k]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    B, ci, L = x.shape
    co, ci2, k = w.shape
    assert ci == ci2
    lout = (L + 2 * pad - k) // stride + 1
    xp = np.zeros((B, ci, L + 2 * pad + stride), np.float64)
    xp[:, :, pad:pad + L] = x
    y = np.zeros((B, co, lout), np.float64)
    for j in range(k):
        cols = xp[:, :, j: j + stride * (lout - 1) + 1: stride]  # [B][ci][lout]
        # sum over C_in of w[:, :, j] with the tap-j columns, as one matrix product
        y += np.tensordot(w[:, :, j], cols, axes=([1], [1])).transpose(1, 0, 2)
    if b is not None:
        y += np.asarray(b, np.float64)[None, :, None]
    return y


def conv_transpose1d(x, w, b, stride, pad, out_pad):
    """y[b,o,u] = bias[o] + sum_{i,t,j} [u == stride*t - pad + j] w[i,o,j] x[b,i,t],
    L_out = (L - 1) stride - 2 pad + k + out_pad.  x: [B][C_in][L], w: [C_in][C_out][k]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    B, ci, L = x.shape
    ci2, co, k = w.shape
    assert ci == ci2
    lout = (L - 1) * stride - 2 * pad + k + out_pad
    full = np.zeros((B, co, max((L - 1) * stride + k, pad + lout)), np.float64)
    for j in range(k):
        full[:, :, j: j + stride * (L - 1) + 1: stride] += np.tensordot(
            w[:, :, j], x, axes=([0], [1])).transpose(1, 0, 2)
    y = full[:, :, pad: pad + lout].copy()
    if b is not None:
        y += np.asarray(b, np.float64)[None, :, None]
    return y


def batchnorm_infer(y, gamma, beta, mean, var, eps=BN_EPS):
    """gamma (y - mean) / sqrt(var + eps) + beta, per channel (axis 1)."""
    c = lambda v: np.asarray(v, np.float64)[None, :, None]
    return c(gamma) * (y - c(mean)) / np.sqrt(c(var) + eps) + c(beta)


def batchnorm_train(y, gamma, beta, eps=BN_EPS):
    """Batch statistics over (batch, time): biased variance.
    Returns (out, mean, var)."""
    mean = y.mean(axis=(0, 2))
    var = ((y - mean[None, :, None]) ** 2).mean(axis=(0, 2))
    return batchnorm_infer(y, gamma, beta, mean, var, eps), mean, var


# ---------------------------------------------------------------------------
# DeepClean-shaped network
# ---------------------------------------------------------------------------

def unpack_deepclean(params, layers=DEEPCLEAN_LAYERS):
    """Split the flat parameter vector (per layer: weight, bias, then if BN:
    gamma, beta, running mean, running var) into per-layer float64 arrays."""
    p = np.asarray(params, np.float64)
    off = 0
    out = []
    for (typ, ci, co, k, s, pad, op, bn) in layers:
        shape = (co, ci, k) if typ == "conv" else (ci, co, k)
        n = ci * co * k
        d = {"w": p[off: off + n].reshape(shape)}
        off += n
        d["b"] = p[off: off + co]
        off += co
        if bn:
            for name in ("gamma", "beta", "mean", "var"):
                d[name] = p[off: off + co]
                off += co
        out.append(d)
    assert off == p.size, (off, p.size)
    return out


def n_params(layers=DEEPCLEAN_LAYERS):
    n = 0
    for (typ, ci, co, k, s, pad, op, bn) in layers:
        n += ci * co * k + co + (4 * co if bn else 0)
    return n


def _layer_linear(typ, a, d, s, pad, op):
    if typ == "conv":
        return conv1d(a, d["w"], d["b"], s, pad)
    return conv_transpose1d(a, d["w"], d["b"], s, pad, op)


def deepclean_forward(params, x, layers=DEEPCLEAN_LAYERS, train=False, keep=False):
    """Network output (predicted noise) for witness windows x [B][C][W].

    Inference mode uses the stored running statistics; train mode uses batch
    statistics.  Returns noise [B][W] (float64), plus the per-layer cache when
    keep=True (used by the gradient)."""
    ps = unpack_deepclean(params, layers)
    a = np.asarray(x, np.float64)
    cache = []
    for (typ, ci, co, k, s, pad, op, bn), d in zip(layers, ps):
        a_in = a
        z = _layer_linear(typ, a, d, s, pad, op)
        ent = {"a_in": a_in, "z": z}
        if bn:
            if train:
                h, m, v = batchnorm_train(z, d["gamma"], d["beta"])
            else:
                m, v = d["mean"], d["var"]
                h = batchnorm_infer(z, d["gamma"], d["beta"], m, v)
            ent.update(mean=np.asarray(m, np.float64), var=np.asarray(v, np.float64))
            a = np.tanh(h)
        else:
            a = z
        ent["a"] = a
        cache.append(ent)
    noise = a[:, 0, :]
    return (noise, cache) if keep else noise


def deepclean_grad(params, x, dnoise, layers=DEEPCLEAN_LAYERS):
    """Gradient of a scalar loss with respect to the flat parameter vector,
    given dL/dnoise [B][W], for the train-mode (batch-statistics) forward.

    Per layer, in reverse: tanh' = 1 - tanh^2; batch-norm backward
    dz = gamma/sigma * (dh - mean(dh) - xhat * mean(dh * xhat)),
    dgamma = sum dh*xhat, dbeta = sum dh; bias grad = sum dz; weight grad is the
    correlation of dz with the (zero-padded) layer input; input grad is the
    adjoint convolution (transposed conv for a conv layer, conv for a transposed
    layer).  Running mean/var get zero gradient."""
    ps = unpack_deepclean(params, layers)
    _, cache = deepclean_forward(params, x, layers, train=True, keep=True)
    g = np.asarray(dnoise, np.float64)[:, None, :]
    grads = []
    for (typ, ci, co, k, s, pad, op, bn), d, ent in reversed(list(zip(layers, ps, cache))):
        gd = {}
        if bn:
            a = ent["a"]
            dh = g * (1.0 - a * a)
            sig = np.sqrt(ent["var"] + BN_EPS)
            xhat = (ent["z"] - ent["mean"][None, :, None]) / sig[None, :, None]
            gd["gamma"] = (dh * xhat).sum(axis=(0, 2))
            gd["beta"] = dh.sum(axis=(0, 2))
            gd["mean"] = np.zeros(co)
            gd["var"] = np.zeros(co)
            mdh = dh.mean(axis=(0, 2))[None, :, None]
            mdhx = (dh * xhat).mean(axis=(0, 2))[None, :, None]
            dz = (d["gamma"] / sig)[None, :, None] * (dh - mdh - xhat * mdhx)
        else:
            dz = g
        a_in = ent["a_in"]
        gd["b"] = dz.sum(axis=(0, 2))
        L_in = a_in.shape[2]
        if typ == "conv":
            lout = dz.shape[2]
            xp = np.zeros((a_in.shape[0], ci, L_in + 2 * pad + s), np.float64)
            xp[:, :, pad:pad + L_in] = a_in
            dw = np.zeros((co, ci, k))
            for j in range(k):
                cols = xp[:, :, j: j + s * (lout - 1) + 1: s]
                dw[:, :, j] = np.einsum("bot,bit->oi", dz, cols, optimize=True)
            gd["w"] = dw
            op_adj = L_in - ((lout - 1) * s - 2 * pad + k)
            g = conv_transpose1d(dz, d["w"], None, s, pad, op_adj)
        else:
            lout = dz.shape[2]
            dzp = np.zeros((dz.shape[0], co, lout + 2 * pad + s * L_in + k), np.float64)
            dzp[:, :, pad:pad + lout] = dz
            dw = np.zeros((ci, co, k))
            for j in range(k):
                cols = dzp[:, :, j: j + s * (L_in - 1) + 1: s]  # dz[s t - pad + j]
                dw[:, :, j] = np.einsum("bit,bot->io", a_in, cols, optimize=True)
            gd["w"] = dw
            g = conv1d(dz, d["w"], None, s, pad)
            assert g.shape[2] == L_in
        grads.append((bn, gd))
    flat = []
    for bn, gd in reversed(grads):
        flat.append(gd["w"].ravel())
        flat.append(gd["b"])
        if bn:
            for name in ("gamma", "beta", "mean", "var"):
                flat.append(gd[name])
    return np.concatenate(flat)


# ---------------------------------------------------------------------------
# Snapshot state and causal output (App. B.1, B.2)
# ---------------------------------------------------------------------------

def snapshot_after(stream, n_samples, W):
    """Closed form of the snapshot after the first n_samples of a stream
    [C][N] have been sent: the last W samples of (W zeros ++ stream[:n])."""
    stream = np.asarray(stream)
    c = stream.shape[0]
    z = np.concatenate([np.zeros((c, W), stream.dtype), stream[:, :n_samples]], axis=1)
    return z[:, -W:]


def snapshot_update(state, new):
    """The stateful model's update: append the strictly new samples [C][s] to
    the held snapshot [C][W] and keep the most recent W."""
    W = state.shape[1]
    return np.concatenate([state, new], axis=1)[:, -W:]


def causal_clean(noise, strain_new):
    """Fully-online output: keep the most recent s predicted samples of each
    window and subtract them from the s newest strain samples.
    noise [B][W], strain_new [B][s] -> (noise_tail [B][s], clean [B][s])."""
    s = strain_new.shape[-1]
    tail = np.asarray(noise, np.float64)[..., -s:]
    return tail, np.asarray(strain_new, np.float64) - tail


def overlap_average(windows, s, depth):
    """Aggregation of overlapping predictions (App. B.2: successive output
    segments overlap and differ; averaging them costs latency).  windows
    [K][W]: the predictions of requests 0..K-1 of one stream with stride s,
    window k ending at t_k = t_0 + k s.  Output k covers the absolute span
    [t_k - depth s, t_k - (depth - 1) s), which every window k - i, i = 0..
    depth-1, contains at positions W - (depth - i) s .. W - (depth - 1 - i) s;
    it is the mean over the windows among those that exist (k - i >= 0).
    depth = 1 is the fully-online tail.  -> [K][s]."""
    w = np.asarray(windows, np.float64)
    K, W = w.shape
    if not (s >= 1 and depth >= 1 and depth * s <= W):
        raise ValueError("need 1 <= s and depth * s <= W")
    out = np.zeros((K, s))
    for k in range(K):
        terms = [w[k - i, W - (depth - i) * s: W - (depth - 1 - i) * s] for i in range(depth) if k - i >= 0]
        out[k] = np.mean(terms, axis=0)
    return out


def delayed_clean(noise, strain_seg, delay):
    """Aggregation latency (App. B, "Aggregation latency"): the newest
    `delay` predicted samples of each window are dropped as edge-degraded;
    the output is the s samples before them, noise[W - s - delay : W - delay],
    subtracted from the strain samples of the same span (the s strain samples
    that end `delay` samples before the newest one).  delay = 0 is
    causal_clean.  noise [B][W], strain_seg [B][s] -> (segment, clean)."""
    noise = np.asarray(noise, np.float64)
    s, W = strain_seg.shape[-1], noise.shape[-1]
    if not 0 <= delay <= W - s:
        raise ValueError("delay must be in [0, W - s]")
    seg = noise[..., W - s - delay: W - delay]
    return seg, np.asarray(strain_seg, np.float64) - seg


# ---------------------------------------------------------------------------
# BBHnet-shaped classifier
# ---------------------------------------------------------------------------

def unpack_bbhnet(params, stages=BBHNET_STAGES):
    p = np.asarray(params, np.float64)
    off = 0
    out = []

    def take(shape):
        nonlocal off
        n = int(np.prod(shape))
        a = p[off: off + n].reshape(shape)
        off += n
        return a

    for ci, co in stages:
        d = {}
        d["wa"], d["ba"] = take((co, ci, 7)), take((co,))
        d["wb"], d["bb"] = take((co, co, 7)), take((co,))
        d["ws"], d["bs"] = take((co, ci, 1)), take((co,))
        out.append(d)
    c_last = stages[-1][1]
    head = {"w": take((1, c_last)), "b": take((1,))}
    assert off == p.size
    return out, head


def bbhnet_forward(params, x, stages=BBHNET_STAGES):
    """Logits [B] for windows x [B][C][L].  Each stage:
    out = relu(conv_b(relu(conv_a(x))) + shortcut(x)) with conv_a k7 s2 p3,
    conv_b k7 s1 p3 and a 1x1 stride-2 projection shortcut; then global average
    pooling over time and a linear layer to one logit."""
    ps, head = unpack_bbhnet(params, stages)
    a = np.asarray(x, np.float64)
    for d in ps:
        h = np.maximum(conv1d(a, d["wa"], d["ba"], 2, 3), 0.0)
        h = conv1d(h, d["wb"], d["bb"], 1, 3)
        sc = conv1d(a, d["ws"], d["bs"], 2, 0)
        a = np.maximum(h + sc, 0.0)
    g = a.mean(axis=2)
    return g @ head["w"][0] + head["b"][0]


# ---------------------------------------------------------------------------
# Band-passed MSE loss
# ---------------------------------------------------------------------------

def band_bins(W, fs, f_lo, f_hi):
    """DFT bins k (0 <= k <= W/2) with f_lo <= k fs / W <= f_hi."""
    k = np.arange(W // 2 + 1)
    f = k * fs / W
    return k[(f >= f_lo) & (f <= f_hi)]


def bandpass(r, fs, f_lo, f_hi):
    """Exact projection of each row of r [B][W] onto the DFT bins in the band."""
    r = np.asarray(r, np.float64)
    W = r.shape[-1]
    R = np.fft.rfft(r, axis=-1)
    mask = np.zeros(R.shape[-1])
    mask[band_bins(W, fs, f_lo, f_hi)] = 1.0
    return np.fft.irfft(R * mask, n=W, axis=-1)


def bandpass_mse(strain, noise, fs=4096.0, f_lo=55.0, f_hi=65.0):
    """L = 1/(B W) sum_b ||P (strain_b - noise_b)||^2 and dL/dnoise = -2/(B W) P r."""
    r = np.asarray(strain, np.float64) - np.asarray(noise, np.float64)
    B, W = r.shape
    pr = bandpass(r, fs, f_lo, f_hi)
    return float(np.sum(pr * pr) / (B * W)), -2.0 / (B * W) * pr


def mse(strain, noise):
    """Plain MSE variant: L = 1/(B W) sum r^2, dL/dnoise = -2/(B W) r."""
    r = np.asarray(strain, np.float64) - np.asarray(noise, np.float64)
    B, W = r.shape
    return float(np.sum(r * r) / (B * W)), -2.0 / (B * W) * r


# ---------------------------------------------------------------------------
# End-to-end ensemble (main text, second offline workflow and its ensemble
# figure): one snapshotter for three sources, DeepClean per detector, the
# cleaned strain combined and resampled to BBHnet's rate, BBHnet logits.
# ---------------------------------------------------------------------------

def lowpass_taps(K, fc):
    """Windowed-sinc low-pass FIR (a reading of the ensemble's unspecified
    "postprocess" before resampling): h[j] = 2 fc sinc(2 fc (j - (K-1)/2))
    times a Hann window of length K, scaled to unit DC gain; fc in cycles per
    input sample."""
    j = np.arange(K, dtype=np.float64)
    c = j - (K - 1) / 2.0
    h = 2.0 * fc * np.sinc(2.0 * fc * c)
    w = 0.5 - 0.5 * np.cos(2.0 * np.pi * (j + 1) / (K + 1))
    h = h * w
    return h / h.sum()


def decimate2(x, taps):
    """Causal FIR then every second sample: y[m] = sum_j h[j] x[2m + 1 - j],
    with x zero before its first sample.  x [..., U] (U even) -> [..., U/2]."""
    x = np.asarray(x, np.float64)
    h = np.asarray(taps, np.float64)
    U = x.shape[-1]
    y = np.zeros(x.shape[:-1] + (U // 2,))
    for m in range(U // 2):
        for j in range(len(h)):
            v = 2 * m + 1 - j
            if v >= 0:
                y[..., m] += h[j] * x[..., v]
    return y


def ensemble_logits(dc_params, witness, strain, bbh_params, taps, s, W_dc, W_bb, K,
                    dc_layers=DEEPCLEAN_LAYERS, bbh_stages=BBHNET_STAGES):
    """K requests of one ensemble stream (stride s at the DeepClean rate).
    witness [2][C][U], strain [2][U] per detector (H1, L1), U = W_dc + K s;
    the detectors' snapshots start full (the first W_dc samples), request k
    adds samples [W_dc + k s, W_dc + (k+1) s).  Per request: each detector's
    DeepClean on its snapshot, fully-online clean block (causal_clean), the
    two cleaned streams decimated by 2 (decimate2 over everything cleaned so
    far), BBHnet on the snapshot of the decimated stream (W_bb samples, zero
    before its start).  Returns logits [K]."""
    cleaned = np.zeros((2, K * s))
    logits = np.zeros(K)
    for k in range(K):
        end = W_dc + (k + 1) * s
        for d in range(2):
            snap = snapshot_after(witness[d], end, W_dc)
            noise = deepclean_forward(dc_params[d], snap[None], dc_layers)
            _, cl = causal_clean(noise, strain[d][None, end - s:end])
            cleaned[d, k * s:(k + 1) * s] = cl[0]
        dec = decimate2(cleaned[:, :(k + 1) * s], taps)
        bsnap = snapshot_after(dec, dec.shape[-1], W_bb)
        logits[k] = bbhnet_forward(bbh_params, bsnap[None], bbh_stages)[0]
    return logits
