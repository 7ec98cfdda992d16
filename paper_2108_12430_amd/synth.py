"""Seeded synthetic inputs: network parameters, witness/strain streams, BBH windows.

This module only draws random numbers and shapes them into the inputs the
streaming networks consume.  It contains none of the networks' arithmetic
(no convolution, normalisation, activation, ring update or loss), so both the
device path and the FP64 checker can take their inputs from here without
sharing any of the method's code.

Workload shapes follow the paper's deployment: 21 witness channels of the
power-mains lines and their harmonics (main text, DeepClean paragraph),
f_s = 4096 Hz after resampling (App. B.5), 8-s online windows (App. B.3) and
1/16-s front-end chunks (App. B.4).  The LIGO data themselves are not
available; coloured Gaussian noise with 60/120 Hz lines stands in for them.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# Parameter tables (shapes only).  A DeepClean layer is
#   (type, C_in, C_out, k, stride, pad, out_pad, bn_tanh)
# with type "conv" (weight [C_out][C_in][k]) or "convT" (weight [C_in][C_out][k]).
# ---------------------------------------------------------------------------

def deepclean_layers(c_in: int = 21):
    """Layer list of the DeepClean-shaped autoencoder used throughout."""
    enc = [8, 16, 32, 64]
    dec = [32, 16, 8, 8]
    layers = []
    c = c_in
    for co in enc:
        layers.append(("conv", c, co, 7, 2, 3, 0, True))
        c = co
    for co in dec:
        layers.append(("convT", c, co, 7, 2, 3, 1, True))
        c = co
    layers.append(("conv", c, 1, 7, 1, 3, 0, False))
    return layers


def tiny_layers():
    """Two-layer, four-channel instance used for finite-difference checks:
    Conv1d 4->4 (k7 s2 p3) + BN + tanh, then ConvTranspose1d 4->1 (k7 s2 p3 op1)."""
    return [("conv", 4, 4, 7, 2, 3, 0, True), ("convT", 4, 1, 7, 2, 3, 1, False)]


def bbhnet_stages(c_in: int = 2):
    """(C_in, C_out) of each residual stage of the BBHnet-shaped classifier."""
    chans = [32, 64, 128]
    out = []
    c = c_in
    for co in chans:
        out.append((c, co))
        c = co
    return out


def _uniform(rng, a, shape):
    return rng.uniform(-a, a, size=shape)


def deepclean_params(seed: int = 0, layers=None) -> np.ndarray:
    """Flat float32 parameter vector.

    Order per layer: weight, bias, then (if BN) gamma, beta, running mean,
    running variance.  Weights/biases ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)) with
    fan_in = C_in*k for conv and C_out*k for convT (PyTorch's convention);
    gamma ~ U(0.5, 1.5), beta ~ N(0, 0.1), mean ~ N(0, 0.1), var ~ U(0.5, 1.5)
    so that the normalisation is far from the identity.
    """
    layers = deepclean_layers() if layers is None else layers
    rng = np.random.default_rng(seed)
    parts = []
    for (typ, ci, co, k, _s, _p, _op, bn) in layers:
        fan_in = (ci if typ == "conv" else co) * k
        a = 1.0 / np.sqrt(fan_in)
        wshape = (co, ci, k) if typ == "conv" else (ci, co, k)
        parts.append(_uniform(rng, a, wshape).ravel())
        parts.append(_uniform(rng, a, (co,)))
        if bn:
            parts.append(rng.uniform(0.5, 1.5, size=co))
            parts.append(rng.normal(0.0, 0.1, size=co))
            parts.append(rng.normal(0.0, 0.1, size=co))
            parts.append(rng.uniform(0.5, 1.5, size=co))
    return np.concatenate(parts).astype(np.float32)


def bbhnet_params(seed: int = 0, c_in: int = 2) -> np.ndarray:
    """Flat float32 parameters: per stage conv_a (w, b), conv_b (w, b),
    shortcut 1x1 (w, b); then head Linear(C_last -> 1) (w, b).
    All ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in))."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in bbhnet_stages(c_in):
        for (cin, k) in ((ci, 7), (co, 7), (ci, 1)):
            a = 1.0 / np.sqrt(cin * k)
            parts.append(_uniform(rng, a, (co, cin, k)).ravel())
            parts.append(_uniform(rng, a, (co,)))
    c_last = bbhnet_stages(c_in)[-1][1]
    a = 1.0 / np.sqrt(c_last)
    parts.append(_uniform(rng, a, (1, c_last)).ravel())
    parts.append(_uniform(rng, a, (1,)))
    return np.concatenate(parts).astype(np.float32)


# ---------------------------------------------------------------------------
# Time series
# ---------------------------------------------------------------------------

def coloured_noise(rng, n_ch: int, n: int, fs: float) -> np.ndarray:
    """Gaussian noise with amplitude spectral density 1 + (10 Hz / max(f, 1 Hz))^2
    (a 1/f^2 rise below 10 Hz on a white floor), unit variance per channel."""
    white = rng.standard_normal((n_ch, n))
    spec = np.fft.rfft(white, axis=-1)
    f = np.fft.rfftfreq(n, d=1.0 / fs)
    asd = 1.0 + (10.0 / np.maximum(f, 1.0)) ** 2
    x = np.fft.irfft(spec * asd, n=n, axis=-1)
    x -= x.mean(axis=-1, keepdims=True)
    x /= x.std(axis=-1, keepdims=True)
    return x


def witness_stream(seed: int, n: int, c: int = 21, fs: float = 4096.0, n_line: int = 4):
    """Witness channels [c][n] and target strain [n] (float32).

    Witnesses 0..n_line-1 carry 60 and 120 Hz mains lines with random amplitude
    and phase plus a slow amplitude modulation (sidebands); the strain is its
    own coloured noise plus a seeded linear combination of those lines, so a
    network could learn to predict and subtract it.
    """
    rng = np.random.default_rng(seed)
    w = coloured_noise(rng, c, n, fs)
    s = coloured_noise(rng, 1, n, fs)[0]
    t = np.arange(n) / fs
    for ch in range(min(n_line, c)):
        line = np.zeros(n)
        for f0 in (60.0, 120.0):
            amp = rng.uniform(0.5, 2.0)
            ph = rng.uniform(0, 2 * np.pi)
            fm = rng.uniform(0.05, 0.5)
            am = 1.0 + 0.2 * np.sin(2 * np.pi * fm * t + rng.uniform(0, 2 * np.pi))
            line += amp * am * np.sin(2 * np.pi * f0 * t + ph)
        w[ch] += line
        s += rng.normal(0.0, 0.5) * line
    return w.astype(np.float32), s.astype(np.float32)


GM_SUN_S = 4.925491e-6  # G * M_sun / c^3 in seconds


def _chirp(fs: float, n: int, mc_sun: float, tc: float, phi0: float) -> np.ndarray:
    """Leading-order (Newtonian quadrupole) inspiral, zero after coalescence.
    f(tau) = (1/pi) (5/256)^(3/8) Mc^(-5/8) tau^(-3/8),
    phi(tau) = phi0 - 2 (5 Mc)^(-5/8) tau^(5/8), h ~ f^(2/3) cos(phi),
    starting at 20 Hz and cut at the ISCO of total mass 2^(6/5) Mc, with a
    10-ms cosine taper at both ends."""
    mc = mc_sun * GM_SUN_S
    t = np.arange(n) / fs
    tau = tc - t
    h = np.zeros(n)
    ok = tau > 0
    tau_ok = tau[ok]
    f = (1 / np.pi) * (5.0 / 256.0) ** 0.375 * mc ** -0.625 * tau_ok ** -0.375
    phi = phi0 - 2.0 * (5.0 * mc) ** -0.625 * tau_ok ** 0.625
    m_tot = 2 ** 1.2 * mc
    f_isco = 1.0 / (6 ** 1.5 * np.pi * m_tot)
    keep = (f >= 20.0) & (f <= f_isco)
    hh = np.where(keep, f ** (2.0 / 3.0) * np.cos(phi), 0.0)
    h[ok] = hh
    idx = np.nonzero(h)[0]
    if idx.size:
        nt = max(1, int(0.01 * fs))
        lo, hi = idx[0], idx[-1]
        ramp = 0.5 * (1 - np.cos(np.pi * np.arange(nt) / nt))
        seg = min(nt, hi - lo + 1)
        h[lo:lo + seg] *= ramp[:seg]
        h[hi - seg + 1:hi + 1] *= ramp[:seg][::-1]
    return h


def bbh_windows(seed: int, batch: int, n: int = 2048, fs: float = 2048.0, n_det: int = 2):
    """Whitened two-detector windows [batch][n_det][n] (float32) and labels.

    Half of the windows (chosen at random) carry an injected chirp with chirp
    mass ~ U(10, 40) Msun and network SNR ~ U(6, 20), split equally over the
    detectors, coalescence time ~ U(0.5, 0.95) of the window and an
    inter-detector shift ~ U(-10, 10) ms.  SNR is sqrt(sum h^2) in unit-variance
    white noise."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((batch, n_det, n))
    labels = np.zeros(batch, dtype=np.int32)
    inj = rng.permutation(batch)[: batch // 2]
    for b in inj:
        labels[b] = 1
        mc = rng.uniform(10.0, 40.0)
        snr = rng.uniform(6.0, 20.0)
        tc = rng.uniform(0.5, 0.95) * n / fs
        phi0 = rng.uniform(0, 2 * np.pi)
        for d in range(n_det):
            shift = rng.uniform(-0.01, 0.01) if d else 0.0
            h = _chirp(fs, n, mc, tc + shift, phi0)
            nrm = np.sqrt(np.sum(h * h))
            if nrm > 0:
                x[b, d] += h * (snr / np.sqrt(n_det)) / nrm
    return x.astype(np.float32), labels


def gaussian(seed: int, shape, scale: float = 1.0) -> np.ndarray:
    """i.i.d. N(0, scale^2) float32 array (generic test input)."""
    return (np.random.default_rng(seed).standard_normal(shape) * scale).astype(np.float32)
