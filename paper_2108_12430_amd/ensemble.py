"""End-to-end ensemble on one GPU (main text, second offline workflow and its
ensemble figure): one snapshotter keeps the state of three sources per
stream -- the H1 witnesses, the L1 witnesses and BBHnet's input -- and each
request runs

  1. one batched snapshot_update of both detectors' witness rings;
  2. DeepClean-H1 and DeepClean-L1 on their snapshots, each writing its
     detector's fully-online cleaned strain block (App. B.2, B.4);
  3. the combine/postprocess step the paper leaves unspecified, read here as
     stacking the two cleaned channels and resampling them from 4096 Hz to
     BBHnet's 2048 Hz with a causal windowed-sinc low-pass FIR and
     decimation by 2 (gw_decimate2, per-stream filter history);
  4. a snapshot_update of the BBHnet ring with the s/2 new 2-channel samples,
     then BBHnet on that snapshot (one logit per stream).

All device work goes through the C ABI; this module allocates the buffers
once and issues the calls.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gwstream as gs


def lowpass_taps(ntaps=63, fc=0.225):
    """Low-pass FIR for the 2x decimation: sinc of cutoff fc (cycles per input
    sample) centred on the middle tap, times a Hann window of ntaps points
    (endpoints excluded), normalised to unit gain at DC."""
    k = np.arange(ntaps, dtype=np.float64)
    t = k - 0.5 * (ntaps - 1)
    h = np.where(t == 0, 2.0 * fc, np.sin(2.0 * np.pi * fc * t) / (np.pi * np.where(t == 0, 1.0, t)))
    h *= np.sin(np.pi * (k + 1) / (ntaps + 1)) ** 2
    return h / np.sum(h)


class Ensemble:
    """n ensemble streams with a common stride s (new samples per request at
    the DeepClean rate; s even).  dc_h1, dc_l1: DeepClean models of the two
    detectors (same input channels); bbh: a 2-channel BBHnet model."""

    def __init__(self, dc_h1, dc_l1, bbh, n, *, W_dc=32768, W_bb=2048, stride=256, taps=None,
                 precision=gs.BF16, device="cuda:0"):
        if stride % 2:
            raise ValueError("the stride must be even (decimation by 2)")
        self.dc = (dc_h1, dc_l1)
        self.bbh = bbh
        self.n, self.W_dc, self.W_bb, self.s = n, W_dc, W_bb, stride
        self.prec = precision
        self.dev = torch.device(device)
        self.C = dc_h1.c_in
        taps = lowpass_taps() if taps is None else np.asarray(taps, np.float64)
        self.taps = torch.from_numpy(taps.astype(np.float32)).to(self.dev)
        K = self.taps.numel()
        ring = lambda c, w: ((c * w * 4 + 255) // 256 + (c * w * 2 + 255) // 256) * 256
        self.pool = gs.Pool(2 * n * ring(self.C, W_dc) + n * ring(2, W_bb) + (8 << 20), max_slots=3 * n,
                            max_items=2 * n)
        self.slots_h1 = [self.pool.open(self.C, W_dc) for _ in range(n)]
        self.slots_l1 = [self.pool.open(self.C, W_dc) for _ in range(n)]
        self.slots_bb = [self.pool.open(2, W_bb) for _ in range(n)]
        s = stride
        self.wit_off = np.arange(2 * n, dtype=np.int64) * self.C * s
        self.bb_off = np.arange(n, dtype=np.int64) * 2 * (s // 2)
        self.cleaned = torch.empty((2, n, s), device=self.dev)
        self.hist = torch.zeros((n, 2, max(K - 1, 1)), device=self.dev)
        self.dec = torch.empty((n, 2, s // 2), device=self.dev)
        self.logits = torch.empty(n, device=self.dev)
        self.ws_dc = torch.empty(dc_h1.workspace_bytes(n, W_dc, precision), dtype=torch.uint8, device=self.dev)
        self.ws_bb = torch.empty(bbh.workspace_bytes(n, W_bb, precision), dtype=torch.uint8, device=self.dev)

    def prefill(self, witness):
        """Fill both detectors' witness rings with a full window: witness
        device [2][n][C][W_dc] float32."""
        W = self.W_dc
        self.pool.update(self.slots_h1 + self.slots_l1, [W] * (2 * self.n), witness.reshape(-1),
                         np.arange(2 * self.n, dtype=np.int64) * self.C * W)

    def step(self, witness, strain, stream=None):
        """One request of every stream.  witness device [2][n][C][s] (H1
        then L1), strain device [2][n][s] (the s newest strain samples of
        each detector).  Returns the logits tensor [n] (device; overwritten
        by the next step)."""
        n, s = self.n, self.s
        self.pool.update(self.slots_h1 + self.slots_l1, [s] * (2 * n), witness.reshape(-1), self.wit_off,
                         stream=stream)
        for d, slots in enumerate((self.slots_h1, self.slots_l1)):
            self.dc[d].forward(pool=self.pool, slots=slots, W=self.W_dc, strides=[s] * n, strain=strain[d],
                               clean=self.cleaned[d], precision=self.prec, ws=self.ws_dc, stream=stream)
        gs.decimate2(x=self.cleaned, taps=self.taps, hist=self.hist, y=self.dec, stream=stream)
        self.pool.update(self.slots_bb, [s // 2] * n, self.dec.reshape(-1), self.bb_off, stream=stream)
        self.bbh.forward(pool=self.pool, slots=self.slots_bb, W=self.W_bb, logits=self.logits, precision=self.prec,
                         ws=self.ws_bb, stream=stream)
        return self.logits
