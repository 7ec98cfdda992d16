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
                 precision=gs.BF16, device="cuda:0", pipeline=False):
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
        # pipeline: request k's decimation and BBHnet run on a second stream
        # while the DeepClean forwards of request k + 1 run on the caller's;
        # the cleaned-strain and logit buffers alternate between two copies
        self.pipeline = pipeline
        nbuf = 2 if pipeline else 1
        self.cleaned_bufs = [torch.empty((2, n, s), device=self.dev) for _ in range(nbuf)]
        self.logit_bufs = [torch.empty(n, device=self.dev) for _ in range(nbuf)]
        self.hist = torch.zeros((n, 2, max(K - 1, 1)), device=self.dev)
        self.dec = torch.empty((n, 2, s // 2), device=self.dev)
        self.k = 0
        if pipeline:
            self.s_post = torch.cuda.Stream(device=self.dev)
            self.ev_clean = [torch.cuda.Event() for _ in range(2)]
            self.ev_post = [torch.cuda.Event() for _ in range(2)]
            for e in self.ev_post:
                e.record(torch.cuda.current_stream(self.dev))
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
        two steps later, or by the next step without the pipeline).  With the
        pipeline the logits are written on the ensemble's second stream: wait
        for ready_event() (or synchronise) before reading them."""
        n, s = self.n, self.s
        main = stream if stream is not None else torch.cuda.current_stream(self.dev)
        b = self.k % len(self.cleaned_bufs)
        cleaned, logits = self.cleaned_bufs[b], self.logit_bufs[b]
        if self.pipeline:
            main.wait_event(self.ev_post[b])  # the decimation that read this buffer is done
        # per detector: the witness update and the DeepClean forward in one
        # call (one launch on the fused BF16 path)
        wit = witness.reshape(-1)
        for d, slots in enumerate((self.slots_h1, self.slots_l1)):
            self.dc[d].update_forward(pool=self.pool, slots=slots, strides=[s] * n, samples=wit,
                                      offsets=self.wit_off[d * n:(d + 1) * n], W=self.W_dc, strain=strain[d],
                                      clean=cleaned[d], precision=self.prec, ws=self.ws_dc, stream=main)
        post = main
        if self.pipeline:
            self.ev_clean[b].record(main)
            post = self.s_post
            post.wait_event(self.ev_clean[b])
        gs.decimate2(x=cleaned, taps=self.taps, hist=self.hist, y=self.dec, stream=post)
        self.pool.update(self.slots_bb, [s // 2] * n, self.dec.reshape(-1), self.bb_off, stream=post)
        self.bbh.forward(pool=self.pool, slots=self.slots_bb, W=self.W_bb, logits=logits, precision=self.prec,
                         ws=self.ws_bb, stream=post)
        if self.pipeline:
            self.ev_post[b].record(post)
        self.k += 1
        return logits

    def ready_event(self):
        """With the pipeline: an event recorded after the last step's logits
        (None without the pipeline: they are ready in stream order)."""
        return self.ev_post[(self.k - 1) % 2] if self.pipeline and self.k else None
