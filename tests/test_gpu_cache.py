"""GPU tests of the incremental DeepClean forward over per-stream activation
caches (deepclean_forward_cached): an incrementally updated cache gives the
bitwise same noise window and clean output as recomputing every position,
over the zero-filled start, the ring's wrap and long runs; the outputs match
the FP64 oracle within the BF16 bound; streams are independent of the rest
of the batch; strides that are not multiples of 16, skipped calls,
reattached caches and caches computed by another model or before a refresh
fall back to a full recompute; bad calls are refused."""
import numpy as np
import pytest
import torch

from oracle import ref
from paper_2108_12430_amd import gwstream as gs
from paper_2108_12430_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
LAYERS = synth.deepclean_layers()


def rel(a, r):
    return float(np.max(np.abs(np.asarray(a, np.float64) - r)) / np.max(np.abs(r)))


@pytest.fixture(scope="module")
def model():
    return gs.DeepClean(torch.from_numpy(synth.deepclean_params(0)).to(DEV), LAYERS)


class Streams:
    """n streams of one window length, each in its own slot with its own
    cache, fed from one seeded witness/strain stream per stream."""

    def __init__(self, m, W, n, seed, total):
        self.m, self.W, self.n = m, W, n
        self.pool = gs.Pool(n * (21 * W * 6 + (1 << 16)) + (4 << 20), max_slots=n, max_items=max(n, 4))
        self.slots = [self.pool.open(21, W) for _ in range(n)]
        self.caches = [m.new_cache(W) for _ in range(n)]
        for sl, c in zip(self.slots, self.caches):
            self.pool.attach_cache(sl, c)
        self.wit, self.strain = [], []
        for i in range(n):
            w, s = synth.witness_stream(seed + i, total)
            self.wit.append(w)
            self.strain.append(s)
        self.pos = [0] * n

    def update(self, idx, s):
        """Feed the next s (or s[k] for stream idx[k]) samples of the streams
        idx (one call)."""
        ss = [s] * len(idx) if np.isscalar(s) else list(s)
        blocks = [self.wit[i][:, self.pos[i]:self.pos[i] + n].reshape(-1) for i, n in zip(idx, ss)]
        offs = np.cumsum([0] + [b.size for b in blocks[:-1]])
        self.pool.update([self.slots[i] for i in idx], ss, torch.from_numpy(np.concatenate(blocks)).to(DEV), offs)
        for i, n in zip(idx, ss):
            self.pos[i] += n

    def forward(self, idx, s, full=False, delays=None):
        """One cached call over the streams idx with clean strides s (scalar
        or per stream); returns noise [len][W], packed clean and strain."""
        ss = [s] * len(idx) if np.isscalar(s) else list(s)
        dl = [0] * len(idx) if delays is None else list(delays)
        strain = np.concatenate([self.strain[i][self.pos[i] - n - d:self.pos[i] - d]
                                 for i, n, d in zip(idx, ss, dl)]).astype(np.float32)
        noise = torch.empty((len(idx), self.W), device=DEV)
        clean = torch.empty(int(sum(ss)), device=DEV)
        self.m.forward_cached(pool=self.pool, slots=[self.slots[i] for i in idx], W=self.W, strides=ss,
                              strain=torch.from_numpy(strain).to(DEV), noise=noise, clean=clean, delays=delays,
                              full=full)
        torch.cuda.synchronize()
        return noise.cpu().numpy(), clean.cpu().numpy(), strain

    def window(self, i):
        return ref.snapshot_after(self.wit[i], self.pos[i], self.W)


@pytest.mark.parametrize("W,s,steps", [(4096, 256, 40), (32768, 256, 24), (2048, 1024, 12)])
def test_incremental_equals_full_recompute_bitwise(model, W, s, steps):
    """Stream 0 is updated incrementally, stream 1 (the same samples) is
    recomputed in full every time: identical noise windows and clean
    outputs, from the zero-filled start through the ring's wrap."""
    st = Streams(model, W, 2, 40, W + (steps + 2) * s)
    st.wit[1], st.strain[1] = st.wit[0], st.strain[0]
    for k in range(steps):
        st.update([0, 1], s)
        na, ca, _ = st.forward([0], s)
        nb, cb, _ = st.forward([1], s, full=True)
        assert np.array_equal(na, nb), k
        assert np.array_equal(ca, cb), k


def test_cached_matches_oracle(model):
    W, s = 32768, 256
    st = Streams(model, W, 3, 50, W + 200 * s)
    params = synth.deepclean_params(0)
    checks = {1, 2, 60, 129, 130, 131, 190}
    for k in range(1, 191):
        st.update([0, 1, 2], s)
        dl = [0, 0, 3072]
        noise, clean, strain = st.forward([0, 1, 2], s, delays=dl)
        if k in checks:
            for i in range(3):
                x = st.window(i)[None]
                en = ref.deepclean_forward(params, x)[0]
                assert rel(noise[i], en) <= 2e-2, (k, i, rel(noise[i], en))
                ec = strain[i * s:(i + 1) * s] - en[W - s - dl[i]:W - dl[i]]
                assert np.max(np.abs(clean[i * s:(i + 1) * s] - ec)) <= 2e-2 * np.max(np.abs(en)), (k, i)


def test_streams_independent_of_batch_and_fallbacks(model):
    """Six streams with strides 256/512/1024 in one call equal the same
    streams run alone; a stride that is not a multiple of 16, a skipped call
    (two updates, one forward) and a reattached cache all give the
    full-recompute result."""
    W = 4096
    mix = Streams(model, W, 6, 60, W + 40 * 1024)
    alone = Streams(model, W, 6, 60, W + 40 * 1024)
    strides = [256, 512, 1024, 256, 512, 1024]
    offs = np.cumsum([0] + strides[:-1])
    for k in range(10):
        mix.update(list(range(6)), strides)
        for i in range(6):
            alone.update([i], strides[i])
        # the whole mix in one call (three shift classes)
        nm, cm, _ = mix.forward(list(range(6)), strides)
        for i in range(6):
            na, ca, _ = alone.forward([i], strides[i], full=(k % 3 == 2))
            assert np.array_equal(nm[i], na[0]), (k, i)
            assert np.array_equal(cm[offs[i]:offs[i] + strides[i]], ca), (k, i)
    # fallbacks: stride 8 (not a multiple of 16), a skipped forward, a reattached cache
    for s, skip, reattach in ((8, False, False), (256, True, False), (256, False, True), (512, False, False)):
        mix.update([0], s)
        alone.update([0], s)
        if skip:
            mix.update([0], s)
            alone.update([0], s)
        if reattach:
            mix.pool.attach_cache(mix.slots[0], mix.caches[0])
        n1, c1, _ = mix.forward([0], s)
        n2, c2, _ = alone.forward([0], s, full=True)
        assert np.array_equal(n1, n2) and np.array_equal(c1, c2), (s, skip, reattach)


def test_refresh_recomputes_caches():
    """After gw_model_refresh with changed weights, caches computed with the
    old weights are recomputed in full: the next call, an ordinary
    incremental step, equals a GW_CACHE_FULL call on the same samples
    bitwise and matches the oracle at the new weights."""
    p0 = synth.deepclean_params(0)
    params = torch.from_numpy(p0.copy()).to(DEV)
    m = gs.DeepClean(params, LAYERS)
    W, s = 4096, 256
    st = Streams(m, W, 2, 70, W + 12 * s)
    st.wit[1], st.strain[1] = st.wit[0], st.strain[0]
    for _ in range(4):
        st.update([0, 1], s)
        st.forward([0], s)
        st.forward([1], s, full=True)
    rng = np.random.default_rng(9)
    p1 = (p0 * np.exp(0.2 * rng.standard_normal(p0.shape))).astype(np.float32)
    params.copy_(torch.from_numpy(p1))
    m.refresh()
    st.update([0, 1], s)
    na, ca, _ = st.forward([0], s)
    nb, cb, _ = st.forward([1], s, full=True)
    assert np.array_equal(na, nb)
    assert np.array_equal(ca, cb)
    exp = ref.deepclean_forward(p1, st.window(0)[None], LAYERS)[0]
    assert rel(na[0], exp) <= 2e-2


def test_cache_from_another_model_recomputed():
    """A cache computed by one model and then used by another (here one made
    after the first was freed, with other weights) is recomputed in full:
    the incremental call equals a GW_CACHE_FULL call bitwise and matches the
    oracle at the second model's weights."""
    p0 = synth.deepclean_params(0)
    m0 = gs.DeepClean(torch.from_numpy(p0.copy()).to(DEV), LAYERS)
    W, s = 4096, 256
    st = Streams(m0, W, 2, 71, W + 12 * s)
    st.wit[1], st.strain[1] = st.wit[0], st.strain[0]
    for _ in range(4):
        st.update([0, 1], s)
        st.forward([0], s)
        st.forward([1], s, full=True)
    torch.cuda.synchronize()
    st.m = None
    del m0
    rng = np.random.default_rng(10)
    p1 = (p0 * np.exp(0.2 * rng.standard_normal(p0.shape))).astype(np.float32)
    st.m = gs.DeepClean(torch.from_numpy(p1).to(DEV), LAYERS)
    st.update([0, 1], s)
    na, ca, _ = st.forward([0], s)
    nb, cb, _ = st.forward([1], s, full=True)
    assert np.array_equal(na, nb)
    assert np.array_equal(ca, cb)
    exp = ref.deepclean_forward(p1, st.window(0)[None], LAYERS)[0]
    assert rel(na[0], exp) <= 2e-2


def test_cached_rejects_bad_calls(model):
    W = 4096
    pool = gs.Pool(8 << 20, max_slots=2, max_items=4)
    sl = pool.open(21, W)
    noise = torch.empty((1, W), device=DEV)
    with pytest.raises(gs.GwError):  # no cache attached
        model.forward_cached(pool=pool, slots=[sl], W=W, noise=noise)
    small = torch.empty(model.cache_bytes(W) - 256, dtype=torch.uint8, device=DEV)
    pool.attach_cache(sl, small)
    with pytest.raises(gs.GwError):  # too small
        model.forward_cached(pool=pool, slots=[sl], W=W, noise=noise)
    pool.attach_cache(sl, model.new_cache(W))
    with pytest.raises(gs.GwError):  # window mismatch
        model.forward_cached(pool=pool, slots=[sl], W=2048, noise=noise)
    with pytest.raises(gs.GwError):  # duplicate slot
        model.forward_cached(pool=pool, slots=[sl, sl], W=W, noise=torch.empty((2, W), device=DEV))
