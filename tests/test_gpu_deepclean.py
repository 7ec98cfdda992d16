"""GPU parity of the DeepClean path and the snapshot rings against the FP64
oracle, through the C ABI.

Error metric per output tensor: max-abs error over max-abs reference
(normwise; element-wise relative error is ill-posed near zero crossings).
FP32 path bound: 1e-5.
"""
import numpy as np
import pytest
import torch

from oracle import ref
from paper_2108_12430_amd import gwstream as gs
from paper_2108_12430_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
FP32_TOL = 1e-5


def rel(a, r):
    a = np.asarray(a, np.float64)
    r = np.asarray(r, np.float64)
    return float(np.max(np.abs(a - r)) / np.max(np.abs(r)))


@pytest.fixture(scope="module")
def dc():
    layers = synth.deepclean_layers()
    params = synth.deepclean_params(0)
    p = torch.from_numpy(params).to(DEV)
    m = gs.DeepClean(p, layers)
    return m, params, layers


def run_dense(m, x, precision=gs.FP32):
    xt = torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(DEV)
    noise = torch.empty((x.shape[0], x.shape[-1]), dtype=torch.float32, device=DEV)
    m.forward(x=xt, noise=noise, precision=precision)
    torch.cuda.synchronize()
    return noise.cpu().numpy()


def test_forward_1s_window_fp32(dc):
    """21 witness channels x 4096 samples (1 s at 4096 Hz), batch 1."""
    m, params, layers = dc
    w, _ = synth.witness_stream(1, 4096)
    x = w[None]
    got = run_dense(m, x)
    exp = ref.deepclean_forward(params, x, layers)
    assert rel(got, exp) <= FP32_TOL


@pytest.mark.parametrize("n,W", [(3, 4096), (2, 16 * 67), (1, 16), (5, 2048)])
def test_forward_shapes_fp32(dc, n, W):
    """Several time tiles plus ragged tails (W not a multiple of the 256-lane
    block), the shortest legal window, and a batch."""
    m, params, layers = dc
    x = synth.gaussian(100 + W, (n, 21, W))
    got = run_dense(m, x)
    exp = ref.deepclean_forward(params, x, layers)
    assert rel(got, exp) <= FP32_TOL


def test_forward_8s_window_sampled(dc):
    """Full 8-s window (21 x 32768) at the batch the streaming bench uses per
    launch; every output checked."""
    m, params, layers = dc
    w, _ = synth.witness_stream(2, 2 * 32768)
    x = np.stack([w[:, :32768], w[:, 32768:]])
    got = run_dense(m, x)
    exp = ref.deepclean_forward(params, x, layers)
    assert rel(got, exp) <= FP32_TOL


def test_batch_independence_bitwise(dc):
    """Each window's output does not depend on what else is in the batch."""
    m, _, _ = dc
    x = synth.gaussian(7, (6, 21, 4096))
    full = run_dense(m, x)
    for i in (0, 3, 5):
        one = run_dense(m, x[i:i + 1])
        assert np.array_equal(one[0], full[i])


def test_invalid_calls(dc):
    m, _, _ = dc
    x = torch.zeros((1, 21, 4008), device=DEV)   # 4008 is not a multiple of 16
    with pytest.raises(gs.GwError) as e:
        m.forward(x=x, noise=torch.empty((1, 4008), device=DEV), ws=torch.empty(1 << 20, dtype=torch.uint8,
                                                                                   device=DEV))
    assert e.value.code == gs.GW_EINVAL
    x = torch.zeros((1, 21, 4096), device=DEV)
    with pytest.raises(gs.GwError) as e:
        m.forward(x=x, noise=torch.empty((1, 4096), device=DEV), ws=torch.empty(256, dtype=torch.uint8,
                                                                                   device=DEV))
    assert e.value.code == gs.GW_EINVAL   # workspace too small


# --------------------------------------------------------------------------- snapshot rings

def bf16_rne_bits(x):
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r & 0xFFFF).astype(np.uint16)


def test_snapshot_ring_matches_closed_form():
    """After every request the snapshot equals the last W samples of the
    stream so far (zero before the start), bitwise; the BF16 shadow equals the
    round-to-nearest-even conversion."""
    rng = np.random.default_rng(21)
    C_, W = 3, 96
    stream = synth.gaussian(22, (C_, 3000))
    pool = gs.Pool(1 << 22, max_slots=4, max_items=4)
    slot = pool.open(C_, W)
    pos = 0
    for it in range(60):
        s = int(rng.integers(1, W + 1)) if it % 5 else [1, W, 4, 8, 17][it // 5 % 5]
        s = min(s, 3000 - pos)
        if s == 0:
            break
        blk = torch.from_numpy(np.ascontiguousarray(stream[:, pos:pos + s])).to(DEV).reshape(-1)
        pool.update([slot], [s], blk, [0])
        pos += s
        win = pool.window(slot).cpu().numpy()
        assert np.array_equal(win, ref.snapshot_after(stream, pos, W).astype(np.float32))
        sh = pool.window(slot, bf16=True).cpu().numpy().view(np.uint16)
        assert np.array_equal(sh, bf16_rne_bits(win))
    assert pool.info(slot) == (C_, W, pos)


def test_snapshot_batched_many_streams():
    """One batched call updates many streams of different C, W and s."""
    rng = np.random.default_rng(5)
    specs = [(21, 4096), (2, 2048), (5, 100), (1, 64), (21, 512)]
    pool = gs.Pool(1 << 26, max_slots=16, max_items=16)
    slots = [pool.open(c, w) for c, w in specs]
    streams = [synth.gaussian(30 + i, (c, 5000)) for i, (c, w) in enumerate(specs)]
    pos = [0] * len(specs)
    for _ in range(12):
        strides = [int(rng.integers(1, min(w, 600) + 1)) for c, w in specs]
        blocks, offs, o = [], [], 0
        for i, ((c, w), s) in enumerate(zip(specs, strides)):
            blocks.append(streams[i][:, pos[i]:pos[i] + s].reshape(-1))
            offs.append(o)
            o += c * s
        samples = torch.from_numpy(np.concatenate(blocks).astype(np.float32)).to(DEV)
        pool.update(slots, strides, samples, offs)
        for i, s in enumerate(strides):
            pos[i] += s
    for i, (c, w) in enumerate(specs):
        assert np.array_equal(pool.window(slots[i]).cpu().numpy(),
                              ref.snapshot_after(streams[i], pos[i], w).astype(np.float32))


def test_pool_admission_and_errors():
    C_, W = 21, 4096
    per = 21 * 4096 * 6
    pool = gs.Pool(2 * per + (1 << 16), max_slots=8, max_items=8)
    a = pool.open(C_, W)
    b = pool.open(C_, W)
    assert pool.try_open(C_, W) is None                      # arena full -> GW_ENOMEM
    with pytest.raises(gs.GwError) as e:
        pool.open(C_, W)
    assert e.value.code == gs.GW_ENOMEM
    blk = torch.zeros(21 * 8, device=DEV)
    with pytest.raises(gs.GwError) as e:                     # duplicate slot in one call
        pool.update([a, a], [8, 8], torch.zeros(2 * 21 * 8, device=DEV), [0, 21 * 8])
    assert e.value.code == gs.GW_EINVAL
    with pytest.raises(gs.GwError) as e:                     # stride > W
        pool.update([a], [W + 1], torch.zeros(21 * (W + 1), device=DEV), [0])
    assert e.value.code == gs.GW_EINVAL
    assert pool.info(a)[2] == 0                              # rejected calls changed nothing
    pool.close(b)
    with pytest.raises(gs.GwError) as e:                     # closed slot
        pool.update([b], [8], blk, [0])
    assert e.value.code == gs.GW_ESTATE
    c = pool.try_open(C_, W)                                 # freed memory is reused
    assert c is not None
    assert np.all(pool.window(c).cpu().numpy() == 0)         # and starts from zeros


def test_stream_restore_continues_bitwise(dc):
    """A stream exported with gw_stream_window / gw_stream_info and restored
    into another slot with gw_stream_load continues bitwise like the source:
    the same window, BF16 shadow and count, then the same forward outputs
    (FP32 and BF16) after further updates applied to both.  The source's
    head is unaligned (odd strides) and the restored head is 0, so the ring
    reads of the two slots take different paths."""
    m, _, _ = dc
    C_, W = 21, 4096
    stream = synth.gaussian(41, (C_, 9000))
    strain = synth.gaussian(42, (1, 9000))[0]
    pool = gs.Pool(1 << 26, max_slots=4, max_items=4)
    a = pool.open(C_, W)
    pos = 0
    for s in [300, 37, 512, 1000, 64, 129, 2048]:
        pool.update([a], [s], torch.from_numpy(np.ascontiguousarray(stream[:, pos:pos + s])).to(DEV).reshape(-1), [0])
        pos += s
    win = pool.window(a)
    n_seen = pool.info(a)[2]
    b = pool.open(C_, W)
    pool.load(b, win, n_seen)
    assert pool.info(b) == pool.info(a)
    assert torch.equal(pool.window(b), win)
    assert torch.equal(pool.window(b, bf16=True), pool.window(a, bf16=True))
    for s in [256, 77, 1024]:
        blk = np.ascontiguousarray(stream[:, pos:pos + s]).reshape(-1)
        pool.update([a, b], [s, s], torch.from_numpy(np.concatenate([blk, blk])).to(DEV), [0, C_ * s])
        st = torch.from_numpy(np.tile(strain[pos:pos + s], 2).astype(np.float32)).to(DEV)
        pos += s
        for prec in (gs.FP32, gs.BF16):
            noise = torch.empty((2, W), device=DEV)
            clean = torch.empty(2 * s, device=DEV)
            m.forward(pool=pool, slots=[a, b], W=W, strides=[s, s], strain=st, noise=noise, clean=clean,
                      precision=prec)
            torch.cuda.synchronize()
            assert torch.equal(noise[0], noise[1]), (s, prec)
            assert torch.equal(clean[:s], clean[s:]), (s, prec)
    assert torch.equal(pool.window(a), pool.window(b))
    with pytest.raises(ValueError):                          # shape checked by the binding
        pool.load(b, win[:, :100].contiguous(), 0)
    with pytest.raises(gs.GwError) as e:                     # negative count
        pool.load(b, win, -1)
    assert e.value.code == gs.GW_EINVAL


def test_refresh_rederives_every_inference_path():
    """After the parameters change in place (as an optimizer step changes
    them) and gw_model_refresh, every inference path (FP32, BF16 fused and
    per layer, FP16 fused) computes with the new parameters: each matches
    the oracle at the new parameters within its bound, while the change is
    large enough that the old outputs are far outside it."""
    layers = synth.deepclean_layers()
    p0 = synth.deepclean_params(0)
    params = torch.from_numpy(p0.copy()).to(DEV)
    m = gs.DeepClean(params, layers)
    wit, _ = synth.witness_stream(12, 2 * 4096)
    x = np.ascontiguousarray(wit.reshape(21, 2, 4096).transpose(1, 0, 2))
    old = run_dense(m, x, gs.BF16)
    rng = np.random.default_rng(10)
    p1 = (p0 * np.exp(0.2 * rng.standard_normal(p0.shape))).astype(np.float32)  # signs kept, variances > 0
    params.copy_(torch.from_numpy(p1))
    m.refresh()
    torch.cuda.synchronize()
    exp = ref.deepclean_forward(p1, x, layers)
    assert rel(old, exp) > 5e-2
    assert rel(run_dense(m, x, gs.FP32), exp) <= FP32_TOL
    assert rel(run_dense(m, x, gs.BF16), exp) <= 2e-2
    assert rel(run_dense(m, x, gs.FP16), exp) <= 2.5e-3
    xt = torch.from_numpy(x).to(DEV)
    noise = torch.empty((2, 4096), device=DEV)
    m.forward(x=xt, noise=noise, precision=gs.BF16, flags=gs.LAYERWISE)
    torch.cuda.synchronize()
    assert rel(noise.cpu().numpy(), exp) <= 2e-2


# --------------------------------------------------------------------------- streaming

def test_streaming_8s_window_fp32(dc):
    """21 x 32768 snapshot advanced by 256-sample strides for 4096 updates.
    Every streamed output is bitwise equal to the GPU offline forward of the
    same window; the oracle checks the zero-fill transition, a sample of later
    updates and the last one; the cleaned strain is strain minus the newest
    256 predicted samples."""
    m, params, layers = dc
    W, s, N = 32768, 256, 4096
    wit, strain = synth.witness_stream(2, N * s)
    wit_t = torch.from_numpy(wit).to(DEV)
    strain_t = torch.from_numpy(strain).to(DEV)
    pool = gs.Pool(64 << 20, max_slots=2, max_items=2)
    slot = pool.open(21, W)
    ws = torch.empty(m.workspace_bytes(1, W), dtype=torch.uint8, device=DEV)
    noise_all = torch.empty((N, W), dtype=torch.float32, device=DEV)
    clean_all = torch.empty((N, s), dtype=torch.float32, device=DEV)
    for u in range(N):
        blk = wit_t[:, u * s:(u + 1) * s].contiguous().reshape(-1)
        pool.update([slot], [s], blk, [0])
        m.forward(pool=pool, slots=[slot], W=W, strides=[s], strain=strain_t[u * s:(u + 1) * s],
                  noise=noise_all[u], clean=clean_all[u], ws=ws)
    torch.cuda.synchronize()
    # offline forward of the same windows, 64 at a time
    zp = torch.cat([torch.zeros((21, W), device=DEV), wit_t], dim=1)
    off = torch.empty((64, W), dtype=torch.float32, device=DEV)
    ws_b = torch.empty(m.workspace_bytes(64, W), dtype=torch.uint8, device=DEV)
    for u0 in range(0, N, 64):
        xs = torch.stack([zp[:, (u + 1) * s:(u + 1) * s + W] for u in range(u0, u0 + 64)]).contiguous()
        m.forward(x=xs, noise=off, ws=ws_b)
        assert torch.equal(off, noise_all[u0:u0 + 64]), f"updates {u0}..{u0 + 63}"
    # oracle on a subset
    check = [0, 1, 63, 126, 127, 128, 129, 1000, 2047, N - 1]
    xs = np.stack([ref.snapshot_after(wit, (u + 1) * s, W) for u in check])
    exp = ref.deepclean_forward(params, xs, layers)
    got = noise_all[check].cpu().numpy()
    assert rel(got, exp) <= FP32_TOL
    st_new = np.stack([strain[u * s:(u + 1) * s] for u in check])
    _, exp_clean = ref.causal_clean(exp, st_new)
    assert rel(clean_all[check].cpu().numpy(), exp_clean) <= FP32_TOL
    # subtraction itself is exact on the device values
    nz = noise_all[:, W - s:]
    assert torch.equal(clean_all, strain_t.reshape(N, s) - nz)


def test_clean_output_mixed_strides(dc):
    """Packed clean outputs for items with different strides in one call."""
    m, params, layers = dc
    W = 4096
    x = synth.gaussian(40, (3, 21, W))
    strides = [16, 256, 1]
    strain = synth.gaussian(41, (sum(strides),))
    xt = torch.from_numpy(x).to(DEV)
    clean = torch.empty(sum(strides), device=DEV)
    m.forward(x=xt, strides=strides, strain=torch.from_numpy(strain).to(DEV), clean=clean)
    torch.cuda.synchronize()
    exp_noise = ref.deepclean_forward(params, x, layers)
    o = 0
    got = clean.cpu().numpy()
    for i, s in enumerate(strides):
        _, ec = ref.causal_clean(exp_noise[i:i + 1], strain[None, o:o + s])
        assert rel(got[o:o + s], ec[0]) <= FP32_TOL
        o += s


# --------------------------------------------------------------------------- BF16 MFMA path
BF16_TOL = 2e-2


@pytest.mark.parametrize("n,W", [(1, 4096), (3, 4096), (2, 32768), (2, 16 * 67)])
def test_forward_bf16(dc, n, W):
    """BF16 operands, FP32 accumulation and epilogue, BF16 activations."""
    m, params, layers = dc
    w, _ = synth.witness_stream(70 + n, n * W)
    x = np.ascontiguousarray(w.reshape(21, n, W).transpose(1, 0, 2))
    got = run_dense(m, x, gs.BF16)
    exp = ref.deepclean_forward(params, x, layers)
    assert rel(got, exp) <= BF16_TOL


def test_streaming_bf16_bitwise(dc):
    """BF16 path: windows read from the rings' BF16 shadow give bitwise the
    same output as the dense offline forward of the same window."""
    m, params, layers = dc
    W, s, N = 32768, 256, 300
    wit, strain = synth.witness_stream(12, N * s)
    wit_t = torch.from_numpy(wit).to(DEV)
    pool = gs.Pool(64 << 20, max_slots=2, max_items=2)
    slot = pool.open(21, W)
    ws = torch.empty(m.workspace_bytes(1, W, gs.BF16), dtype=torch.uint8, device=DEV)
    noise_all = torch.empty((N, W), dtype=torch.float32, device=DEV)
    for u in range(N):
        pool.update([slot], [s], wit_t[:, u * s:(u + 1) * s].contiguous().reshape(-1), [0])
        m.forward(pool=pool, slots=[slot], W=W, noise=noise_all[u], precision=gs.BF16, ws=ws)
    zp = torch.cat([torch.zeros((21, W), device=DEV), wit_t], dim=1)
    off = torch.empty((50, W), dtype=torch.float32, device=DEV)
    for u0 in range(0, N, 50):
        xs = torch.stack([zp[:, (u + 1) * s:(u + 1) * s + W] for u in range(u0, u0 + 50)]).contiguous()
        m.forward(x=xs, noise=off, precision=gs.BF16)
        assert torch.equal(off, noise_all[u0:u0 + 50]), f"updates {u0}..{u0 + 49}"
    check = [0, 127, 128, N - 1]
    xs = np.stack([ref.snapshot_after(wit, (u + 1) * s, W) for u in check])
    assert rel(noise_all[check].cpu().numpy(), ref.deepclean_forward(params, xs, layers)) <= BF16_TOL


@pytest.mark.parametrize("prec,tol", [(gs.FP32, FP32_TOL), (gs.BF16, BF16_TOL)])
def test_pool_batch_mixed_strides(dc, prec, tol):
    """One batched call over several streams with different strides: every
    item's noise window and packed clean block match the oracle."""
    m, params, layers = dc
    W, strides = 4096, [256, 512, 128, 1024]
    n = len(strides)
    pool = gs.Pool(64 << 20, max_slots=8, max_items=8)
    slots = [pool.open(21, W) for _ in range(n)]
    data = [synth.witness_stream(300 + i, 6000) for i in range(n)]
    pos = [0] * n
    for k in range(3):
        blocks = [np.ascontiguousarray(data[i][0][:, pos[i]:pos[i] + strides[i]]).reshape(-1) for i in range(n)]
        offs = np.cumsum([0] + [21 * s for s in strides[:-1]])
        pool.update(slots, strides, torch.from_numpy(np.concatenate(blocks)).to(DEV), offs)
        pos = [p + s for p, s in zip(pos, strides)]
    strain = np.concatenate([data[i][1][pos[i] - strides[i]:pos[i]] for i in range(n)])
    clean = torch.empty(sum(strides), device=DEV)
    noise = torch.empty((n, W), device=DEV)
    m.forward(pool=pool, slots=slots, W=W, strides=strides, strain=torch.from_numpy(strain).to(DEV),
              clean=clean, noise=noise, precision=prec)
    torch.cuda.synchronize()
    xs = np.stack([ref.snapshot_after(data[i][0], pos[i], W) for i in range(n)])
    en = ref.deepclean_forward(params, xs, layers)
    assert rel(noise.cpu().numpy(), en) <= tol
    o = 0
    got = clean.cpu().numpy()
    for i, s in enumerate(strides):
        _, ec = ref.causal_clean(en[i:i + 1], data[i][1][None, pos[i] - s:pos[i]])
        assert rel(got[o:o + s], ec[0]) <= tol
        o += s


@pytest.mark.parametrize("prec", [gs.FP32, gs.BF16])
@pytest.mark.parametrize("W", [4096, 32768])
def test_causal_band_bitwise(dc, prec, W):
    """GW_CAUSAL runs the network only on the band of the window that the
    newest s outputs depend on (receptive field); its clean output is bitwise
    the full-window result, from rings and from dense windows, for mixed
    strides in one call."""
    m, params, layers = dc
    strides = [256, 1, 1024, 16, 512]
    n = len(strides)
    pool = gs.Pool(256 << 20, max_slots=8, max_items=8)
    slots = [pool.open(21, W) for _ in range(n)]
    wit, strain_all = synth.witness_stream(90, W + 3000)
    pos = [0] * n
    for i in range(n):          # fill each ring with a different amount so heads differ
        fill = W // 2 + 997 * i
        blocks, sofar = [], 0
        while sofar < fill:
            s = min(W, fill - sofar)
            pool.update([slots[i]], [s], torch.from_numpy(np.ascontiguousarray(wit[:, sofar:sofar + s])).to(DEV)
                        .reshape(-1), [0])
            sofar += s
        pos[i] = fill
    strain = torch.from_numpy(np.concatenate([strain_all[:s] for s in strides])).to(DEV)
    full = torch.empty(sum(strides), device=DEV)
    band = torch.empty(sum(strides), device=DEV)
    m.forward(pool=pool, slots=slots, W=W, strides=strides, strain=strain, clean=full, precision=prec)
    m.forward(pool=pool, slots=slots, W=W, strides=strides, strain=strain, clean=band, precision=prec,
              flags=gs.CAUSAL)
    torch.cuda.synchronize()
    assert torch.equal(full, band)
    # dense windows
    xs = torch.stack([pool.window(sl) for sl in slots]).contiguous()
    dense_full = torch.empty_like(full)
    dense_band = torch.empty_like(full)
    m.forward(x=xs, strides=strides, strain=strain, clean=dense_full, precision=prec)
    m.forward(x=xs, strides=strides, strain=strain, clean=dense_band, precision=prec, flags=gs.CAUSAL)
    torch.cuda.synchronize()
    assert torch.equal(dense_full, dense_band)
    assert torch.equal(dense_full, full)
    # and the oracle agrees
    x64 = np.stack([ref.snapshot_after(wit, pos[i], W) for i in range(n)])
    en = ref.deepclean_forward(params, x64, layers)
    o = 0
    got = band.cpu().numpy()
    st = strain.cpu().numpy()
    tol = FP32_TOL if prec == gs.FP32 else BF16_TOL
    for i, s in enumerate(strides):
        _, ec = ref.causal_clean(en[i:i + 1], st[None, o:o + s])
        assert rel(got[o:o + s], ec[0]) <= tol
        o += s


@pytest.mark.parametrize("W,n", [(32768, 2), (4096, 3), (16 * 67, 2), (16, 1)])
def test_fused_vs_layerwise_bf16(dc, W, n):
    """The whole-network fused BF16 kernel and the per-layer BF16 kernels both
    match the oracle within the BF16 tolerance (full tiles, a ragged last tile,
    the shortest window)."""
    m, params, layers = dc
    x = synth.gaussian(500 + W, (n, 21, W))
    xt = torch.from_numpy(x).to(DEV)
    a = torch.empty((n, W), device=DEV)
    b = torch.empty((n, W), device=DEV)
    m.forward(x=xt, noise=a, precision=gs.BF16)
    m.forward(x=xt, noise=b, precision=gs.BF16, flags=gs.LAYERWISE)
    torch.cuda.synchronize()
    exp = ref.deepclean_forward(params, x, layers)
    assert rel(a.cpu().numpy(), exp) <= BF16_TOL
    assert rel(b.cpu().numpy(), exp) <= BF16_TOL
    a2 = torch.empty_like(a)
    m.forward(x=xt, noise=a2, precision=gs.BF16)
    torch.cuda.synchronize()
    assert torch.equal(a, a2)   # deterministic


def test_cu_budget_bitwise(dc):
    """A CU budget only resizes the fused kernel's persistent grid (fewer
    blocks, more tiles each): outputs are bitwise those of the full grid.
    Budgets: a few CUs, odd counts, and more CUs than the device has."""
    m, _, _ = dc
    n, W = 5, 32768
    xt = torch.from_numpy(synth.gaussian(611, (n, 21, W))).to(DEV)
    ref_out = torch.empty((n, W), device=DEV)
    m.forward(x=xt, noise=ref_out, precision=gs.BF16)
    try:
        for ncu in (1, 7, 240, 100000):
            m.set_cu_budget(ncu)
            out = torch.empty((n, W), device=DEV)
            m.forward(x=xt, noise=out, precision=gs.BF16)
            torch.cuda.synchronize()
            assert torch.equal(out, ref_out), ncu
    finally:
        m.set_cu_budget(0)
    with pytest.raises(gs.GwError):
        m.set_cu_budget(-1)


@pytest.mark.parametrize("prec,flags,tol", [(gs.FP32, 0, FP32_TOL), (gs.BF16, 0, BF16_TOL),
                                            (gs.BF16, gs.LAYERWISE, BF16_TOL)])
def test_aggregation_delay(dc, prec, flags, tol):
    """Aggregation latency: item i keeps noise[W - s_i - d_i, W - d_i) and
    subtracts it from the strain of that span (delays 0, mid-window, the
    oldest possible block, and a delay that is not a multiple of 16), for
    both clean-output epilogues (fused BF16 kernel, per-layer kernels, FP32);
    GW_CAUSAL with the same delays gives the same clean output bitwise."""
    m, params, layers = dc
    W = 4096
    strides = [256, 512, 128, 1000]
    delays = [0, 1536, W - 128, 37]
    n = len(strides)
    pool = gs.Pool(64 << 20, max_slots=8, max_items=8)
    slots = [pool.open(21, W) for _ in range(n)]
    data = [synth.witness_stream(700 + i, 6000) for i in range(n)]
    fill = [4200, 4096, 5000, 4500]   # each >= W: the ring holds samples [fill - W, fill)
    for i in range(n):
        pool.update([slots[i]], [W], torch.from_numpy(np.ascontiguousarray(data[i][0][:, fill[i] - W:fill[i]]))
                    .to(DEV).reshape(-1), [0])
    # strain block of item i: the s_i samples ending d_i before the newest
    strain = np.concatenate([data[i][1][fill[i] - strides[i] - delays[i]:fill[i] - delays[i]] for i in range(n)])
    st_dev = torch.from_numpy(strain).to(DEV)
    clean = torch.empty(sum(strides), device=DEV)
    noise = torch.empty((n, W), device=DEV)
    m.forward(pool=pool, slots=slots, W=W, strides=strides, delays=delays, strain=st_dev, clean=clean,
              noise=noise, precision=prec, flags=flags)
    torch.cuda.synchronize()
    xs = np.stack([data[i][0][:, fill[i] - W:fill[i]] for i in range(n)])
    en = ref.deepclean_forward(params, xs, layers)
    assert rel(noise.cpu().numpy(), en) <= tol
    got = clean.cpu().numpy()
    o = 0
    for i, s in enumerate(strides):
        seg, ec = ref.delayed_clean(en[i:i + 1], strain[None, o:o + s], delays[i])
        assert rel(got[o:o + s], ec[0]) <= tol, i
        # the noise subtracted is the window's, at the delayed span
        np.testing.assert_array_equal(got[o:o + s], strain[o:o + s] - noise.cpu().numpy()[i, W - s - delays[i]:
                                                                                            W - delays[i]])
        o += s
    if flags == 0:
        band = torch.empty_like(clean)
        m.forward(pool=pool, slots=slots, W=W, strides=strides, delays=delays, strain=st_dev, clean=band,
                  precision=prec, flags=gs.CAUSAL)
        torch.cuda.synchronize()
        assert torch.equal(clean, band)


def test_aggregation_delay_rejected(dc):
    m, _, _ = dc
    W = 4096
    x = torch.zeros((2, 21, W), device=DEV)
    clean = torch.empty(512, device=DEV)
    strain = torch.zeros(512, device=DEV)
    for bad in ([0, -1], [0, W - 255]):
        with pytest.raises(gs.GwError):
            m.forward(x=x, strides=[256, 256], delays=bad, strain=strain, clean=clean, precision=gs.BF16)
    with pytest.raises(gs.GwError):     # delays without a clean output
        m.forward(x=x, noise=torch.empty((2, W), device=DEV), delays=[0, 0], precision=gs.BF16)


def test_overlap_average_kernel(dc):
    """Overlap averaging against the oracle on synthetic prediction windows:
    three streams with different strides, eight successive requests (the
    first depth - 1 average fewer windows), state carried on the device."""
    m, _, _ = dc
    W, depth, K = 1024, 3, 8
    strides = [64, 256, 100]
    n = len(strides)
    wins = [synth.gaussian(40 + i, (K, W)) for i in range(n)]
    strain = [synth.gaussian(60 + i, (K, s)) for i, s in enumerate(strides)]
    state = torch.zeros(m.overlap_state_floats(strides, depth), device=DEV)
    exp = [ref.overlap_average(wins[i], s, depth) for i, s in enumerate(strides)]
    for k in range(K):
        noise = torch.from_numpy(np.stack([wins[i][k] for i in range(n)])).to(DEV)
        st = torch.from_numpy(np.concatenate([strain[i][k] for i in range(n)])).to(DEV)
        avg = torch.empty(sum(strides), device=DEV)
        clean = torch.empty(sum(strides), device=DEV)
        m.overlap_average(noise=noise, strides=strides, depth=depth, counts=[k] * n, state=state, strain=st,
                          clean=clean, avg=avg)
        torch.cuda.synchronize()
        a, c = avg.cpu().numpy(), clean.cpu().numpy()
        o = 0
        for i, s in enumerate(strides):
            assert rel(a[o:o + s], exp[i][k]) <= FP32_TOL, (k, i)
            assert rel(c[o:o + s], strain[i][k] - exp[i][k]) <= FP32_TOL, (k, i)
            o += s


def test_overlap_average_streaming(dc):
    """End to end: ring-resident streams, BF16 forward of every request's
    window, then overlap averaging (depth 4), against the oracle forward of
    the same snapshots averaged by the oracle.  The BF16 bound holds for the
    predicted windows (2e-2 of their largest magnitude); a mean over
    sub-spans of them keeps that absolute bound, so the averaged output is
    checked against 2e-2 of the windows' scale, not of its own span's."""
    m, params, layers = dc
    W, depth, K, s = 4096, 4, 6, 256
    n = 2
    pool = gs.Pool(64 << 20, max_slots=4, max_items=4)
    slots = [pool.open(21, W) for _ in range(n)]
    data = [synth.witness_stream(800 + i, W + K * s)[0] for i in range(n)]
    for i in range(n):
        pool.update([slots[i]], [W], torch.from_numpy(np.ascontiguousarray(data[i][:, :W])).to(DEV).reshape(-1),
                    [0])
    state = torch.zeros(m.overlap_state_floats([s] * n, depth), device=DEV)
    ws = torch.empty(m.workspace_bytes(n, W, gs.BF16), dtype=torch.uint8, device=DEV)
    got = np.zeros((n, K, s))
    snaps = np.zeros((n, K, 21, W))
    for k in range(K):
        blocks = np.concatenate([np.ascontiguousarray(data[i][:, W + k * s:W + (k + 1) * s]).reshape(-1)
                                 for i in range(n)])
        pool.update(slots, [s] * n, torch.from_numpy(blocks).to(DEV), [0, 21 * s])
        noise = torch.empty((n, W), device=DEV)
        m.forward(pool=pool, slots=slots, W=W, noise=noise, precision=gs.BF16, ws=ws)
        avg = torch.empty(n * s, device=DEV)
        m.overlap_average(noise=noise, strides=[s] * n, depth=depth, counts=[k] * n, state=state, avg=avg)
        torch.cuda.synchronize()
        got[:, k] = avg.cpu().numpy().reshape(n, s)
        for i in range(n):
            snaps[i, k] = data[i][:, (k + 1) * s:(k + 1) * s + W]
    for i in range(n):
        wins = ref.deepclean_forward(params, snaps[i], layers)
        exp = ref.overlap_average(wins, s, depth)
        assert np.max(np.abs(got[i] - exp)) <= BF16_TOL * np.max(np.abs(wins)), i


def test_overlap_average_rejected(dc):
    m, _, _ = dc
    noise = torch.zeros((1, 64), device=DEV)
    state = torch.zeros(64, device=DEV)
    avg = torch.empty(32, device=DEV)
    with pytest.raises(gs.GwError):     # depth * s > W
        m.overlap_average(noise=noise, strides=[32], depth=3, counts=[0], state=state, avg=avg)
    with pytest.raises(gs.GwError):     # no output
        m.overlap_average(noise=noise, strides=[32], depth=2, counts=[0], state=state)
    with pytest.raises(gs.GwError):     # negative count
        m.overlap_average(noise=noise, strides=[32], depth=2, counts=[-1], state=state, avg=avg)


# ---------------------------------------------------------------- FP16 variant
FP16_TOL = 2.5e-3   # the BF16 bound scaled by the ratio of the unit roundoffs (2^-11 / 2^-8)


@pytest.mark.parametrize("W,n", [(32768, 2), (4096, 3), (16 * 67, 2), (16, 1)])
def test_forward_fp16(dc, W, n):
    """FP16 operands in the fused kernel (FP32 accumulation and epilogue):
    within the FP16 bound of the oracle and at least 4x closer than BF16 on
    the same input (full tiles, a ragged last tile, the shortest window)."""
    m, params, layers = dc
    x = synth.gaussian(620 + W, (n, 21, W))
    xt = torch.from_numpy(x).to(DEV)
    a = torch.empty((n, W), device=DEV)
    b = torch.empty((n, W), device=DEV)
    m.forward(x=xt, noise=a, precision=gs.FP16)
    m.forward(x=xt, noise=b, precision=gs.BF16)
    torch.cuda.synchronize()
    exp = ref.deepclean_forward(params, x, layers)
    e16, ebf = rel(a.cpu().numpy(), exp), rel(b.cpu().numpy(), exp)
    assert e16 <= FP16_TOL
    assert e16 * 4 <= ebf


def test_fp16_ring_equals_dense_and_causal(dc):
    """The FP16 kernel reads the rings' FP32 samples (wrapping at each ring's
    head): outputs from rings equal those from the same windows passed
    densely, bitwise; GW_CAUSAL gives the full-window clean output bitwise."""
    m, params, layers = dc
    W, strides = 4096, [256, 1, 1024, 512]
    n = len(strides)
    pool = gs.Pool(64 << 20, max_slots=8, max_items=8)
    slots = [pool.open(21, W) for _ in range(n)]
    wit, strain_all = synth.witness_stream(91, W + 3000)
    for i in range(n):
        fill = W // 2 + 997 * i + 3          # heads not multiples of 8 for some rings
        sofar = 0
        while sofar < fill:
            s = min(W, fill - sofar)
            pool.update([slots[i]], [s], torch.from_numpy(np.ascontiguousarray(wit[:, sofar:sofar + s])).to(DEV)
                        .reshape(-1), [0])
            sofar += s
    strain = torch.from_numpy(np.concatenate([strain_all[:s] for s in strides])).to(DEV)
    noise_r = torch.empty((n, W), device=DEV)
    full = torch.empty(sum(strides), device=DEV)
    band = torch.empty(sum(strides), device=DEV)
    m.forward(pool=pool, slots=slots, W=W, strides=strides, strain=strain, clean=full, noise=noise_r,
              precision=gs.FP16)
    m.forward(pool=pool, slots=slots, W=W, strides=strides, strain=strain, clean=band, precision=gs.FP16,
              flags=gs.CAUSAL)
    xs = torch.stack([pool.window(sl) for sl in slots]).contiguous()
    noise_d = torch.empty((n, W), device=DEV)
    m.forward(x=xs, noise=noise_d, precision=gs.FP16)
    torch.cuda.synchronize()
    assert torch.equal(noise_r, noise_d)
    assert torch.equal(full, band)
    exp = ref.deepclean_forward(params, xs.cpu().numpy().astype(np.float64), layers)
    assert rel(noise_r.cpu().numpy(), exp) <= FP16_TOL


def test_fp16_unsupported_paths(dc):
    m, _, _ = dc
    x = torch.zeros((1, 21, 4096), device=DEV)
    noise = torch.empty((1, 4096), device=DEV)
    for flags in (gs.LAYERWISE, gs.TRAIN):
        with pytest.raises(gs.GwError) as e:
            m.forward(x=x, noise=noise, precision=gs.FP16, flags=flags)
        assert e.value.code == gs.GW_EUNSUPPORTED
    bbm = gs.BBHnet(torch.from_numpy(synth.bbhnet_params(0)).to(DEV), synth.bbhnet_stages())
    with pytest.raises(gs.GwError) as e:
        bbm.forward(x=torch.zeros((1, 2, 2048), device=DEV), precision=gs.FP16)
    assert e.value.code == gs.GW_EUNSUPPORTED
