"""GPU parity of the BBHnet-shaped classifier against the FP64 oracle, dense
and from snapshot rings: the FP32 path, and the BF16 path both as the fused
whole-network kernel (the default for this shape) and as per-layer kernels."""
import numpy as np
import pytest
import torch

from oracle import ref
from paper_2108_12430_amd import gwstream as gs
from paper_2108_12430_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rel(a, r):
    return float(np.max(np.abs(np.asarray(a, np.float64) - r)) / np.max(np.abs(r)))


@pytest.fixture(scope="module")
def bb():
    params = synth.bbhnet_params(0)
    m = gs.BBHnet(torch.from_numpy(params).to(DEV), synth.bbhnet_stages())
    return m, params


@pytest.fixture(autouse=True)
def _fused_after_each_test(bb):
    yield
    bb[0].set_layerwise(False)


MODES = [pytest.param(False, id="fused"), pytest.param(True, id="layerwise")]


def test_bbhnet_refresh_rederives_every_path():
    """After the parameters change in place and gw_model_refresh, the FP32
    path and the BF16 fused and per-layer paths compute with the new
    parameters (oracle at the new parameters), and the change is large
    enough that the old logits are far outside the bounds."""
    p0 = synth.bbhnet_params(0)
    params = torch.from_numpy(p0.copy()).to(DEV)
    m = gs.BBHnet(params, synth.bbhnet_stages())
    x, _ = synth.bbh_windows(91, 32)
    xt = torch.from_numpy(x).to(DEV)
    old = m.forward(x=xt, precision=gs.BF16).cpu().numpy()
    rng = np.random.default_rng(11)
    p1 = (p0 * np.exp(0.2 * rng.standard_normal(p0.shape))).astype(np.float32)
    params.copy_(torch.from_numpy(p1))
    m.refresh()
    exp = ref.bbhnet_forward(p1, x)
    assert rel(old, exp) > 5e-2
    assert rel(m.forward(x=xt).cpu().numpy(), exp) <= 1e-5
    assert rel(m.forward(x=xt, precision=gs.BF16).cpu().numpy(), exp) <= 2e-2
    m.set_layerwise(True)
    assert rel(m.forward(x=xt, precision=gs.BF16).cpu().numpy(), exp) <= 2e-2


@pytest.mark.parametrize("B", [64, 256, 1024])
def test_bbhnet_fp32(bb, B):
    m, params = bb
    x, _ = synth.bbh_windows(3 + B, B)
    got = m.forward(x=torch.from_numpy(x).to(DEV)).cpu().numpy()
    # each logit depends only on its own window: check a sample of 64 of them
    idx = np.sort(np.random.default_rng(B).choice(B, size=min(B, 64), replace=False))
    exp = ref.bbhnet_forward(params, x[idx])
    assert rel(got[idx], exp) <= 1e-5


@pytest.mark.parametrize("W", [8, 264, 2048 + 512])
def test_bbhnet_shapes(bb, W):
    m, params = bb
    x = synth.gaussian(W, (3, 2, W))
    got = m.forward(x=torch.from_numpy(x).to(DEV)).cpu().numpy()
    assert rel(got, ref.bbhnet_forward(params, x)) <= 1e-5


def test_bbhnet_from_pool_bitwise(bb):
    m, params = bb
    W, n = 2048, 5
    pool = gs.Pool(1 << 24, max_slots=8, max_items=8)
    slots = [pool.open(2, W) for _ in range(n)]
    x, _ = synth.bbh_windows(9, n, n=W + 300)
    # feed 300 + 2048 samples in strides of 128..512 so the rings wrap
    pos = [0] * n
    rng = np.random.default_rng(1)
    while min(pos) < W + 300:
        strides = [int(min(rng.choice([128, 256, 512]), W + 300 - p)) or 1 for p in pos]
        act = [i for i in range(n) if pos[i] < W + 300]
        blocks, offs, o = [], [], 0
        for i in act:
            blocks.append(x[i, :, pos[i]:pos[i] + strides[i]].reshape(-1))
            offs.append(o)
            o += 2 * strides[i]
        pool.update([slots[i] for i in act], [strides[i] for i in act],
                    torch.from_numpy(np.concatenate(blocks)).to(DEV), offs)
        for i in act:
            pos[i] += strides[i]
    got = m.forward(pool=pool, slots=slots, W=W).cpu().numpy()
    dense = np.ascontiguousarray(x[:, :, -W:])
    got_d = m.forward(x=torch.from_numpy(dense).to(DEV)).cpu().numpy()
    assert np.array_equal(got, got_d)
    assert rel(got, ref.bbhnet_forward(params, dense)) <= 1e-5


@pytest.mark.parametrize("B", [8, 64, 256, 1024])
@pytest.mark.parametrize("layerwise", MODES)
def test_bbhnet_bf16(bb, B, layerwise):
    """BF16 MFMA convolutions with FP32 accumulation, epilogue and logits.
    Per-layer kernels: 8 windows take the small-batch kernels in every layer,
    64 and 256 a mix (the wide layers switch to the weight-staging kernels
    first), 1024 the weight-staging kernels in every layer."""
    m, params = bb
    m.set_layerwise(layerwise)
    x, _ = synth.bbh_windows(3 + B, B)
    got = m.forward(x=torch.from_numpy(x).to(DEV), precision=gs.BF16).cpu().numpy()
    idx = np.sort(np.random.default_rng(B + 1).choice(B, size=min(B, 64), replace=False))
    exp = ref.bbhnet_forward(params, x[idx])
    assert rel(got[idx], exp) <= 2e-2


@pytest.mark.parametrize("layerwise", MODES)
def test_bbhnet_bf16_batch_independent(bb, layerwise):
    """24 and 12 windows take the same (small-batch) kernel in every layer:
    a window's logit does not depend on the rest of the batch."""
    m, _ = bb
    m.set_layerwise(layerwise)
    x, _ = synth.bbh_windows(77, 24)
    xt = torch.from_numpy(x).to(DEV)
    full = m.forward(x=xt, precision=gs.BF16)
    part = m.forward(x=xt[7:19].contiguous(), precision=gs.BF16)
    assert torch.equal(full[7:19], part)


def test_bbhnet_bf16_across_kernel_modes(bb):
    """64 windows run the wide layers of stages 1 and 2 on the weight-staging
    kernels, 12 windows every layer on the small-batch kernels: the same
    windows agree to well within the BF16 bound (only the summation order
    differs)."""
    m, params = bb
    m.set_layerwise(True)
    x, _ = synth.bbh_windows(81, 64)
    xt = torch.from_numpy(x).to(DEV)
    full = m.forward(x=xt, precision=gs.BF16).cpu().numpy()
    part = m.forward(x=xt[20:32].contiguous(), precision=gs.BF16).cpu().numpy()
    assert rel(full[20:32], part) <= 2e-3
    assert rel(part, ref.bbhnet_forward(params, x[20:32])) <= 2e-2


@pytest.mark.parametrize("layerwise", MODES)
def test_bbhnet_bf16_batch_independent_large(bb, layerwise):
    """Large batches use the weight-staging variants (every layer of both
    calls below); a window's logit does not depend on the rest of the batch."""
    m, _ = bb
    m.set_layerwise(layerwise)
    x, _ = synth.bbh_windows(78, 1024)
    xt = torch.from_numpy(x).to(DEV)
    full = m.forward(x=xt, precision=gs.BF16)
    part = m.forward(x=xt[256:768].contiguous(), precision=gs.BF16)
    assert torch.equal(full[256:768], part)


@pytest.mark.parametrize("layerwise", MODES)
def test_bbhnet_bf16_large_batch_ragged_window(bb, layerwise):
    """Large-batch variants on a window whose layer lengths are not multiples
    of their 128/256-column tiles (2576 -> 1288 -> 644 -> 322): sampled
    windows against the oracle."""
    m, params = bb
    m.set_layerwise(layerwise)
    B, W = 1024, 2576
    x = synth.gaussian(79, (B, 2, W))
    got = m.forward(x=torch.from_numpy(x).to(DEV), precision=gs.BF16).cpu().numpy()
    assert np.isfinite(got).all()
    idx = np.sort(np.random.default_rng(80).choice(B, size=24, replace=False))
    assert rel(got[idx], ref.bbhnet_forward(params, x[idx])) <= 2e-2


@pytest.mark.parametrize("W", [8, 264, 2048, 2560, 2576])
def test_bbhnet_fused_shapes(bb, W):
    """The fused kernel at window lengths whose last stage is shorter than one
    64-position tile (8, 264), exactly whole tiles (2048, 2560) and a ragged
    last tile (2576 -> 322): against the oracle and the per-layer kernels."""
    m, params = bb
    x = synth.gaussian(W + 1, (6, 2, W))
    xt = torch.from_numpy(x).to(DEV)
    got = m.forward(x=xt, precision=gs.BF16).cpu().numpy()
    exp = ref.bbhnet_forward(params, x)
    assert rel(got, exp) <= 2e-2
    m.set_layerwise(True)
    lw = m.forward(x=xt, precision=gs.BF16).cpu().numpy()
    assert rel(lw, exp) <= 2e-2
    print(f"W={W}: fused {rel(got, exp):.1e}, per-layer {rel(lw, exp):.1e}, apart {rel(got, lw):.1e}")


def test_bbhnet_fused_from_rings_bitwise(bb):
    """Windows read in place from wrapped snapshot rings give bitwise the
    logits of the same windows as dense input (the ring's BF16 shadow holds
    exactly the rounding the dense staging applies)."""
    m, params = bb
    W, n = 2048, 7
    pool = gs.Pool(1 << 24, max_slots=8, max_items=8)
    slots = [pool.open(2, W) for _ in range(n)]
    x, _ = synth.bbh_windows(19, n, n=W + 700)
    for k in range((W + 700) // 100):
        pool.update(slots, [100] * n, torch.from_numpy(
            np.concatenate([x[i, :, 100 * k:100 * (k + 1)].reshape(-1) for i in range(n)])).to(DEV),
            [200 * i for i in range(n)])
    got = m.forward(pool=pool, slots=slots, W=W, precision=gs.BF16).cpu().numpy()
    dense = np.ascontiguousarray(x[:, :, 100 * ((W + 700) // 100) - W:100 * ((W + 700) // 100)])
    got_d = m.forward(x=torch.from_numpy(dense).to(DEV), precision=gs.BF16).cpu().numpy()
    assert np.array_equal(got, got_d)
    assert rel(got, ref.bbhnet_forward(params, dense)) <= 2e-2
