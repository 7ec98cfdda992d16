"""GPU parity of the DeepClean training step (batch-statistics forward,
band-passed MSE, hand-written backward) against the FP64 oracle."""
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


def tensor_slices(layers):
    """(name, start, stop) of every parameter tensor in the flat vector."""
    out, off = [], 0
    for l, (typ, ci, co, k, s, p, op, bn) in enumerate(layers):
        for name, n in [("w", ci * co * k), ("b", co)] + ([("gamma", co), ("beta", co), ("mean", co),
                                                             ("var", co)] if bn else []):
            out.append((f"L{l}.{name}", off, off + n))
            off += n
    return out


def grad_errors(got, exp, layers):
    """Per-tensor normwise error.  Some gradients are exactly zero: the bias of
    a conv followed by batch normalisation (the batch mean removes it) and the
    output bias under the band-passed loss (the band excludes the DC bin).
    For such a tensor (reference below 1e-12 of the largest gradient) the
    error is measured against the largest gradient of the layer's weight."""
    errs = {}
    sl = tensor_slices(layers)
    top = np.max(np.abs(exp))
    for name, a, b in sl:
        if name.endswith(".mean") or name.endswith(".var"):
            assert np.all(got[a:b] == 0)
            continue
        r = exp[a:b]
        scale = np.max(np.abs(r))
        if scale < 1e-12 * top:
            lname = name.split(".")[0]
            wa, wb = [(x, y) for nm, x, y in sl if nm == lname + ".w"][0]
            scale = np.max(np.abs(exp[wa:wb]))
        errs[name] = float(np.max(np.abs(got[a:b] - r)) / scale)
    return errs


def test_bandpass_loss_and_grad():
    n, W = 4, 32768
    strain = synth.gaussian(50, (n, W))
    t = np.arange(W) / 4096.0
    strain = (strain + 2 * np.sin(2 * np.pi * 60.3 * t)).astype(np.float32)
    noise = synth.gaussian(51, (n, W), 0.5)
    loss, dn = gs.bandpass_mse(torch.from_numpy(strain).to(DEV), torch.from_numpy(noise).to(DEV))
    el, edn = ref.bandpass_mse(strain, noise, 4096.0, 55.0, 65.0)
    assert abs(loss.item() - el) <= 1e-5 * abs(el)
    assert rel(dn.cpu().numpy(), edn) <= 1e-5


@pytest.mark.parametrize("n,W,f_lo,f_hi", [
    (33, 4096, 55.0, 65.0),      # 11 bins: two window groups of the 32-window gradient kernel
    (3, 4096, 10.0, 1500.0),     # 1491 bins: the two-window kernel
    (2, 32768, 0.0, 2048.0),     # 16385 bins (DC and Nyquist included): the wide-band kernel
])
def test_bandpass_gradient_paths(n, W, f_lo, f_hi):
    """The band-passed loss and gradient against the oracle for bands that
    take each of the gradient kernel's paths, with ragged window groups."""
    strain = synth.gaussian(52, (n, W))
    noise = synth.gaussian(53, (n, W), 0.5)
    loss, dn = gs.bandpass_mse(torch.from_numpy(strain).to(DEV), torch.from_numpy(noise).to(DEV), 4096.0, f_lo, f_hi)
    el, edn = ref.bandpass_mse(strain, noise, 4096.0, f_lo, f_hi)
    assert abs(loss.item() - el) <= 1e-5 * abs(el)
    assert rel(dn.cpu().numpy(), edn) <= 1e-5


def _train_step(m, x, strain, flags, fs=4096.0, lossfn="bandpass"):
    n, W = x.shape[0], x.shape[-1]
    xt = torch.from_numpy(x).to(DEV)
    st = torch.from_numpy(strain).to(DEV)
    noise = torch.empty((n, W), device=DEV)
    ws = m.forward(x=xt, noise=noise, flags=flags)
    if lossfn == "bandpass":
        loss, dn = gs.bandpass_mse(st, noise, fs, 55.0, 65.0)
    else:
        dn = (-2.0 / (n * W)) * (st - noise)
    dp = torch.empty_like(m.params)
    m.backward(xt, dn.contiguous(), ws, dp, flags=flags)
    torch.cuda.synchronize()
    return noise.cpu().numpy(), dp.cpu().numpy()


@pytest.mark.parametrize("lossfn", ["bandpass", "mse"])
def test_grad_tiny_instance(lossfn):
    """Two-layer, four-channel, 256-sample instance: GPU gradient vs the
    oracle gradient (which is itself pinned by finite differences)."""
    layers = synth.tiny_layers()
    params = synth.deepclean_params(5, layers)
    m = gs.DeepClean(torch.from_numpy(params).to(DEV), layers)
    x = synth.gaussian(5, (2, 4, 256))
    t = np.arange(256) / 4096.0
    strain = (synth.gaussian(6, (2, 256)) + 3 * np.sin(2 * np.pi * 64 * t)).astype(np.float32)
    noise, g = _train_step(m, x, strain, gs.TRAIN, lossfn=lossfn)
    en = ref.deepclean_forward(params, x, layers, train=True)
    assert rel(noise, en) <= 1e-5
    if lossfn == "bandpass":
        _, dn = ref.bandpass_mse(strain, en, 4096.0, 55.0, 65.0)
    else:
        _, dn = ref.mse(strain, en)
    eg = ref.deepclean_grad(params, x, dn, layers)
    errs = grad_errors(g, eg, layers)
    assert max(errs.values()) <= 1e-5, errs


def test_grad_full_window():
    """8-s windows (21 x 32768) through the full network, batch 4, band-passed
    loss: per-tensor error of every gradient against the oracle."""
    layers = synth.deepclean_layers()
    params = synth.deepclean_params(0)
    m = gs.DeepClean(torch.from_numpy(params).to(DEV), layers)
    wit, strain = synth.witness_stream(4, 4 * 32768)
    x = np.ascontiguousarray(wit.reshape(21, 4, 32768).transpose(1, 0, 2))
    sb = np.ascontiguousarray(strain.reshape(4, 32768))
    noise, g = _train_step(m, x, sb, gs.TRAIN)
    en = ref.deepclean_forward(params, x, layers, train=True)
    assert rel(noise, en) <= 1e-5
    _, dn = ref.bandpass_mse(sb, en, 4096.0, 55.0, 65.0)
    eg = ref.deepclean_grad(params, x, dn, layers)
    errs = grad_errors(g, eg, layers)
    assert max(errs.values()) <= 1e-5, errs


def test_recompute_bitwise():
    layers = synth.deepclean_layers()
    params = synth.deepclean_params(0)
    m = gs.DeepClean(torch.from_numpy(params).to(DEV), layers)
    x = synth.gaussian(60, (2, 21, 8192))
    strain = synth.gaussian(61, (2, 8192))
    n0, g0 = _train_step(m, x, strain, gs.TRAIN)
    n1, g1 = _train_step(m, x, strain, gs.TRAIN | gs.RECOMPUTE)
    assert np.array_equal(n0, n1)
    assert np.array_equal(g0, g1)
    assert m.workspace_bytes(2, 8192, gs.FP32, gs.TRAIN | gs.RECOMPUTE) < m.workspace_bytes(2, 8192, gs.FP32,
                                                                                             gs.TRAIN)
    n2, g2 = _train_step(m, x, strain, gs.TRAIN)
    assert np.array_equal(g0, g2)   # deterministic across runs


def test_autograd_function_and_training_steps():
    """DeepCleanFn exposes the hand-written backward to torch.autograd: its
    parameter gradient equals the oracle's, and a few optimizer steps with the
    band-passed loss lower that loss."""
    from paper_2108_12430_amd.autograd import DeepCleanFn, bandpass_mse_loss, train_step
    layers = synth.deepclean_layers()
    p0 = synth.deepclean_params(0)
    params = torch.from_numpy(p0.copy()).to(DEV).requires_grad_(True)
    m = gs.DeepClean(params.detach(), layers)
    wit, strain = synth.witness_stream(8, 2 * 8192)
    x = torch.from_numpy(np.ascontiguousarray(wit.reshape(21, 2, 8192).transpose(1, 0, 2))).to(DEV)
    st = torch.from_numpy(np.ascontiguousarray(strain.reshape(2, 8192))).to(DEV)
    noise = DeepCleanFn.apply(params, x, m, True)
    loss = bandpass_mse_loss(st, noise)
    loss.backward()
    xn = x.cpu().numpy()
    sn = st.cpu().numpy()
    en = ref.deepclean_forward(p0, xn, layers, train=True)
    el, dn = ref.bandpass_mse(sn, en, 4096.0, 55.0, 65.0)
    assert abs(loss.item() - el) <= 1e-5 * abs(el)
    eg = ref.deepclean_grad(p0, xn, dn, layers)
    errs = grad_errors(params.grad.cpu().numpy(), eg, layers)
    assert max(errs.values()) <= 1e-5, errs
    opt = torch.optim.SGD([params], lr=0.05)
    losses = [train_step(m, params, opt, x, st).item() for _ in range(4)]
    assert losses[-1] < losses[0]


def test_grad_bf16_conv_variant():
    """Training step with the forward (and recomputed) convolutions on BF16
    matrix cores, each FP32 operand split into two BF16 terms (three MFMAs
    per product); activations, statistics and gradients stay FP32.  Every
    output and gradient tensor within the BF16 bound 2e-2 of the oracle;
    recomputation still bitwise."""
    layers = synth.deepclean_layers()
    params = synth.deepclean_params(0)
    m = gs.DeepClean(torch.from_numpy(params).to(DEV), layers)
    wit, strain = synth.witness_stream(14, 2 * 32768)
    x = np.ascontiguousarray(wit.reshape(21, 2, 32768).transpose(1, 0, 2))
    sb = np.ascontiguousarray(strain.reshape(2, 32768))
    xt = torch.from_numpy(x).to(DEV)
    st = torch.from_numpy(sb).to(DEV)
    out = []
    for flags in (gs.TRAIN, gs.TRAIN | gs.RECOMPUTE):
        noise = torch.empty((2, 32768), device=DEV)
        ws = m.forward(x=xt, noise=noise, flags=flags, precision=gs.BF16)
        _, dn = gs.bandpass_mse(st, noise)
        dp = torch.empty_like(m.params)
        m.backward(xt, dn, ws, dp, flags=flags, precision=gs.BF16)
        torch.cuda.synchronize()
        out.append((noise.cpu().numpy(), dp.cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    en = ref.deepclean_forward(params, x, layers, train=True)
    err_noise = rel(out[0][0], en)
    _, dn = ref.bandpass_mse(sb, en, 4096.0, 55.0, 65.0)
    eg = ref.deepclean_grad(params, x, dn, layers)
    errs = grad_errors(out[0][1], eg, layers)
    print("bf16 split training, batch 2: noise", f"{err_noise:.2e}",
          {k: f"{v:.1e}" for k, v in errs.items()})
    assert err_noise <= 2e-2
    assert max(errs.values()) <= 2e-2, errs


@pytest.fixture(scope="module")
def batch32():
    """The benchmark's training configuration: 32 distinct 8-s windows of 21
    witness channels and strain, with the oracle's batch-statistics forward
    and band-passed-loss gradient (FP64)."""
    B, W = 32, 32768
    layers = synth.deepclean_layers()
    params = synth.deepclean_params(0)
    wit, strain = synth.witness_stream(40, B * W)
    x = np.ascontiguousarray(wit.reshape(21, B, W).transpose(1, 0, 2))
    sb = np.ascontiguousarray(strain.reshape(B, W))
    en = ref.deepclean_forward(params, x, layers, train=True)
    _, dn = ref.bandpass_mse(sb, en, 4096.0, 55.0, 65.0)
    eg = ref.deepclean_grad(params, x, dn, layers)
    return layers, params, x, sb, en, eg


@pytest.mark.parametrize("precision,bound", [("fp32", 1e-5), ("bf16", 2e-2)])
def test_grad_batch32_benchmark_config(batch32, precision, bound):
    """Batch 32 x 21 x 32768 with recomputation, as the training benchmark
    runs it: the per-channel statistics chunking and the weight-gradient
    reduction tree at this size, every gradient tensor against the oracle
    (FP32 <= 1e-5, BF16-conv variant <= 2e-2)."""
    layers, params, x, sb, en, eg = batch32
    m = gs.DeepClean(torch.from_numpy(params).to(DEV), layers)
    prec = gs.BF16 if precision == "bf16" else gs.FP32
    flags = gs.TRAIN | gs.RECOMPUTE
    xt = torch.from_numpy(x).to(DEV)
    st = torch.from_numpy(sb).to(DEV)
    noise = torch.empty(sb.shape, device=DEV)
    ws = m.forward(x=xt, noise=noise, flags=flags, precision=prec)
    _, dn = gs.bandpass_mse(st, noise)
    dp = torch.empty_like(m.params)
    m.backward(xt, dn, ws, dp, flags=flags, precision=prec)
    torch.cuda.synchronize()
    err_noise = rel(noise.cpu().numpy(), en)
    errs = grad_errors(dp.cpu().numpy(), eg, layers)
    print(f"{precision} training, batch 32: noise {err_noise:.2e}", {k: f"{v:.1e}" for k, v in errs.items()})
    assert err_noise <= bound
    assert max(errs.values()) <= bound, errs
