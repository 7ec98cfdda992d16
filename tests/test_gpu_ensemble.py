"""End-to-end ensemble (main text, second offline workflow): streaming
decimation kernel against the oracle's whole-signal definition, and the full
pipeline -- two detectors' witness snapshots, DeepClean-H1/L1 with the
fully-online clean output, decimation to 2048 Hz into the BBHnet ring,
BBHnet logits -- against the oracle pipeline over successive requests."""
import numpy as np
import pytest
import torch

from oracle import ref
from paper_2108_12430_amd import ensemble
from paper_2108_12430_amd import gwstream as gs
from paper_2108_12430_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rel(a, r):
    a = np.asarray(a, np.float64)
    r = np.asarray(r, np.float64)
    return float(np.max(np.abs(a - r)) / np.max(np.abs(r)))


@pytest.mark.parametrize("s,K", [(128, 63), (256, 7), (16, 63), (2, 1)])
def test_decimate2_streaming(s, K):
    """Blocks of s samples through gw_decimate2 with the history carried on
    the device give the oracle's decimation of the whole stream (blocks
    shorter than the filter included)."""
    n, C, B = 3, 2, 6
    x = synth.gaussian(900 + s + K, (C, n, B * s))
    taps = ref.lowpass_taps(K, 0.225) if K > 1 else np.array([1.0])
    tt = torch.from_numpy(taps.astype(np.float32)).to(DEV)
    hist = torch.zeros((n, C, max(K - 1, 1)), device=DEV)
    got = np.zeros((n, C, B * s // 2))
    for b in range(B):
        xb = torch.from_numpy(np.ascontiguousarray(x[:, :, b * s:(b + 1) * s])).to(DEV)
        y = torch.empty((n, C, s // 2), device=DEV)
        gs.decimate2(x=xb, taps=tt, hist=hist, y=y)
        torch.cuda.synchronize()
        got[:, :, b * s // 2:(b + 1) * s // 2] = y.cpu().numpy()
    want = ref.decimate2(np.transpose(x, (1, 0, 2)), taps.astype(np.float32))
    assert rel(got, want) <= 1e-5


def test_decimate2_rejected():
    x = torch.zeros((2, 1, 8), device=DEV)
    taps = torch.ones(3, device=DEV)
    hist = torch.zeros((1, 2, 2), device=DEV)
    with pytest.raises(gs.GwError):       # odd stride
        gs.decimate2(x=torch.zeros((2, 1, 7), device=DEV), taps=taps, hist=hist, y=torch.empty(8, device=DEV))
    with pytest.raises(gs.GwError):       # too many taps
        gs.decimate2(x=x, taps=torch.ones(300, device=DEV), hist=torch.zeros(600, device=DEV),
                     y=torch.empty(8, device=DEV))


@pytest.mark.parametrize("prec", [gs.FP32, gs.BF16])
def test_ensemble_matches_oracle(prec):
    """Two ensemble streams, four requests each: the logits of every request
    against the oracle pipeline (FP32: 1e-5 normwise over all logits; BF16:
    the 2e-2 bound)."""
    n, W_dc, W_bb, s, K = 2, 4096, 2048, 256, 4
    dcp = [synth.deepclean_params(0), synth.deepclean_params(1)]
    bbp = synth.bbhnet_params(0)
    layers = synth.deepclean_layers()
    dcm = [gs.DeepClean(torch.from_numpy(p).to(DEV), layers) for p in dcp]
    bbm = gs.BBHnet(torch.from_numpy(bbp).to(DEV), synth.bbhnet_stages())
    taps = ref.lowpass_taps(63, 0.225)
    ens = ensemble.Ensemble(dcm[0], dcm[1], bbm, n, W_dc=W_dc, W_bb=W_bb, stride=s, taps=taps, precision=prec)
    U = W_dc + K * s
    # per stream and detector: witnesses [21][U] and strain [U]
    data = [[synth.witness_stream(1000 + 10 * i + d, U) for d in range(2)] for i in range(n)]
    wit0 = np.stack([np.stack([data[i][d][0][:, :W_dc] for i in range(n)]) for d in range(2)])
    ens.prefill(torch.from_numpy(np.ascontiguousarray(wit0)).to(DEV))
    got = np.zeros((n, K))
    for k in range(K):
        a, b = W_dc + k * s, W_dc + (k + 1) * s
        wit = np.stack([np.stack([data[i][d][0][:, a:b] for i in range(n)]) for d in range(2)])
        st = np.stack([np.stack([data[i][d][1][a:b] for i in range(n)]) for d in range(2)])
        lg = ens.step(torch.from_numpy(np.ascontiguousarray(wit)).to(DEV), torch.from_numpy(st).to(DEV))
        torch.cuda.synchronize()
        got[:, k] = lg.cpu().numpy()
    want = np.stack([ref.ensemble_logits(dcp, np.stack([data[i][d][0] for d in range(2)]),
                                         np.stack([data[i][d][1] for d in range(2)]), bbp,
                                         taps.astype(np.float32), s, W_dc, W_bb, K) for i in range(n)])
    assert np.isfinite(got).all()
    assert rel(got, want) <= (1e-5 if prec == gs.FP32 else 2e-2)


def test_ensemble_bench_configuration():
    """The benchmark's ensemble launch: 64 streams, 21 x 32768 witness
    snapshots per detector, BBHnet 2 x 2048, 256 new samples per request,
    BF16.  Two requests; every logit finite; two sampled streams against the
    oracle pipeline (2e-2 normwise over their logits)."""
    n, W_dc, W_bb, s, K = 64, 32768, 2048, 256, 2
    dcp = [synth.deepclean_params(0), synth.deepclean_params(1)]
    bbp = synth.bbhnet_params(0)
    layers = synth.deepclean_layers()
    dcm = [gs.DeepClean(torch.from_numpy(p).to(DEV), layers) for p in dcp]
    bbm = gs.BBHnet(torch.from_numpy(bbp).to(DEV), synth.bbhnet_stages())
    taps = ref.lowpass_taps(63, 0.225)
    ens = ensemble.Ensemble(dcm[0], dcm[1], bbm, n, W_dc=W_dc, W_bb=W_bb, stride=s, taps=taps, precision=gs.BF16)
    U = W_dc + K * s
    pick = (5, 50)
    data = {i: [synth.witness_stream(2000 + 10 * i + d, U) for d in range(2)] for i in pick}
    wit = torch.from_numpy(synth.gaussian(77, (2, n, 21, U))).to(DEV)
    st = torch.from_numpy(synth.gaussian(78, (2, n, U))).to(DEV)
    for i in pick:
        for d in range(2):
            wit[d, i] = torch.from_numpy(data[i][d][0]).to(DEV)
            st[d, i] = torch.from_numpy(data[i][d][1]).to(DEV)
    ens.prefill(wit[..., :W_dc].contiguous())
    got = np.zeros((n, K))
    for k in range(K):
        a, b = W_dc + k * s, W_dc + (k + 1) * s
        lg = ens.step(wit[..., a:b].contiguous(), st[..., a:b].contiguous())
        torch.cuda.synchronize()
        got[:, k] = lg.cpu().numpy()
    assert np.isfinite(got).all()
    want = np.stack([ref.ensemble_logits(dcp, np.stack([data[i][d][0] for d in range(2)]),
                                         np.stack([data[i][d][1] for d in range(2)]), bbp,
                                         taps.astype(np.float32), s, W_dc, W_bb, K) for i in pick])
    assert rel(got[list(pick)], want) <= 2e-2


def test_ensemble_pipeline_bitwise():
    """With the pipeline (request k's decimation and BBHnet on a second
    stream while request k + 1's DeepClean forwards run) every request's
    logits equal those of the sequential schedule bitwise."""
    n, W_dc, W_bb, s, K = 3, 4096, 2048, 256, 6
    dcm = [gs.DeepClean(torch.from_numpy(synth.deepclean_params(d)).to(DEV), synth.deepclean_layers())
           for d in range(2)]
    bbm = gs.BBHnet(torch.from_numpy(synth.bbhnet_params(0)).to(DEV), synth.bbhnet_stages())
    U = W_dc + K * s
    wit = torch.from_numpy(synth.gaussian(91, (2, n, 21, U))).to(DEV)
    st = torch.from_numpy(synth.gaussian(92, (2, n, U))).to(DEV)
    res = []
    for pipe in (False, True):
        ens = ensemble.Ensemble(dcm[0], dcm[1], bbm, n, W_dc=W_dc, W_bb=W_bb, stride=s, pipeline=pipe)
        ens.prefill(wit[..., :W_dc].contiguous())
        out = []
        for k in range(K):
            a, b = W_dc + k * s, W_dc + (k + 1) * s
            lg = ens.step(wit[..., a:b].contiguous(), st[..., a:b].contiguous())
            out.append(lg.clone() if not pipe else lg)
            if pipe and k % 2 == 1:        # read the two live buffers before they are reused
                torch.cuda.synchronize()
                out[-2], out[-1] = out[-2].clone(), out[-1].clone()
        torch.cuda.synchronize()
        res.append(torch.stack(out).cpu())
    assert torch.isfinite(res[0]).all()
    assert torch.equal(res[0], res[1])
