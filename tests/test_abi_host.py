"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every declared symbol, and its argument validation rejects bad input before
touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2108_12430_amd import gwstream as gs
from paper_2108_12430_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gwstream.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = gs.lib()
    names = declared_functions()
    assert "snapshot_update" in names and "deepclean_forward" in names and "bbhnet_forward" in names
    assert "deepclean_backward" in names
    for name in names:
        assert hasattr(L, name), name
    assert sorted(gs.EXPORTS) == names


def test_param_counts_match_generators():
    desc = gs.deepclean_desc(synth.deepclean_layers())
    assert gs.model_n_params(gs.MODEL_DEEPCLEAN, desc) == synth.deepclean_params(0).size
    tiny = gs.deepclean_desc(synth.tiny_layers())
    assert gs.model_n_params(gs.MODEL_DEEPCLEAN, tiny) == synth.deepclean_params(0, synth.tiny_layers()).size
    bd = gs.bbhnet_desc(synth.bbhnet_stages())
    assert gs.model_n_params(gs.MODEL_BBHNET, bd) == synth.bbhnet_params(0).size


def _rc(fn, *args):
    rc = fn(*args)
    return rc, gs.lib().gw_last_error().decode()


@pytest.mark.parametrize("mutate,code", [
    (lambda d: d.__setitem__(1 + 8 * 0 + 3, 9), gs.GW_EUNSUPPORTED),   # k = 9
    (lambda d: d.__setitem__(1 + 8 * 1 + 1, 7), gs.GW_EINVAL),         # channel chain broken
    (lambda d: d.__setitem__(1 + 8 * 8 + 7, 1), gs.GW_EINVAL),         # BN on the output layer
    (lambda d: d.__setitem__(1 + 8 * 2 + 4, 3), gs.GW_EUNSUPPORTED),   # stride 3
    (lambda d: d.__setitem__(1 + 8 * 2 + 5, 7), gs.GW_EINVAL),         # pad >= k
    (lambda d: d.__setitem__(0, 4), gs.GW_EINVAL),                     # length mismatch
])
def test_bad_descriptions_rejected(mutate, code):
    d = gs.deepclean_desc(synth.deepclean_layers())
    mutate(d)
    n = C.c_int64()
    rc, msg = _rc(gs.lib().gw_model_n_params, gs.MODEL_DEEPCLEAN, d.ctypes.data_as(C.c_void_p), len(d),
                  C.byref(n))
    assert rc == code and msg


def test_null_and_range_arguments_rejected():
    L = gs.lib()
    h = C.c_void_p()
    assert L.gw_pool_init(None, 1 << 20, 4, 4, C.byref(h)) == gs.GW_EINVAL
    assert L.gw_pool_init(C.c_void_p(256), 1 << 20, 0, 4, C.byref(h)) == gs.GW_EINVAL
    assert L.gw_pool_init(C.c_void_p(257), 1 << 20, 4, 4, C.byref(h)) == gs.GW_EINVAL   # misaligned
    assert L.snapshot_update(None, 1, None, None, None, None, None) == gs.GW_EINVAL
    assert L.deepclean_forward(None, None, None, None, 1, 4096, None, None, None, None, None, 0, 0, None, 0,
                               None) == gs.GW_EINVAL
    assert L.deepclean_update_forward(None, None, 1, None, None, None, None, 4096, None, None, None, None, 1, 0,
                                      None, 0, None) == gs.GW_EINVAL
    assert L.bbhnet_forward(None, None, None, None, 1, 2048, None, 0, None, 0, None) == gs.GW_EINVAL
    assert L.gw_model_set_cu_budget(None, 16) == gs.GW_EINVAL
    b = C.c_size_t()
    assert L.gw_bandpass_workspace(4, 32768, 4096.0, 70.0, 60.0, C.byref(b)) == gs.GW_EINVAL
    assert L.gw_bandpass_workspace(4, 32768, 4096.0, 55.0, 65.0, C.byref(b)) == gs.GW_OK
    assert b.value >= 4 * 81 * 2 * 4   # 81 bins (k = 440..520) x (cos, sin) per row


def test_packed_bytes_query():
    d = gs.deepclean_desc(synth.deepclean_layers())
    b = C.c_size_t()
    assert gs.lib().gw_model_packed_bytes(gs.MODEL_DEEPCLEAN, d.ctypes.data_as(C.c_void_p), len(d),
                                          C.byref(b)) == gs.GW_OK
    assert b.value > 0 and b.value % 256 == 0


@pytest.mark.parametrize("threads", [1, 3, 8, 16])
def test_host_copy_batch(threads):
    """gw_host_copy_batch copies every region exactly (sizes from 0 bytes to
    a few MB, so the batch is split across the pool's threads), and refuses
    bad arguments before copying anything."""
    rng = np.random.default_rng(threads)
    sizes = [0, 1, 3, 4096, 1 << 20, 12345, 3 << 20, 7] + list(rng.integers(0, 1 << 16, 40))
    src = [rng.integers(0, 255, int(n), dtype=np.uint8) for n in sizes]
    dst = [np.zeros(int(n), np.uint8) for n in sizes]
    addr = lambda a: a.__array_interface__["data"][0] if a.size else 0
    gs.host_copy_batch([addr(d) for d in dst], [addr(s) for s in src], [s.size for s in src], threads)
    assert all(np.array_equal(d, s) for d, s in zip(dst, src))
    keep = np.zeros(16, np.uint8)
    for d, s, n, t in (([addr(keep)], [0], [16], threads),       # null source with bytes > 0
                       ([addr(keep)], [addr(src[3])], [16], 0)):  # no threads
        with pytest.raises(gs.GwError):
            gs.host_copy_batch(d, s, n, t)
    assert not keep.any()
    gs.host_copy_batch([], [], [], threads)  # nothing to do


def test_host_copy_batch_concurrent_calls():
    """Calls from several threads at once (the interpreter lock is released
    during each call) are serialised inside the library: every copy lands."""
    import threading
    rng = np.random.default_rng(7)
    jobs = []
    for _ in range(4):
        src = [rng.integers(0, 255, int(n), dtype=np.uint8) for n in rng.integers(1 << 16, 1 << 20, 12)]
        jobs.append((src, [np.zeros_like(s) for s in src]))
    errors = []

    def work(src, dst):
        try:
            for _ in range(10):
                gs.host_copy_batch([d.ctypes.data for d in dst], [s.ctypes.data for s in src],
                                   [s.size for s in src], 8)
        except Exception as e:  # surfaced below
            errors.append(e)

    th = [threading.Thread(target=work, args=j) for j in jobs]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors
    assert all(np.array_equal(d, s) for src, dst in jobs for d, s in zip(dst, src))
