"""Thin Python binding of libgwstream.so (ctypes).

Argument marshalling only: every step of the streaming path runs in the HIP
kernels behind the C ABI.  PyTorch provides device memory (tensors passed by
pointer) and the HIP stream the work is enqueued on.  The library must be
built (``python -m paper_2108_12430_amd.build``); importing this module on a
machine where it is missing raises immediately - there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgwstream.so")

GW_OK, GW_EINVAL, GW_ENOMEM, GW_ESTATE, GW_EHIP, GW_EUNSUPPORTED = range(6)
FP32, BF16, FP16 = 0, 1, 2
MODEL_DEEPCLEAN, MODEL_BBHNET = 1, 2
TRAIN, RECOMPUTE, CAUSAL, LAYERWISE, CACHE_FULL = 1, 2, 4, 8, 16
_CODES = {1: "GW_EINVAL", 2: "GW_ENOMEM", 3: "GW_ESTATE", 4: "GW_EHIP", 5: "GW_EUNSUPPORTED"}

EXPORTS = [
    "gw_last_error", "gw_pool_init", "gw_pool_free", "gw_stream_open", "gw_stream_close",
    "gw_stream_info", "gw_stream_window", "gw_stream_load", "gw_pool_usage", "snapshot_update", "gw_model_packed_bytes",
    "gw_model_create", "gw_model_refresh", "gw_model_free", "gw_model_set_cu_budget", "gw_model_n_params",
    "gw_model_set_layerwise",
    "deepclean_workspace", "deepclean_forward", "deepclean_update_forward", "deepclean_overlap_average", "gw_decimate2",
    "deepclean_cache_bytes", "gw_stream_attach_cache", "deepclean_cache_bands", "deepclean_forward_cached",
    "deepclean_backward_scratch",
    "deepclean_backward",
    "gw_bandpass_workspace", "gw_bandpass_mse", "gw_bandpass_mse_noalloc", "bbhnet_workspace", "bbhnet_forward",
    "gw_host_copy_batch", "gw_profile_begin", "gw_profile_end",
]


class GwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load the shared library once (torch is imported first so that the
    process has a single HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2108_12430_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz, u32, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_uint32, C.c_float
        P = C.POINTER
        sig = {
            "gw_last_error": ([], C.c_char_p),
            "gw_pool_init": ([vp, sz, i32, i32, P(vp)], C.c_int),
            "gw_pool_free": ([vp], C.c_int),
            "gw_stream_open": ([vp, i32, i32, vp, P(i32)], C.c_int),
            "gw_stream_close": ([vp, i32], C.c_int),
            "gw_stream_info": ([vp, i32, P(i32), P(i32), P(i64)], C.c_int),
            "gw_pool_usage": ([vp, P(sz), P(sz)], C.c_int),
            "gw_stream_window": ([vp, i32, vp, vp, vp], C.c_int),
            "gw_stream_load": ([vp, i32, vp, i64, vp], C.c_int),
            "snapshot_update": ([vp, i32, vp, vp, vp, vp, vp], C.c_int),
            "gw_model_packed_bytes": ([i32, vp, i32, P(sz)], C.c_int),
            "gw_model_create": ([i32, vp, i32, vp, i64, vp, sz, vp, P(vp)], C.c_int),
            "gw_model_refresh": ([vp, vp], C.c_int),
            "gw_model_free": ([vp], C.c_int),
            "gw_model_set_cu_budget": ([vp, i32], C.c_int),
            "gw_model_set_layerwise": ([vp, i32], C.c_int),
            "gw_model_n_params": ([i32, vp, i32, P(i64)], C.c_int),
            "deepclean_workspace": ([vp, i32, i32, i32, u32, P(sz)], C.c_int),
            "deepclean_forward": ([vp, vp, vp, vp, i32, i32, vp, vp, vp, vp, vp, i32, u32, vp, sz, vp], C.c_int),
            "deepclean_update_forward": ([vp, vp, i32, vp, vp, vp, vp, i32, vp, vp, vp, vp, i32, u32, vp, sz, vp],
                                         C.c_int),
            "deepclean_overlap_average": ([vp, i32, i32, vp, i32, vp, vp, vp, vp, vp, vp, vp], C.c_int),
            "gw_decimate2": ([i32, i32, i32, i32, vp, vp, vp, vp, vp], C.c_int),
            "deepclean_cache_bytes": ([vp, i32, P(sz)], C.c_int),
            "gw_stream_attach_cache": ([vp, i32, vp, sz], C.c_int),
            "deepclean_cache_bands": ([vp, i32, i32, i32, vp, vp], C.c_int),
            "deepclean_forward_cached": ([vp, vp, vp, i32, i32, vp, vp, vp, vp, vp, u32, vp], C.c_int),
            "deepclean_backward_scratch": ([vp, i32, i32, u32, P(sz)], C.c_int),
            "deepclean_backward": ([vp, i32, i32, vp, vp, vp, vp, u32, i32, vp, sz, vp], C.c_int),
            "gw_bandpass_workspace": ([i32, i32, f32, f32, f32, P(sz)], C.c_int),
            "gw_bandpass_mse": ([i32, i32, f32, f32, f32, vp, vp, vp, vp, vp, sz, vp], C.c_int),
            "gw_bandpass_mse_noalloc": ([i32, i32, f32, f32, f32, vp, vp, vp, vp, vp], C.c_int),
            "bbhnet_workspace": ([vp, i32, i32, i32, P(sz)], C.c_int),
            "bbhnet_forward": ([vp, vp, vp, vp, i32, i32, vp, i32, vp, sz, vp], C.c_int),
            "gw_host_copy_batch": ([vp, vp, vp, i32, i32], C.c_int),
            "gw_profile_begin": ([], C.c_int),
            "gw_profile_end": ([C.c_char_p, sz], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(rc):
    if rc != GW_OK:
        raise GwError(rc, lib().gw_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _host_i32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return a, a.ctypes.data_as(C.c_void_p)


def _host_i64(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    return a, a.ctypes.data_as(C.c_void_p)


def _f32(t, name):
    if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError(f"{name} must be a contiguous float32 device tensor")
    return t


def _buffer(nbytes, device):
    # 256-byte aligned device buffer (torch's caching allocator aligns to 512)
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------------------
# Descriptions
# ---------------------------------------------------------------------------

def deepclean_desc(layers):
    """int32 description from (type, C_in, C_out, k, stride, pad, out_pad, bn) tuples."""
    d = [len(layers)]
    for (typ, ci, co, k, s, p, op, bn) in layers:
        d += [0 if typ == "conv" else 1, ci, co, k, s, p, op, 1 if bn else 0]
    return np.array(d, dtype=np.int32)


def bbhnet_desc(stages):
    return np.array([len(stages), stages[0][0]] + [co for _, co in stages], dtype=np.int32)


# ---------------------------------------------------------------------------
# Pool of snapshot rings
# ---------------------------------------------------------------------------

class Pool:
    """Device-resident snapshot rings for many concurrent streams (App. B.1)."""

    def __init__(self, arena_bytes, max_slots=1024, max_items=1024, device="cuda:0"):
        self.device = torch.device(device)
        self.arena = _buffer(arena_bytes, self.device)
        h = C.c_void_p()
        check(lib().gw_pool_init(_ptr(self.arena), self.arena.numel(), max_slots, max_items, C.byref(h)))
        self.h = h

    def open(self, C_, W, stream=None):
        s = C.c_int32()
        check(lib().gw_stream_open(self.h, C_, W, _stream(stream), C.byref(s)))
        return s.value

    def try_open(self, C_, W, stream=None):
        """Slot id, or None when the pool refuses with GW_ENOMEM."""
        s = C.c_int32()
        rc = lib().gw_stream_open(self.h, C_, W, _stream(stream), C.byref(s))
        if rc == GW_ENOMEM:
            return None
        check(rc)
        return s.value

    def close(self, slot):
        check(lib().gw_stream_close(self.h, slot))

    def info(self, slot):
        c, w, n = C.c_int32(), C.c_int32(), C.c_int64()
        check(lib().gw_stream_info(self.h, slot, C.byref(c), C.byref(w), C.byref(n)))
        return c.value, w.value, n.value

    def window(self, slot, bf16=False, stream=None):
        """Current snapshot of a slot as a [C][W] float32 tensor (or the bf16
        shadow's bit patterns as int16 when bf16=True)."""
        c, w, _ = self.info(slot)
        if bf16:
            out = torch.empty((c, w), dtype=torch.int16, device=self.device)
            check(lib().gw_stream_window(self.h, slot, None, _ptr(out), _stream(stream)))
        else:
            out = torch.empty((c, w), dtype=torch.float32, device=self.device)
            check(lib().gw_stream_window(self.h, slot, _ptr(out), None, _stream(stream)))
        return out

    def load(self, slot, window, n_seen, stream=None):
        """gw_stream_load: restore a slot from an exported [C][W] float32
        device window (oldest sample first, as window() returns it) and the
        source's received-sample count."""
        _f32(window, "window")
        c, w, _ = self.info(slot)
        if tuple(window.shape) != (c, w):
            raise ValueError(f"window must be [{c}][{w}]")
        check(lib().gw_stream_load(self.h, slot, _ptr(window), int(n_seen), _stream(stream)))

    def attach_cache(self, slot, cache):
        """gw_stream_attach_cache: a uint8 device tensor (or None to detach)
        holding the slot's activation cache; it must outlive its use."""
        if cache is None:
            check(lib().gw_stream_attach_cache(self.h, slot, None, 0))
        else:
            if cache.dtype != torch.uint8 or not cache.is_cuda or not cache.is_contiguous():
                raise ValueError("cache must be a contiguous uint8 device tensor")
            check(lib().gw_stream_attach_cache(self.h, slot, _ptr(cache), cache.numel()))

    def usage(self):
        u, f = C.c_size_t(), C.c_size_t()
        check(lib().gw_pool_usage(self.h, C.byref(u), C.byref(f)))
        return u.value, f.value

    def update(self, slots, strides, samples, offsets, stream=None):
        """snapshot_update: samples is a packed float32 device tensor."""
        _f32(samples, "samples")
        sl, psl = _host_i32(slots)
        st, pst = _host_i32(strides)
        of, pof = _host_i64(offsets)
        check(lib().snapshot_update(self.h, len(sl), psl, pst, _ptr(samples), pof, _stream(stream)))

    def free(self):
        if self.h is not None:
            check(lib().gw_pool_free(self.h))
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Models
# ---------------------------------------------------------------------------

class _Model:
    kind = 0

    def __init__(self, params, desc, stream=None):
        self.params = _f32(params, "params")
        self.desc = np.ascontiguousarray(desc, dtype=np.int32)
        self.device = params.device
        nb = C.c_size_t()
        check(lib().gw_model_packed_bytes(self.kind, self.desc.ctypes.data_as(C.c_void_p), len(self.desc),
                                          C.byref(nb)))
        self.packed = _buffer(nb.value, self.device)
        h = C.c_void_p()
        check(lib().gw_model_create(self.kind, self.desc.ctypes.data_as(C.c_void_p), len(self.desc),
                                    _ptr(self.params), self.params.numel(), _ptr(self.packed),
                                    self.packed.numel(), _stream(stream), C.byref(h)))
        self.h = h

    def refresh(self, stream=None):
        check(lib().gw_model_refresh(self.h, _stream(stream)))

    def set_cu_budget(self, ncu):
        """Size the model's persistent kernels for at most ncu compute units
        (0: all), leaving the rest to kernels on other streams."""
        check(lib().gw_model_set_cu_budget(self.h, int(ncu)))

    def set_layerwise(self, on):
        """BBHnet: per-layer kernels (True) or the fused network kernel (False,
        the default for the reference shape)."""
        check(lib().gw_model_set_layerwise(self.h, 1 if on else 0))

    def free(self):
        if getattr(self, "h", None) is not None:
            check(lib().gw_model_free(self.h))
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def cache_bands(layers, W, shift):
    """deepclean_cache_bands for a layer list: [(zl, zr)] per layer, the dirty
    positions [0, zl) and [zr, L) after the window advanced by shift samples
    (-1: everything).  Needs no GPU."""
    d = deepclean_desc(layers)
    zl = np.zeros(len(layers), np.int32)
    zr = np.zeros(len(layers), np.int32)
    check(lib().deepclean_cache_bands(d.ctypes.data_as(C.c_void_p), len(d), W, shift, zl.ctypes.data_as(C.c_void_p),
                                      zr.ctypes.data_as(C.c_void_p)))
    return list(zip(zl.tolist(), zr.tolist()))


def model_n_params(kind, desc):
    d = np.ascontiguousarray(desc, dtype=np.int32)
    n = C.c_int64()
    check(lib().gw_model_n_params(kind, d.ctypes.data_as(C.c_void_p), len(d), C.byref(n)))
    return n.value


class DeepClean(_Model):
    kind = MODEL_DEEPCLEAN

    def __init__(self, params, layers, stream=None):
        self.layers = list(layers)
        super().__init__(params, deepclean_desc(self.layers), stream)
        self.c_in = self.layers[0][1]

    def workspace_bytes(self, n, W, precision=FP32, flags=0):
        b = C.c_size_t()
        check(lib().deepclean_workspace(self.h, n, W, precision, flags, C.byref(b)))
        return b.value

    def cache_bytes(self, W):
        """deepclean_cache_bytes: one stream's activation cache."""
        b = C.c_size_t()
        check(lib().deepclean_cache_bytes(self.h, W, C.byref(b)))
        return b.value

    def new_cache(self, W):
        """A device buffer of cache_bytes(W) bytes (256-byte aligned)."""
        return _buffer(self.cache_bytes(W), self.device)

    def cache_bands(self, W, shift):
        """deepclean_cache_bands: [(zl, zr)] per layer (host query)."""
        return cache_bands(self.layers, W, shift)

    def forward_cached(self, *, pool, slots, W, strides=None, strain=None, noise=None, clean=None, delays=None,
                       full=False, stream=None):
        """Enqueue deepclean_forward_cached (every slot needs an attached
        cache); outputs are caller-provided tensors or None."""
        sl, psl = _host_i32(slots)
        st = pst = dl = pdl = None
        if strides is not None:
            st, pst = _host_i32(strides)
        if delays is not None:
            dl, pdl = _host_i32(delays)
        for t, nm in ((strain, "strain"), (noise, "noise"), (clean, "clean")):
            if t is not None:
                _f32(t, nm)
        check(lib().deepclean_forward_cached(self.h, pool.h, psl, len(sl), W, pst, pdl, _ptr(strain), _ptr(noise),
                                             _ptr(clean), CACHE_FULL if full else 0, _stream(stream)))

    def forward(self, *, x=None, pool=None, slots=None, n=None, W=None, strides=None, strain=None,
                noise=None, clean=None, precision=FP32, flags=0, ws=None, stream=None, delays=None):
        """Enqueue deepclean_forward; outputs are caller-provided tensors (or
        None).  Returns the workspace used (holds the saved state for
        backward when flags has TRAIN)."""
        if x is not None:
            _f32(x, "x")
            n = x.shape[0] if n is None else n
            W = x.shape[-1] if W is None else W
        else:
            n = len(slots) if n is None else n
        if ws is None:
            ws = _buffer(self.workspace_bytes(n, W, precision, flags), self.device)
        sl = psl = st = pst = None
        if slots is not None:
            sl, psl = _host_i32(slots)
        if strides is not None:
            st, pst = _host_i32(strides)
        dl = pdl = None
        if delays is not None:
            dl, pdl = _host_i32(delays)
        check(lib().deepclean_forward(self.h, pool.h if pool is not None else None, psl, _ptr(x), n, W, pst, pdl,
                                      _ptr(strain), _ptr(noise), _ptr(clean), precision, flags, _ptr(ws),
                                      ws.numel(), _stream(stream)))
        return ws

    def update_forward(self, *, pool, slots, strides, samples, offsets, W, strain=None, clean=None, noise=None,
                       precision=FP32, flags=0, ws=None, stream=None, delays=None):
        """Enqueue deepclean_update_forward: pool.update(slots, strides,
        samples, offsets) then forward(pool=pool, slots=slots, ...) with the
        same strides, in one launch on the fused BF16 inference path."""
        _f32(samples, "samples")
        n = len(slots)
        if ws is None:
            ws = _buffer(self.workspace_bytes(n, W, precision, flags), self.device)
        sl, psl = _host_i32(slots)
        st, pst = _host_i32(strides)
        of, pof = _host_i64(offsets)
        dl = pdl = None
        if delays is not None:
            dl, pdl = _host_i32(delays)
        check(lib().deepclean_update_forward(self.h, pool.h, n, psl, pst, _ptr(samples), pof, W, pdl, _ptr(strain),
                                             _ptr(noise), _ptr(clean), precision, flags, _ptr(ws), ws.numel(),
                                             _stream(stream)))
        return ws

    @staticmethod
    def overlap_state_floats(strides, depth):
        """Floats of the caller-owned state overlap_average needs."""
        return int(depth) * int(np.sum(np.asarray(strides, np.int64)))

    def overlap_average(self, *, noise, strides, depth, counts, state, strain=None, clean=None, avg=None,
                        stream=None):
        """Enqueue deepclean_overlap_average for n = noise.shape[0] items."""
        _f32(noise, "noise")
        _f32(state, "state")
        n, W = noise.shape
        st, pst = _host_i32(strides)
        cn = np.ascontiguousarray(counts, dtype=np.int64)
        check(lib().deepclean_overlap_average(self.h, n, W, pst, int(depth), cn.ctypes.data_as(C.c_void_p),
                                              _ptr(noise), _ptr(state), _ptr(strain), _ptr(clean), _ptr(avg),
                                              _stream(stream)))

    def backward_scratch_bytes(self, n, W, flags):
        b = C.c_size_t()
        check(lib().deepclean_backward_scratch(self.h, n, W, flags, C.byref(b)))
        return b.value

    def backward(self, x, dnoise, saved, dparams, flags=TRAIN, precision=FP32, scratch=None, stream=None):
        n, W = x.shape[0], x.shape[-1]
        if scratch is None:
            scratch = _buffer(self.backward_scratch_bytes(n, W, flags), self.device)
        check(lib().deepclean_backward(self.h, n, W, _ptr(_f32(x, "x")), _ptr(_f32(dnoise, "dnoise")),
                                       _ptr(saved), _ptr(_f32(dparams, "dparams")), flags, precision,
                                       _ptr(scratch), scratch.numel(), _stream(stream)))
        return dparams


class BBHnet(_Model):
    kind = MODEL_BBHNET

    def __init__(self, params, stages, stream=None):
        self.stages = list(stages)
        super().__init__(params, bbhnet_desc(self.stages), stream)
        self.c_in = self.stages[0][0]

    def workspace_bytes(self, n, W, precision=FP32):
        b = C.c_size_t()
        check(lib().bbhnet_workspace(self.h, n, W, precision, C.byref(b)))
        return b.value

    def forward(self, *, x=None, pool=None, slots=None, n=None, W=None, logits=None, precision=FP32, ws=None,
                stream=None):
        if x is not None:
            _f32(x, "x")
            n = x.shape[0] if n is None else n
            W = x.shape[-1] if W is None else W
        else:
            n = len(slots) if n is None else n
        if logits is None:
            logits = torch.empty(n, dtype=torch.float32, device=self.device)
        if ws is None:
            ws = _buffer(self.workspace_bytes(n, W, precision), self.device)
        sl = psl = None
        if slots is not None:
            sl, psl = _host_i32(slots)
        check(lib().bbhnet_forward(self.h, pool.h if pool is not None else None, psl, _ptr(x), n, W,
                                   _ptr(logits), precision, _ptr(ws), ws.numel(), _stream(stream)))
        return logits


def bandpass_mse(strain, noise, fs=4096.0, f_lo=55.0, f_hi=65.0, want_grad=True, stream=None):
    """gw_bandpass_mse: returns (loss [1] tensor, dnoise or None)."""
    n, W = strain.shape
    b = C.c_size_t()
    check(lib().gw_bandpass_workspace(n, W, fs, f_lo, f_hi, C.byref(b)))
    ws = _buffer(b.value, strain.device)
    loss = torch.empty(1, dtype=torch.float32, device=strain.device)
    dn = torch.empty_like(strain) if want_grad else None
    check(lib().gw_bandpass_mse(n, W, fs, f_lo, f_hi, _ptr(_f32(strain, "strain")), _ptr(_f32(noise, "noise")),
                                _ptr(loss), _ptr(dn), _ptr(ws), ws.numel(), _stream(stream)))
    return loss, dn


def bandpass_mse_noalloc(strain, noise, loss, dnoise=None, fs=4096.0, f_lo=55.0, f_hi=65.0, stream=None):
    """gw_bandpass_mse_noalloc: writes the loss into `loss` ([1] float32) and
    the gradient into `dnoise` (or skips it when None); allocates nothing."""
    n, W = strain.shape
    check(lib().gw_bandpass_mse_noalloc(n, W, fs, f_lo, f_hi, _ptr(_f32(strain, "strain")),
                                        _ptr(_f32(noise, "noise")), _ptr(_f32(loss, "loss")),
                                        _ptr(None if dnoise is None else _f32(dnoise, "dnoise")), _stream(stream)))


def decimate2(*, x, taps, hist, y, stream=None):
    """Enqueue gw_decimate2.  x [C][n][s], hist [n][C][ntaps - 1] (state),
    y [n][C][s / 2]; all float32 device tensors."""
    for t, nm in ((x, "x"), (taps, "taps"), (hist, "hist"), (y, "y")):
        _f32(t, nm)
    C_, n, s = x.shape
    check(lib().gw_decimate2(n, C_, s, taps.numel(), _ptr(taps), _ptr(x), _ptr(hist), _ptr(y), _stream(stream)))


def host_copy_batch(dst, src, nbytes, threads=8):
    """gw_host_copy_batch: dst[i] <- src[i] (nbytes[i] bytes) for host
    addresses given as integer sequences or uintp arrays, spread over up to
    `threads` host threads; returns when every copy is complete.  The call
    releases the interpreter lock."""
    d = np.ascontiguousarray(dst, dtype=np.uintp)
    s = np.ascontiguousarray(src, dtype=np.uintp)
    b = np.ascontiguousarray(nbytes, dtype=np.uintp)
    if not (d.shape == s.shape == b.shape) or d.ndim != 1:
        raise ValueError("dst, src and nbytes must be 1-D of one length")
    check(lib().gw_host_copy_batch(d.ctypes.data, s.ctypes.data, b.ctypes.data, int(d.size), int(threads)))


def profile_begin():
    """Start recording per-launch HIP-event timings inside the library."""
    check(lib().gw_profile_begin())


def profile_end():
    """Stop recording; returns {launch name: (count, total_ms)}."""
    buf = C.create_string_buffer(1 << 16)
    check(lib().gw_profile_end(buf, len(buf)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out
