"""ctypes binding of libnrng.so (argument marshalling only).

Every function has the name and argument order of the C entry point in
include/nrng.h.  Buffer arguments accept a torch tensor on the GPU (its
data_ptr() is passed), an integer device address, or None for NULL.  The
stream argument accepts a torch.cuda.Stream, an integer hipStream_t, or None
for torch's current stream on the current device.  A non-zero status raises
NrngError.  There is no fallback: if the library is not built, the first
call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnrng.so")

NRNG_F64, NRNG_F32, NRNG_BF16, NRNG_F16 = 0, 1, 2, 3
NRNG_METHOD_B1, NRNG_METHOD_POLAR, NRNG_METHOD_P2, NRNG_METHOD_B3, NRNG_METHOD_R, NRNG_METHOD_B2 = 0, 1, 2, 3, 4, 5
NRNG_OK, NRNG_EINVAL, NRNG_EDTYPE, NRNG_ERANGE = 0, -1, -2, -3
NRNG_EHIP, NRNG_ENODEV, NRNG_ECAPTURE, NRNG_ENOMEM = -4, -5, -6, -7
KERNEL_B1, KERNEL_POLAR, KERNEL_B1_BATCHED = 0, 1, 2

_u64, _u32, _i32, _f64, _vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double, ctypes.c_void_p

_SIGS = {
    "nrng_strerror": (ctypes.c_char_p, [_i32]),
    "nrng_version": (_i32, []),
    "nrng_init": (_i32, []),
    "nrng_device_cus": (_i32, []),
    "nrng_reserve": (_i32, [_u64, _u32]),
    "nrng_boxmuller": (_i32, [_u64, _u64, _u64, _f64, _f64, _vp, _i32, _vp]),
    "nrng_b3": (_i32, [_u64, _u64, _u64, _f64, _f64, _vp, _i32, _vp]),
    "nrng_b2": (_i32, [_u64, _u64, _u64, _f64, _f64, _vp, _i32, _vp]),
    "nrng_polar": (_i32, [_u64, _u64, _u64, _f64, _f64, _vp, _i32, _vp, _vp]),
    "nrng_polar2": (_i32, [_u64, _u64, _u64, _f64, _f64, _vp, _i32, _vp, _vp]),
    "nrng_ratio": (_i32, [_u64, _u64, _u64, _f64, _f64, _vp, _i32, _vp, _vp]),
    "nrng_polar_dev": (_i32, [_u64, _vp, _u64, _f64, _f64, _vp, _i32, _vp]),
    "nrng_polar_noalloc": (_i32, [_u64, _u64, _u64, _f64, _f64, _vp, _i32, _vp, _vp]),
    "nrng_batched": (_i32, [_i32, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _u64, _i32, _vp, _vp]),
    "nrng_batched_plan": (_i32, [_i32, _u32, _vp, _vp, _u64, _i32, _vp, _vp]),
    "nrng_batched_exec": (_i32, [_i32, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp]),
    "nrng_batched_exec_part": (_i32, [_i32, _i32, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp]),
    "nrng_batched_exec_timed": (_i32, [_i32, _i32, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp,
                                       _vp]),
    "nrng_fillgraph_create": (_i32, [_u64, _vp, _u64, _f64, _f64, _vp, _i32, _vp, ctypes.POINTER(_vp)]),
    "nrng_fillgraph_launch": (_i32, [_vp, _vp]),
    "nrng_fillgraph_destroy": (_i32, [_vp]),
    "nrng_tune_set": (_i32, [_i32, _i32, _u32, _u32, _u32]),
    "nrng_tune_get": (_i32, [_i32, _i32, ctypes.POINTER(_u32), ctypes.POINTER(_u32), ctypes.POINTER(_u32)]),
    "nrng_tune_variants": (_i32, [_i32, ctypes.POINTER(_u32), _i32]),
    "nrng_test_b1_words": (_i32, [_vp, _u64, _f64, _f64, _vp, _i32, _vp]),
    "nrng_test_b3_words": (_i32, [_vp, _u64, _f64, _f64, _vp, _i32, _vp]),
    "nrng_test_b2_words": (_i32, [_vp, _u64, _f64, _f64, _vp, _i32, _vp]),
    "nrng_test_polar_xy": (_i32, [_vp, _u64, _f64, _f64, _vp, _i32, _vp, _vp, _vp]),
    "nrng_test_polar2_xy": (_i32, [_vp, _u64, _f64, _f64, _vp, _i32, _vp, _vp, _vp]),
    "nrng_test_ratio_words": (_i32, [_vp, _u64, _f64, _f64, _vp, _i32, _vp, _vp, _vp]),
    "nrng_ratio_trace": (_i32, [_u64, _u64, _u64, _vp, _vp, _vp]),
    "nrng_polar_trace": (_i32, [_u64, _u64, _u64, _vp, _vp, _vp]),
    "nrng_test_polar_budget": (_i32, [_u64, _u64, _u64, _f64, _f64, _vp, _i32, _u32, _vp, _vp]),
    "nrng_test_ratio_budget": (_i32, [_u64, _u64, _u64, _f64, _f64, _vp, _i32, _u32, _vp, _vp]),
    "nrng_probe_store": (_i32, [_vp, _u64, _vp]),
    "nrng_probe_copy": (_i32, [_vp, _vp, _u64, _vp]),
    "nrng_probe_store_variant": (_i32, [_vp, _u64, _i32, _u32, _u32, _vp]),
    "nrng_probe_hash": (_i32, [_u64, _u64, _vp, _u64, _vp]),
    "nrng_probe_valu": (_i32, [_i32, ctypes.c_uint32, _vp, _u64, _vp]),
    "nrng_tune_load": (_i32, [ctypes.c_char_p]),
}

_lock = threading.Lock()
_lib = None


class NrngError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__("%s failed: %s (%d)" % (fn, msg, status))
        self.status = status


def lib() -> ctypes.CDLL:
    """Load libnrng.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libnrng.so is not built (%s); run __graft_entry__.build() or "
                                   "python -m paper_1004_3105_amd.build" % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                f = getattr(L, name)
                f.restype, f.argtypes = res, args
            _lib = L
    return _lib


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        if not x.is_cuda:
            raise ValueError("device tensor expected")
        return x.data_ptr()
    raise TypeError("expected a tensor, an int address or None, got %r" % type(x))


_ESIZE = {NRNG_F64: 8, NRNG_F32: 4, NRNG_BF16: 2, NRNG_F16: 2}


def _need(t, nbytes: int, what: str) -> None:
    """When a buffer argument is a tensor, check that it holds nbytes bytes
    (raw addresses cannot be checked and are trusted)."""
    if t is None or isinstance(t, int) or not hasattr(t, "data_ptr"):
        return
    have = t.numel() * t.element_size()
    if not t.is_contiguous():
        raise ValueError("%s: contiguous tensor expected" % what)
    if have < nbytes:
        raise ValueError("%s: tensor holds %d bytes, the call writes or reads %d" % (what, have, nbytes))


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _check(fn: str, rc: int) -> int:
    if rc != NRNG_OK:
        raise NrngError(fn, rc, lib().nrng_strerror(rc).decode())
    return rc


def nrng_strerror(status: int) -> str:
    return lib().nrng_strerror(status).decode()


def nrng_version() -> int:
    return lib().nrng_version()


def nrng_init() -> None:
    _check("nrng_init", lib().nrng_init())


def nrng_device_cus() -> int:
    return lib().nrng_device_cus()


def nrng_reserve(max_n: int, max_streams: int = 0) -> None:
    _check("nrng_reserve", lib().nrng_reserve(max_n, max_streams))


def nrng_boxmuller(seed, offset, n, mu, sigma, out, dtype, stream=None) -> None:
    _need(out, n * _ESIZE.get(dtype, 0), "nrng_boxmuller out")
    _check("nrng_boxmuller", lib().nrng_boxmuller(seed & (2**64 - 1), offset & (2**64 - 1), n, mu, sigma,
                                                  _ptr(out), dtype, _stream(stream)))


def nrng_b3(seed, offset, n, mu, sigma, out, dtype, stream=None) -> None:
    _need(out, n * _ESIZE.get(dtype, 0), "nrng_b3 out")
    _check("nrng_b3", lib().nrng_b3(seed & (2**64 - 1), offset & (2**64 - 1), n, mu, sigma, _ptr(out), dtype,
                                    _stream(stream)))


def nrng_b2(seed, offset, n, mu, sigma, out, dtype, stream=None) -> None:
    _need(out, n * _ESIZE.get(dtype, 0), "nrng_b2 out")
    _check("nrng_b2", lib().nrng_b2(seed & (2**64 - 1), offset & (2**64 - 1), n, mu, sigma, _ptr(out), dtype,
                                    _stream(stream)))


def nrng_polar(seed, offset, n, mu, sigma, out, dtype, stream=None, d_consumed=None) -> None:
    _need(out, n * _ESIZE.get(dtype, 0), "nrng_polar out")
    _need(d_consumed, 8, "nrng_polar d_consumed")
    _check("nrng_polar", lib().nrng_polar(seed & (2**64 - 1), offset & (2**64 - 1), n, mu, sigma, _ptr(out),
                                          dtype, _stream(stream), _ptr(d_consumed)))


def nrng_polar_noalloc(seed, offset, n, mu, sigma, out, dtype, stream=None, d_consumed=None) -> None:
    _need(out, n * _ESIZE.get(dtype, 0), "nrng_polar_noalloc out")
    _need(d_consumed, 8, "nrng_polar_noalloc d_consumed")
    _check("nrng_polar_noalloc", lib().nrng_polar_noalloc(seed & (2**64 - 1), offset & (2**64 - 1), n, mu, sigma,
                                                          _ptr(out), dtype, _stream(stream), _ptr(d_consumed)))


def nrng_polar2(seed, offset, n, mu, sigma, out, dtype, stream=None, d_consumed=None) -> None:
    _need(out, n * _ESIZE.get(dtype, 0), "nrng_polar2 out")
    _need(d_consumed, 8, "nrng_polar2 d_consumed")
    _check("nrng_polar2", lib().nrng_polar2(seed & (2**64 - 1), offset & (2**64 - 1), n, mu, sigma, _ptr(out),
                                            dtype, _stream(stream), _ptr(d_consumed)))


def nrng_ratio(seed, offset, n, mu, sigma, out, dtype, stream=None, d_consumed=None) -> None:
    _need(out, n * _ESIZE.get(dtype, 0), "nrng_ratio out")
    _need(d_consumed, 8, "nrng_ratio d_consumed")
    _check("nrng_ratio", lib().nrng_ratio(seed & (2**64 - 1), offset & (2**64 - 1), n, mu, sigma, _ptr(out), dtype,
                                          _stream(stream), _ptr(d_consumed)))


def nrng_polar_dev(seed, d_cursor, n, mu, sigma, out, dtype, stream=None) -> None:
    _need(out, n * _ESIZE.get(dtype, 0), "nrng_polar_dev out")
    _need(d_cursor, 8, "nrng_polar_dev d_cursor")
    _check("nrng_polar_dev", lib().nrng_polar_dev(seed & (2**64 - 1), _ptr(d_cursor), n, mu, sigma, _ptr(out),
                                                  dtype, _stream(stream)))


def nrng_batched(method, nstreams, d_seed, d_offset, d_n, d_out_off, d_mu, d_sigma, out, out_len, dtype,
                 stream=None, d_consumed=None) -> None:
    _need(out, out_len * _ESIZE.get(dtype, 0), "nrng_batched out")
    for t, nm in ((d_seed, "d_seed"), (d_offset, "d_offset"), (d_n, "d_n"), (d_out_off, "d_out_off"),
                  (d_mu, "d_mu"), (d_sigma, "d_sigma"), (d_consumed, "d_consumed")):
        _need(t, 8 * nstreams, "nrng_batched " + nm)
    _check("nrng_batched", lib().nrng_batched(method, nstreams, _ptr(d_seed), _ptr(d_offset), _ptr(d_n),
                                              _ptr(d_out_off), _ptr(d_mu), _ptr(d_sigma), _ptr(out), out_len,
                                              dtype, _stream(stream), _ptr(d_consumed)))


def nrng_batched_plan(method, nstreams, d_n, d_out_off, out_len, dtype, stream=None, d_consumed=None) -> None:
    for t, nm in ((d_n, "d_n"), (d_out_off, "d_out_off"), (d_consumed, "d_consumed")):
        _need(t, 8 * nstreams, "nrng_batched_plan " + nm)
    _check("nrng_batched_plan", lib().nrng_batched_plan(method, nstreams, _ptr(d_n), _ptr(d_out_off), out_len,
                                                        dtype, _stream(stream), _ptr(d_consumed)))


def nrng_batched_exec(method, nstreams, d_seed, d_offset, d_n, d_out_off, d_mu, d_sigma, out, dtype, stream=None,
                      d_consumed=None) -> None:
    for t, nm in ((d_seed, "d_seed"), (d_offset, "d_offset"), (d_n, "d_n"), (d_out_off, "d_out_off"),
                  (d_mu, "d_mu"), (d_sigma, "d_sigma"), (d_consumed, "d_consumed")):
        _need(t, 8 * nstreams, "nrng_batched_exec " + nm)
    _check("nrng_batched_exec", lib().nrng_batched_exec(method, nstreams, _ptr(d_seed), _ptr(d_offset), _ptr(d_n),
                                                        _ptr(d_out_off), _ptr(d_mu), _ptr(d_sigma), _ptr(out),
                                                        dtype, _stream(stream), _ptr(d_consumed)))


def nrng_batched_exec_part(part, method, nstreams, d_seed, d_offset, d_n, d_out_off, d_mu, d_sigma, out, dtype,
                           stream=None, d_consumed=None) -> None:
    for t, nm in ((d_seed, "d_seed"), (d_offset, "d_offset"), (d_n, "d_n"), (d_out_off, "d_out_off"),
                  (d_mu, "d_mu"), (d_sigma, "d_sigma"), (d_consumed, "d_consumed")):
        _need(t, 8 * nstreams, "nrng_batched_exec_part " + nm)
    _check("nrng_batched_exec_part",
           lib().nrng_batched_exec_part(part, method, nstreams, _ptr(d_seed), _ptr(d_offset), _ptr(d_n),
                                        _ptr(d_out_off), _ptr(d_mu), _ptr(d_sigma), _ptr(out), dtype,
                                        _stream(stream), _ptr(d_consumed)))


def _event(e):
    """A hipEvent_t handle from a torch.cuda.Event (which must have been
    recorded once, so that torch has created it) or an int handle."""
    if isinstance(e, int):
        return e
    h = getattr(e, "cuda_event", 0)
    if not h:
        raise ValueError("event expected (a torch.cuda.Event recorded once, or a hipEvent_t handle)")
    return h


def nrng_batched_exec_timed(part, method, nstreams, d_seed, d_offset, d_n, d_out_off, d_mu, d_sigma, out, dtype,
                            stream, d_consumed, ev_start, ev_stop) -> None:
    for t, nm in ((d_seed, "d_seed"), (d_offset, "d_offset"), (d_n, "d_n"), (d_out_off, "d_out_off"),
                  (d_mu, "d_mu"), (d_sigma, "d_sigma"), (d_consumed, "d_consumed")):
        _need(t, 8 * nstreams, "nrng_batched_exec_timed " + nm)
    _check("nrng_batched_exec_timed",
           lib().nrng_batched_exec_timed(part, method, nstreams, _ptr(d_seed), _ptr(d_offset), _ptr(d_n),
                                         _ptr(d_out_off), _ptr(d_mu), _ptr(d_sigma), _ptr(out), dtype,
                                         _stream(stream), _ptr(d_consumed), _event(ev_start), _event(ev_stop)))


def nrng_fillgraph_create(seed, d_cursor, n, mu, sigma, out, dtype, stream) -> int:
    _need(out, n * _ESIZE.get(dtype, 0), "nrng_fillgraph_create out")
    _need(d_cursor, 8, "nrng_fillgraph_create d_cursor")
    h = _vp()
    _check("nrng_fillgraph_create", lib().nrng_fillgraph_create(seed & (2**64 - 1), _ptr(d_cursor), n, mu, sigma,
                                                                _ptr(out), dtype, _stream(stream),
                                                                ctypes.byref(h)))
    return h.value


def nrng_fillgraph_launch(graph: int, stream=None) -> None:
    _check("nrng_fillgraph_launch", lib().nrng_fillgraph_launch(graph, _stream(stream)))


def nrng_fillgraph_destroy(graph: int) -> None:
    _check("nrng_fillgraph_destroy", lib().nrng_fillgraph_destroy(graph))


def nrng_tune_set(kernel, dtype, wg, unroll, grid_per_cu=0) -> None:
    _check("nrng_tune_set", lib().nrng_tune_set(kernel, dtype, wg, unroll, grid_per_cu))


def nrng_tune_get(kernel, dtype):
    a, b, c = _u32(), _u32(), _u32()
    _check("nrng_tune_get", lib().nrng_tune_get(kernel, dtype, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def nrng_tune_variants(kernel):
    buf = (_u32 * 64)()
    nv = lib().nrng_tune_variants(kernel, buf, 32)
    if nv < 0:
        _check("nrng_tune_variants", nv)
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(nv)]


def nrng_test_b1_words(d_words, npairs, mu, sigma, out, dtype, stream=None) -> None:
    _need(d_words, 16 * npairs, "nrng_test_b1_words d_words")
    _need(out, 2 * npairs * _ESIZE.get(dtype, 0), "nrng_test_b1_words out")
    _check("nrng_test_b1_words", lib().nrng_test_b1_words(_ptr(d_words), npairs, mu, sigma, _ptr(out), dtype,
                                                          _stream(stream)))


def nrng_test_b3_words(d_words, npairs, mu, sigma, out, dtype, stream=None) -> None:
    _need(d_words, 24 * npairs, "nrng_test_b3_words d_words")
    _need(out, 2 * npairs * _ESIZE.get(dtype, 0), "nrng_test_b3_words out")
    _check("nrng_test_b3_words", lib().nrng_test_b3_words(_ptr(d_words), npairs, mu, sigma, _ptr(out), dtype,
                                                          _stream(stream)))


def nrng_test_b2_words(d_words, npairs, mu, sigma, out, dtype, stream=None) -> None:
    _need(d_words, 16 * npairs, "nrng_test_b2_words d_words")
    _need(out, 2 * npairs * _ESIZE.get(dtype, 0), "nrng_test_b2_words out")
    _check("nrng_test_b2_words", lib().nrng_test_b2_words(_ptr(d_words), npairs, mu, sigma, _ptr(out), dtype,
                                                          _stream(stream)))


def nrng_test_polar_xy(d_xy, ncand, mu, sigma, out, dtype, d_mask_words, d_count, stream=None) -> None:
    _need(d_xy, 8 * ncand, "nrng_test_polar_xy d_xy")
    _need(out, 2 * ncand * _ESIZE.get(dtype, 0), "nrng_test_polar_xy out")
    _need(d_mask_words, 8 * ((ncand + 63) // 64), "nrng_test_polar_xy d_mask_words")
    _need(d_count, 8, "nrng_test_polar_xy d_count")
    _check("nrng_test_polar_xy", lib().nrng_test_polar_xy(_ptr(d_xy), ncand, mu, sigma, _ptr(out), dtype,
                                                          _ptr(d_mask_words), _ptr(d_count), _stream(stream)))


def nrng_test_polar2_xy(d_xy, ncand, mu, sigma, out, dtype, d_mask_words, d_count, stream=None) -> None:
    _need(d_xy, 8 * ncand, "nrng_test_polar2_xy d_xy")
    _need(out, 2 * ncand * _ESIZE.get(dtype, 0), "nrng_test_polar2_xy out")
    _need(d_mask_words, 8 * ((ncand + 63) // 64), "nrng_test_polar2_xy d_mask_words")
    _need(d_count, 8, "nrng_test_polar2_xy d_count")
    _check("nrng_test_polar2_xy", lib().nrng_test_polar2_xy(_ptr(d_xy), ncand, mu, sigma, _ptr(out), dtype,
                                                            _ptr(d_mask_words), _ptr(d_count), _stream(stream)))


def nrng_test_ratio_words(d_words, ncand, mu, sigma, out, dtype, d_mask_words, d_count, stream=None) -> None:
    _need(d_words, 16 * ncand, "nrng_test_ratio_words d_words")
    _need(out, ncand * _ESIZE.get(dtype, 0), "nrng_test_ratio_words out")
    _need(d_mask_words, 8 * ((ncand + 63) // 64), "nrng_test_ratio_words d_mask_words")
    _need(d_count, 8, "nrng_test_ratio_words d_count")
    _check("nrng_test_ratio_words", lib().nrng_test_ratio_words(_ptr(d_words), ncand, mu, sigma, _ptr(out), dtype,
                                                                _ptr(d_mask_words), _ptr(d_count), _stream(stream)))


def nrng_ratio_trace(seed, offset, ncand, d_mask_words, d_word_prefix, stream=None) -> None:
    _need(d_mask_words, 8 * ((ncand + 63) // 64), "nrng_ratio_trace d_mask_words")
    _need(d_word_prefix, 8 * ((ncand + 63) // 64), "nrng_ratio_trace d_word_prefix")
    _check("nrng_ratio_trace", lib().nrng_ratio_trace(seed & (2**64 - 1), offset & (2**64 - 1), ncand,
                                                      _ptr(d_mask_words), _ptr(d_word_prefix), _stream(stream)))


def nrng_polar_trace(seed, offset, ncand, d_mask_words, d_word_prefix, stream=None) -> None:
    _need(d_mask_words, 8 * ((ncand + 63) // 64), "nrng_polar_trace d_mask_words")
    _need(d_word_prefix, 8 * ((ncand + 63) // 64), "nrng_polar_trace d_word_prefix")
    _check("nrng_polar_trace", lib().nrng_polar_trace(seed & (2**64 - 1), offset & (2**64 - 1), ncand,
                                                      _ptr(d_mask_words), _ptr(d_word_prefix), _stream(stream)))


def nrng_test_polar_budget(seed, offset, n, mu, sigma, out, dtype, words, stream=None, d_consumed=None) -> None:
    _need(out, n * _ESIZE.get(dtype, 0), "nrng_test_polar_budget out")
    _need(d_consumed, 8, "nrng_test_polar_budget d_consumed")
    _check("nrng_test_polar_budget", lib().nrng_test_polar_budget(seed & (2**64 - 1), offset & (2**64 - 1), n, mu,
                                                                  sigma, _ptr(out), dtype, words, _stream(stream),
                                                                  _ptr(d_consumed)))


def nrng_test_ratio_budget(seed, offset, n, mu, sigma, out, dtype, words, stream=None, d_consumed=None) -> None:
    _need(out, n * _ESIZE.get(dtype, 0), "nrng_test_ratio_budget out")
    _need(d_consumed, 8, "nrng_test_ratio_budget d_consumed")
    _check("nrng_test_ratio_budget", lib().nrng_test_ratio_budget(seed & (2**64 - 1), offset & (2**64 - 1), n, mu,
                                                                  sigma, _ptr(out), dtype, words, _stream(stream),
                                                                  _ptr(d_consumed)))


def nrng_probe_store(out, nbytes, stream=None) -> None:
    _need(out, nbytes, "nrng_probe_store out")
    _check("nrng_probe_store", lib().nrng_probe_store(_ptr(out), nbytes, _stream(stream)))


def nrng_probe_store_variant(out, nbytes, nontemporal, blocks_per_cu, unroll, stream=None) -> None:
    _need(out, nbytes, "nrng_probe_store_variant out")
    _check("nrng_probe_store_variant", lib().nrng_probe_store_variant(_ptr(out), nbytes, int(nontemporal),
                                                                      blocks_per_cu, unroll, _stream(stream)))


def nrng_probe_copy(dst, src, nbytes, stream=None) -> None:
    _need(dst, nbytes, "nrng_probe_copy dst")
    _need(src, nbytes, "nrng_probe_copy src")
    _check("nrng_probe_copy", lib().nrng_probe_copy(_ptr(dst), _ptr(src), nbytes, _stream(stream)))


def nrng_probe_hash(seed, nhash, d_sink, sink_len, stream=None) -> None:
    _need(d_sink, 8 * sink_len, "nrng_probe_hash d_sink")
    _check("nrng_probe_hash", lib().nrng_probe_hash(seed & (2**64 - 1), nhash, _ptr(d_sink), sink_len,
                                                    _stream(stream)))



def nrng_tune_load(path: str) -> None:
    _check("nrng_tune_load", lib().nrng_tune_load(os.fsencode(path)))


VALU_PROBE_OPS = ["v_add_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_mul_u32_u24", "v_fma_f32", "v_cvt_f32_u32",
                  "v_log_f32", "v_sin_f32", "v_sqrt_f32", "v_rcp_f32", "v_lshrrev_b64", "v_lshl_add_u64",
                  "v_mad_u64_u32", "v_mad_i64_i32", "v_fma_f64"]


def nrng_probe_valu(op, iters, d_sink, sink_len, stream=None) -> None:
    _need(d_sink, 4 * sink_len, "nrng_probe_valu d_sink")
    _check("nrng_probe_valu", lib().nrng_probe_valu(op, iters, _ptr(d_sink), sink_len, _stream(stream)))


EXPORTED = sorted(_SIGS)
