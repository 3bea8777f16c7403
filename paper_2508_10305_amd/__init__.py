"""MI355X-native GPZ particle compressor (arXiv 2508.10305).

Python binding of ``libgpz.so`` (C ABI in ``include/gpz.h``).  It only
marshals arguments: torch supplies device memory and the current HIP stream,
and every step of compression and decompression runs in the library's gfx950
kernels.  There is no CPU fallback: if the library is missing, every call
raises ``GpzLibraryMissing``.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libgpz.so")

GPZ_OK, GPZ_EINVAL, GPZ_ENOSPC, GPZ_ECORRUPT, GPZ_EDEVICE, GPZ_ENOMEM, GPZ_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6)

EXPORTS = (
    "gpz_default_params", "gpz_max_compressed_bytes", "gpz_compress_workspace_bytes",
    "gpz_decompress_workspace_bytes", "gpz_compress", "gpz_compress_async", "gpz_decompress",
    "gpz_decompress_async", "gpz_compress_f64", "gpz_max_compressed_bytes_f64",
    "gpz_compress_workspace_bytes_f64", "gpz_decompress_f64", "gpz_stats_workspace_bytes", "gpz_bound_check", "gpz_error_stats",
    "gpz_stream_stats", "gpz_field_range", "gpz_field_range_noalloc", "gpz_field_range_async", "gpz_rel_to_abs", "gpz_inspect",
    "gpz_set_timing", "gpz_set_timing_kinds", "gpz_timing_collect", "gpz_strerror",
    "gpz_default_batch_config",
    "gpz_batch_workspace_bytes", "gpz_batch_create", "gpz_batch_rebind", "gpz_batch_compress",
    "gpz_batch_decompress", "gpz_batch_sizes", "gpz_batch_errors", "gpz_batch_destroy",
)


class GpzLibraryMissing(RuntimeError):
    pass


class GpzError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = _lib().gpz_strerror(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_uint32), ("seg_bits", ctypes.c_uint32),
                ("key_fields", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class Job(ctypes.Structure):
    _fields_ = [("fields", ctypes.c_void_p), ("n", ctypes.c_uint64), ("nfields", ctypes.c_uint32),
                ("eb", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("out_capacity", ctypes.c_uint64), ("dec_fields", ctypes.c_void_p),
                ("ws", ctypes.c_void_p)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_uint32), ("tile", ctypes.c_uint32),
                ("use_graph", ctypes.c_uint32), ("max_jobs", ctypes.c_uint32),
                ("max_blocks", ctypes.c_uint64)]


class FieldError(ctypes.Structure):
    _fields_ = [("violations", ctypes.c_uint64), ("max_abs_err", ctypes.c_double),
                ("sum_sq_err", ctypes.c_double), ("nrmse", ctypes.c_double),
                ("min", ctypes.c_float), ("max", ctypes.c_float)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("nfields", ctypes.c_uint32),
                ("block_size", ctypes.c_uint32), ("seg_bits", ctypes.c_uint32),
                ("key_fields", ctypes.c_uint32), ("nblocks", ctypes.c_uint64),
                ("flags", ctypes.c_uint32)]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise GpzLibraryMissing(
                f"{LIB_PATH} not built; run paper_2508_10305_amd/build.py (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
        pp = ctypes.POINTER(Params)
        L.gpz_default_params.argtypes = [pp, u32]
        L.gpz_default_params.restype = None
        L.gpz_max_compressed_bytes.argtypes = [u64, u32, pp]
        L.gpz_max_compressed_bytes.restype = u64
        L.gpz_compress_workspace_bytes.argtypes = [u64, u32, pp]
        L.gpz_compress_workspace_bytes.restype = u64
        L.gpz_decompress_workspace_bytes.argtypes = []
        L.gpz_decompress_workspace_bytes.restype = u64
        L.gpz_compress.argtypes = [vp, u64, u32, vp, pp, vp, u64, ctypes.POINTER(u64), vp, vp, u64,
                                   vp]
        L.gpz_compress.restype = ctypes.c_int
        L.gpz_compress_async.argtypes = [vp, u64, u32, vp, pp, vp, u64, vp, vp, vp, u64, vp]
        L.gpz_compress_async.restype = ctypes.c_int
        L.gpz_decompress.argtypes = [vp, u64, vp, u64, u32, vp, u64, vp]
        L.gpz_decompress.restype = ctypes.c_int
        L.gpz_decompress_async.argtypes = [vp, u64, vp, u64, u32, pp, vp, vp]
        L.gpz_decompress_async.restype = ctypes.c_int
        L.gpz_compress_f64.argtypes = L.gpz_compress.argtypes
        L.gpz_compress_f64.restype = ctypes.c_int
        L.gpz_max_compressed_bytes_f64.argtypes = [u64, u32, pp]
        L.gpz_max_compressed_bytes_f64.restype = u64
        L.gpz_compress_workspace_bytes_f64.argtypes = [u64, u32, pp]
        L.gpz_compress_workspace_bytes_f64.restype = u64
        L.gpz_decompress_f64.argtypes = L.gpz_decompress.argtypes
        L.gpz_decompress_f64.restype = ctypes.c_int
        L.gpz_stats_workspace_bytes.argtypes = [u32]
        L.gpz_stats_workspace_bytes.restype = u64
        L.gpz_bound_check.argtypes = [vp, vp, vp, u64, u32, vp, vp, vp, vp, u64, vp]
        L.gpz_bound_check.restype = ctypes.c_int
        L.gpz_error_stats.argtypes = [vp, vp, vp, u64, u32, vp, ctypes.POINTER(FieldError),
                                      ctypes.POINTER(ctypes.c_double), vp, u64, vp]
        L.gpz_error_stats.restype = ctypes.c_int
        L.gpz_stream_stats.argtypes = [vp, u64, u64, u32, vp, vp, vp, u64, vp]
        L.gpz_stream_stats.restype = ctypes.c_int
        L.gpz_field_range.argtypes = [vp, u64, u32, vp, vp, u64, vp]
        L.gpz_field_range.restype = ctypes.c_int
        L.gpz_field_range_async.argtypes = [vp, u64, u32, vp, vp, u64, vp]
        L.gpz_field_range_async.restype = ctypes.c_int
        L.gpz_field_range_noalloc.argtypes = [vp, u64, u32, vp, vp]
        L.gpz_field_range_noalloc.restype = ctypes.c_int
        L.gpz_rel_to_abs.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_float]
        L.gpz_rel_to_abs.restype = ctypes.c_float
        L.gpz_inspect.argtypes = [vp, u64, ctypes.POINTER(Info)]
        L.gpz_inspect.restype = ctypes.c_int
        L.gpz_set_timing.argtypes = [ctypes.c_int]
        L.gpz_set_timing.restype = ctypes.c_int
        L.gpz_set_timing_kinds.argtypes = [ctypes.c_uint32]
        L.gpz_set_timing_kinds.restype = ctypes.c_int
        L.gpz_timing_collect.argtypes = [ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_uint32), ctypes.c_int]
        L.gpz_timing_collect.restype = ctypes.c_int
        L.gpz_strerror.argtypes = [ctypes.c_int]
        L.gpz_strerror.restype = ctypes.c_char_p
        jp, cp = ctypes.POINTER(Job), ctypes.POINTER(BatchConfig)
        L.gpz_default_batch_config.argtypes = [cp]
        L.gpz_default_batch_config.restype = None
        L.gpz_batch_workspace_bytes.argtypes = [jp, u32, pp]
        L.gpz_batch_workspace_bytes.restype = u64
        L.gpz_batch_create.argtypes = [ctypes.POINTER(vp), jp, u32, pp, cp, vp, u64]
        L.gpz_batch_create.restype = ctypes.c_int
        L.gpz_batch_rebind.argtypes = [vp, jp, u32, vp, u64, vp]
        L.gpz_batch_rebind.restype = ctypes.c_int
        L.gpz_batch_compress.argtypes = [vp, vp]
        L.gpz_batch_compress.restype = ctypes.c_int
        L.gpz_batch_decompress.argtypes = [vp, vp]
        L.gpz_batch_decompress.restype = ctypes.c_int
        L.gpz_batch_sizes.argtypes = [vp]
        L.gpz_batch_sizes.restype = vp
        L.gpz_batch_errors.argtypes = [vp]
        L.gpz_batch_errors.restype = vp
        L.gpz_batch_destroy.argtypes = [vp]
        L.gpz_batch_destroy.restype = ctypes.c_int
        _LIB = L
    return _LIB


def lib():
    """The loaded ctypes library (raises GpzLibraryMissing if not built)."""
    return _lib()


def _check(rc: int, what: str):
    if rc != GPZ_OK:
        raise GpzError(rc, what)


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr_array(tensors: Sequence) -> ctypes.Array:
    arr = (ctypes.c_void_p * max(1, len(tensors)))()
    for i, t in enumerate(tensors):
        arr[i] = t.data_ptr()
    return arr


def _check_fields(fields: Sequence, n: Optional[int] = None, dtype=None):
    torch = _torch()
    dtype = torch.float32 if dtype is None else dtype
    if len(fields) < 1 or len(fields) > 64:
        raise ValueError("1..64 fields")
    n = fields[0].numel() if n is None else n
    for f in fields:
        if f.dtype != dtype or not f.is_cuda or not f.is_contiguous() or f.numel() != n:
            raise ValueError(f"fields must be contiguous {dtype} CUDA tensors of equal length")
    return n


GPZ_FLAG_SINGLE_PASS = 1


def params(nfields: int, block_size: int = 1024, seg_bits: int = 3,
           key_fields: Optional[int] = None, single_pass: bool = False) -> Params:
    """Parameters; `single_pass` selects the look-back compaction instead of
    the paper's encode / scan / copy sequence (same stream)."""
    p = Params()
    _lib().gpz_default_params(ctypes.byref(p), nfields)
    p.block_size = block_size
    p.seg_bits = seg_bits
    if key_fields is not None:
        p.key_fields = key_fields
    p.flags = GPZ_FLAG_SINGLE_PASS if single_pass else 0
    return p


def _eb_array(eb, F: int) -> np.ndarray:
    e = np.asarray(eb, dtype=np.float32)
    if e.ndim == 0:
        e = np.full(F, e, np.float32)
    if e.shape != (F,):
        raise ValueError("eb: scalar or one bound per field")
    return np.ascontiguousarray(e)


def max_compressed_bytes(n: int, nfields: int, p: Optional[Params] = None) -> int:
    return int(_lib().gpz_max_compressed_bytes(n, nfields, ctypes.byref(p) if p else None))


def compress_workspace_bytes(n: int, nfields: int, p: Optional[Params] = None) -> int:
    return int(_lib().gpz_compress_workspace_bytes(n, nfields, ctypes.byref(p) if p else None))


class Compressor:
    """Reusable device buffers for repeated compression of one shape."""

    def __init__(self, n: int, nfields: int, p: Optional[Params] = None, device="cuda"):
        torch = _torch()
        self.n, self.F = n, nfields
        self.p = p if p is not None else params(nfields)
        self.out = torch.empty(max_compressed_bytes(n, nfields, self.p), dtype=torch.uint8,
                               device=device)
        self.ws = torch.empty(max(compress_workspace_bytes(n, nfields, self.p), 256),
                              dtype=torch.uint8, device=device)
        self.perm = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        self.nbytes_dev = torch.zeros(1, dtype=torch.int64, device=device)

    def compress(self, fields: Sequence, eb, want_perm: bool = False, stream=None):
        """Synchronous compress; returns (stream view, perm view or None)."""
        n = _check_fields(fields, self.n)
        ebs = _eb_array(eb, self.F)
        nbytes = ctypes.c_uint64(0)
        rc = _lib().gpz_compress(
            ctypes.cast(_ptr_array(fields), ctypes.c_void_p), n, self.F,
            ebs.ctypes.data_as(ctypes.c_void_p), ctypes.byref(self.p), self.out.data_ptr(),
            self.out.numel(), ctypes.byref(nbytes), self.perm.data_ptr() if want_perm else None,
            self.ws.data_ptr(), self.ws.numel(), _stream_handle(stream))
        _check(rc, "gpz_compress")
        return self.out[: nbytes.value], (self.perm[:n] if want_perm else None)

    def compress_async(self, fields: Sequence, eb, want_perm: bool = False, stream=None):
        """Enqueue only; the stream size lands in self.nbytes_dev."""
        n = _check_fields(fields, self.n)
        ebs = _eb_array(eb, self.F)
        rc = _lib().gpz_compress_async(
            ctypes.cast(_ptr_array(fields), ctypes.c_void_p), n, self.F,
            ebs.ctypes.data_as(ctypes.c_void_p), ctypes.byref(self.p), self.out.data_ptr(),
            self.out.numel(), self.nbytes_dev.data_ptr(),
            self.perm.data_ptr() if want_perm else None, self.ws.data_ptr(), self.ws.numel(),
            _stream_handle(stream))
        _check(rc, "gpz_compress_async")


def compress(fields: Sequence, eb, *, block_size: int = 1024, seg_bits: int = 3,
             key_fields: Optional[int] = None, want_perm: bool = False, stream=None,
             single_pass: bool = False):
    """Compress SoA float32 CUDA tensors; returns (uint8 CUDA tensor, perm or None)."""
    F = len(fields)
    p = params(F, block_size, seg_bits, key_fields, single_pass)
    c = Compressor(fields[0].numel(), F, p, device=fields[0].device)
    s, perm = c.compress(fields, eb, want_perm=want_perm, stream=stream)
    return s.clone(), (perm.clone() if perm is not None else None)


def decompress(stream_bytes, n: int, nfields: int, out: Optional[List] = None, ws=None,
               stream=None) -> List:
    """Decompress a uint8 CUDA tensor holding a stream into F float32 tensors."""
    torch = _torch()
    if not stream_bytes.is_cuda or stream_bytes.dtype != torch.uint8:
        raise ValueError("stream must be a uint8 CUDA tensor")
    if out is None:
        out = [torch.empty(max(n, 1), dtype=torch.float32, device=stream_bytes.device)[:n]
               for _ in range(nfields)]
    if ws is None:
        ws = torch.empty(256, dtype=torch.uint8, device=stream_bytes.device)
    rc = _lib().gpz_decompress(stream_bytes.data_ptr(), stream_bytes.numel(),
                               ctypes.cast(_ptr_array(out), ctypes.c_void_p), n, nfields,
                               ws.data_ptr(), ws.numel(), _stream_handle(stream))
    _check(rc, "gpz_decompress")
    return out


def decompress_async(stream_bytes, n: int, nfields: int, out: List, err, p: Optional[Params] = None,
                     stream=None):
    rc = _lib().gpz_decompress_async(stream_bytes.data_ptr(), stream_bytes.numel(),
                                     ctypes.cast(_ptr_array(out), ctypes.c_void_p), n, nfields,
                                     ctypes.byref(p) if p else None, err.data_ptr(),
                                     _stream_handle(stream))
    _check(rc, "gpz_decompress_async")


def compress_f64(fields: Sequence, eb, *, block_size: int = 1024, seg_bits: int = 3,
                 key_fields: Optional[int] = None, want_perm: bool = False, stream=None):
    """Compress SoA float64 CUDA tensors (Sec. 5.1: float32 steps per field and
    block where they meet the bound, 64-bit steps elsewhere); float32 bounds.
    Returns (uint8 CUDA tensor, perm or None)."""
    torch = _torch()
    F = len(fields)
    n = _check_fields(fields, dtype=torch.float64)
    p = params(F, block_size, seg_bits, key_fields)
    dev = fields[0].device
    out = torch.empty(int(_lib().gpz_max_compressed_bytes_f64(n, F, ctypes.byref(p))),
                      dtype=torch.uint8, device=dev)
    ws = torch.empty(max(int(_lib().gpz_compress_workspace_bytes_f64(n, F, ctypes.byref(p))), 256),
                     dtype=torch.uint8, device=dev)
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if want_perm else None
    ebs = _eb_array(eb, F)
    nbytes = ctypes.c_uint64(0)
    rc = _lib().gpz_compress_f64(
        ctypes.cast(_ptr_array(fields), ctypes.c_void_p), n, F,
        ebs.ctypes.data_as(ctypes.c_void_p), ctypes.byref(p), out.data_ptr(), out.numel(),
        ctypes.byref(nbytes), perm.data_ptr() if want_perm else None, ws.data_ptr(), ws.numel(),
        _stream_handle(stream))
    _check(rc, "gpz_compress_f64")
    return out[: nbytes.value].clone(), (perm[:n].clone() if want_perm else None)


def decompress_f64(stream_bytes, n: int, nfields: int, out: Optional[List] = None, ws=None,
                   stream=None) -> List:
    """Decompress a float64 stream (uint8 CUDA tensor) into F float64 tensors."""
    torch = _torch()
    if not stream_bytes.is_cuda or stream_bytes.dtype != torch.uint8:
        raise ValueError("stream must be a uint8 CUDA tensor")
    if out is None:
        out = [torch.empty(max(n, 1), dtype=torch.float64, device=stream_bytes.device)[:n]
               for _ in range(nfields)]
    if ws is None:
        ws = torch.empty(256, dtype=torch.uint8, device=stream_bytes.device)
    rc = _lib().gpz_decompress_f64(stream_bytes.data_ptr(), stream_bytes.numel(),
                                   ctypes.cast(_ptr_array(out), ctypes.c_void_p), n, nfields,
                                   ws.data_ptr(), ws.numel(), _stream_handle(stream))
    _check(rc, "gpz_decompress_f64")
    return out


def stats_workspace(nfields: int, device="cuda"):
    """A device workspace for the reporting calls (bound check, error and
    stream statistics, field range) of up to `nfields` fields."""
    torch = _torch()
    return torch.empty(int(_lib().gpz_stats_workspace_bytes(nfields)), dtype=torch.uint8,
                       device=device)


def _ws_args(ws):
    return (ws.data_ptr(), ws.numel()) if ws is not None else (None, 0)


def bound_check(orig: Sequence, recon: Sequence, eb, perm=None, stream=None, ws=None
                ) -> Tuple[np.ndarray, np.ndarray]:
    """(violations, max abs error) per field; `ws` from stats_workspace (None:
    the library allocates one for the call)."""
    F = len(orig)
    n = _check_fields(orig)
    _check_fields(recon, n)
    ebs = _eb_array(eb, F)
    viol = np.zeros(F, np.uint64)
    mx = np.zeros(F, np.float64)
    rc = _lib().gpz_bound_check(ctypes.cast(_ptr_array(orig), ctypes.c_void_p),
                                ctypes.cast(_ptr_array(recon), ctypes.c_void_p),
                                perm.data_ptr() if perm is not None else None, n, F,
                                ebs.ctypes.data_as(ctypes.c_void_p),
                                viol.ctypes.data_as(ctypes.c_void_p),
                                mx.ctypes.data_as(ctypes.c_void_p), *_ws_args(ws),
                                _stream_handle(stream))
    _check(rc, "gpz_bound_check")
    return viol, mx


def error_stats(orig: Sequence, recon: Sequence, eb, perm=None, stream=None, ws=None) -> dict:
    """Bound check plus the rate-distortion figures of Sec. 3.1, all computed
    by the library: per-field violation counts, maximum and summed squared
    errors, normalized RMSE over each original field's range, and the
    aggregate PSNR in dB."""
    F = len(orig)
    n = _check_fields(orig)
    _check_fields(recon, n)
    ebs = _eb_array(eb, F)
    res = (FieldError * F)()
    psnr = ctypes.c_double(0.0)
    rc = _lib().gpz_error_stats(ctypes.cast(_ptr_array(orig), ctypes.c_void_p),
                                ctypes.cast(_ptr_array(recon), ctypes.c_void_p),
                                perm.data_ptr() if perm is not None else None, n, F,
                                ebs.ctypes.data_as(ctypes.c_void_p), res, ctypes.byref(psnr),
                                *_ws_args(ws), _stream_handle(stream))
    _check(rc, "gpz_error_stats")
    return {"violations": np.array([r.violations for r in res], np.uint64),
            "max_abs_err": np.array([r.max_abs_err for r in res], np.float64),
            "sum_sq": np.array([r.sum_sq_err for r in res], np.float64),
            "nrmse": np.array([r.nrmse for r in res], np.float64),
            "range": np.array([[r.min, r.max] for r in res], np.float32),
            "psnr": psnr.value}


def stream_stats(stream_bytes, n: int, nfields: int, stream=None, ws=None):
    """(outliers per field, raw blocks) of a stream held in a uint8 CUDA tensor."""
    out = np.zeros(nfields, np.uint64)
    raw = np.zeros(1, np.uint64)
    rc = _lib().gpz_stream_stats(stream_bytes.data_ptr(), stream_bytes.numel(), n, nfields,
                                 out.ctypes.data_as(ctypes.c_void_p),
                                 raw.ctypes.data_as(ctypes.c_void_p), *_ws_args(ws),
                                 _stream_handle(stream))
    _check(rc, "gpz_stream_stats")
    return out, int(raw[0])


def field_range(fields: Sequence, stream=None, ws=None) -> np.ndarray:
    """(F, 2) float32 array of each field's finite minimum and maximum."""
    F = len(fields)
    n = _check_fields(fields)
    mm = np.zeros(2 * F, np.float32)
    rc = _lib().gpz_field_range(ctypes.cast(_ptr_array(fields), ctypes.c_void_p), n, F,
                                mm.ctypes.data_as(ctypes.c_void_p), *_ws_args(ws),
                                _stream_handle(stream))
    _check(rc, "gpz_field_range")
    return mm.reshape(F, 2)


def field_range_async(fields: Sequence, minmax, ws, stream=None):
    """Queue the field range of `fields` into the float32 CUDA tensor
    `minmax` (2F values: min, max per field) without synchronizing; `ws`
    from stats_workspace."""
    F = len(fields)
    n = _check_fields(fields)
    rc = _lib().gpz_field_range_async(ctypes.cast(_ptr_array(fields), ctypes.c_void_p), n, F,
                                      minmax.data_ptr(), *_ws_args(ws), _stream_handle(stream))
    _check(rc, "gpz_field_range_async")


def field_range_noalloc(fields: Sequence, stream=None) -> np.ndarray:
    """As field_range, through the allocation-free entry point (library-owned
    per-GPU scratch; calls on one GPU must not overlap)."""
    F = len(fields)
    n = _check_fields(fields)
    mm = np.zeros(2 * F, np.float32)
    rc = _lib().gpz_field_range_noalloc(ctypes.cast(_ptr_array(fields), ctypes.c_void_p), n, F,
                                        mm.ctypes.data_as(ctypes.c_void_p),
                                        _stream_handle(stream))
    _check(rc, "gpz_field_range_noalloc")
    return mm.reshape(F, 2)


def rel_to_abs(rel: float, lo: float, hi: float) -> float:
    return float(np.float32(_lib().gpz_rel_to_abs(rel, lo, hi)))


def rel_ebs(fields: Sequence, rel: float, stream=None, ws=None) -> np.ndarray:
    """Absolute per-field bounds for a value-range-relative bound (the field
    range kernel, then gpz_rel_to_abs per field)."""
    mm = field_range(fields, stream, ws)
    return np.array([rel_to_abs(rel, float(a), float(b)) for a, b in mm], np.float32)


def inspect(prefix: bytes) -> dict:
    info = Info()
    buf = ctypes.create_string_buffer(bytes(prefix), len(prefix))
    _check(_lib().gpz_inspect(buf, len(prefix), ctypes.byref(info)), "gpz_inspect")
    return dict(n=info.n, nfields=info.nfields, block_size=info.block_size,
                seg_bits=info.seg_bits, key_fields=info.key_fields, nblocks=info.nblocks,
                flags=info.flags)


KERNEL_KINDS = ("encode", "prepare", "decode", "scan", "copy", "generic")


def set_timing(enable: bool, kinds: Optional[Sequence[str]] = None):
    """Turn kernel timing on or off for this host thread; `kinds` limits it
    to some of KERNEL_KINDS (each timed kernel costs an event pair)."""
    if not enable:
        _check(_lib().gpz_set_timing_kinds(0), "gpz_set_timing_kinds")
        return
    if kinds is None:
        _lib().gpz_set_timing(1)
        return
    mask = 0
    for k in kinds:
        mask |= 1 << KERNEL_KINDS.index(k)
    _check(_lib().gpz_set_timing_kinds(mask), "gpz_set_timing_kinds")


def timing_collect() -> dict:
    """Per-kernel (total ms, launches) recorded since the last collection."""
    k = len(KERNEL_KINDS)
    ms = (ctypes.c_double * k)()
    cnt = (ctypes.c_uint32 * k)()
    _check(_lib().gpz_timing_collect(ms, cnt, k), "gpz_timing_collect")
    return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_KINDS)}
