"""GPZ CPU oracle -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper around ``gpz_oracle.c``: a plain, slow, obviously-correct
CPU implementation of the GPZ compressor (arXiv 2508.10305, Sec. 4.1-4.4 and
Sec. 3.2).  It exists to check the HIP implementation; only the tests, the
smoke check and the benchmark's CPU-baseline leg may import it.  It shares no
code with the HIP path and never calls into it.

Build with ``oracle.build_oracle()`` (gcc, ``-ffp-contract=off``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gpz_oracle.c")
LIB = os.path.join(HERE, "_build", "liboracle.so")

OK, EINVAL, ENOSPC, ECORRUPT = 0, -1, -2, -3


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build_oracle() -> str:
    """Compile the oracle shared library (always recompiles)."""
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = f"{LIB}.tmp{os.getpid()}"  # concurrent builds never share a file
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


FUZZ_SRC = os.path.join(HERE, "fuzz_decode.c")
FUZZ_BIN = os.path.join(os.path.dirname(LIB), "fuzz_decode")


def build_fuzz_driver() -> str:
    """Compile the stream-reader robustness driver with AddressSanitizer and
    UndefinedBehaviorSanitizer (host code only)."""
    os.makedirs(os.path.dirname(FUZZ_BIN), exist_ok=True)
    tmp = f"{FUZZ_BIN}.tmp{os.getpid()}"  # concurrent builds never share a file
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-o", tmp, SRC, FUZZ_SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, FUZZ_BIN)
    return FUZZ_BIN


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle()
        L = ctypes.CDLL(LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        f32p = ctypes.POINTER(ctypes.c_float)
        f64p = ctypes.POINTER(ctypes.c_double)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        fpp = ctypes.POINTER(f32p)
        L.oracle_block_min.restype = ctypes.c_float
        L.oracle_block_min.argtypes = [f32p, ctypes.c_uint32]
        L.oracle_quantize.restype = ctypes.c_uint32
        L.oracle_quantize.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                      ctypes.POINTER(ctypes.c_int)]
        L.oracle_sort_rle.restype = ctypes.c_uint32
        L.oracle_sort_rle.argtypes = [u32p, ctypes.c_uint32, u32p, u32p, u32p, u32p]
        dpp = ctypes.POINTER(f64p)
        L.oracle_quantize_wide.restype = ctypes.c_uint64
        L.oracle_quantize_wide.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_float,
                                           ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.oracle_max_bytes.restype = ctypes.c_uint64
        L.oracle_max_bytes.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        L.oracle_max_bytes_typed.restype = ctypes.c_uint64
        L.oracle_max_bytes_typed.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_int]
        L.oracle_compress.restype = ctypes.c_int
        L.oracle_compress.argtypes = [fpp, ctypes.c_uint64, ctypes.c_uint32, f32p, ctypes.c_uint32,
                                      ctypes.c_uint32, ctypes.c_uint32, u8p, ctypes.c_uint64, u64p,
                                      u32p]
        L.oracle_compress_f64.restype = ctypes.c_int
        L.oracle_compress_f64.argtypes = [dpp, ctypes.c_uint64, ctypes.c_uint32, f32p,
                                          ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, u8p,
                                          ctypes.c_uint64, u64p, u32p]
        L.oracle_decompress_f64.restype = ctypes.c_int
        L.oracle_decompress_f64.argtypes = [u8p, ctypes.c_uint64, dpp, ctypes.c_uint64,
                                            ctypes.c_uint32]
        L.oracle_encode_block.restype = ctypes.c_int
        L.oracle_encode_block.argtypes = [fpp, ctypes.c_uint32, ctypes.c_uint32, f32p,
                                          ctypes.c_uint32, ctypes.c_uint32, u32p, ctypes.c_uint32,
                                          u32p, u32p]
        L.oracle_block_trace.restype = ctypes.c_int
        L.oracle_block_trace.argtypes = [fpp, dpp, ctypes.c_uint32, ctypes.c_uint32, f32p,
                                         ctypes.c_uint32, ctypes.c_uint32, f64p, u8p, u32p, u64p,
                                         u8p, u32p, u32p, u32p, u32p, u32p, u32p, u32p]
        L.oracle_inspect.restype = ctypes.c_int
        L.oracle_inspect.argtypes = [u8p, ctypes.c_uint64, u64p]
        L.oracle_decompress.restype = ctypes.c_int
        L.oracle_decompress.argtypes = [u8p, ctypes.c_uint64, fpp, ctypes.c_uint64, ctypes.c_uint32]
        L.oracle_bound_check.restype = ctypes.c_int
        L.oracle_bound_check.argtypes = [fpp, fpp, u32p, ctypes.c_uint64, ctypes.c_uint32, f32p,
                                         u64p, f64p]
        L.oracle_field_range.restype = ctypes.c_int
        L.oracle_field_range.argtypes = [fpp, ctypes.c_uint64, ctypes.c_uint32, f32p]
        L.oracle_error_stats.restype = ctypes.c_int
        L.oracle_error_stats.argtypes = [fpp, fpp, u32p, ctypes.c_uint64, ctypes.c_uint32, f64p,
                                         f64p, f64p]
        L.oracle_stream_stats.restype = ctypes.c_int
        L.oracle_stream_stats.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                          u64p, u64p]
        L.oracle_rel_to_abs.restype = ctypes.c_float
        L.oracle_rel_to_abs.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_float]
        _lib = L
    return _lib


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _field_ptrs(fields: Sequence[np.ndarray]):
    arr = (ctypes.POINTER(ctypes.c_float) * max(1, len(fields)))()
    for i, f in enumerate(fields):
        arr[i] = _ptr(f, ctypes.c_float)
    return arr


def _field_ptrs64(fields: Sequence[np.ndarray]):
    arr = (ctypes.POINTER(ctypes.c_double) * max(1, len(fields)))()
    for i, f in enumerate(fields):
        arr[i] = _ptr(f, ctypes.c_double)
    return arr


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _is_f64(fields) -> bool:
    return len(fields) > 0 and np.asarray(fields[0]).dtype == np.float64


def _ebs(eb, F: int) -> np.ndarray:
    e = np.asarray(eb, dtype=np.float32)
    if e.ndim == 0:
        e = np.full(F, e, dtype=np.float32)
    if e.shape != (F,):
        raise ValueError("eb must be a scalar or one value per field")
    return np.ascontiguousarray(e)


# ---------------------------------------------------------------- steps

def block_min(x) -> float:
    x = _f32(x)
    return float(np.float32(lib().oracle_block_min(_ptr(x, ctypes.c_float), x.size)))


def quantize(x: float, lo: float, eb: float):
    """Grid index and outlier flag of one value (Sec. 4.1 equation)."""
    o = ctypes.c_int(0)
    q = lib().oracle_quantize(ctypes.c_float(x), ctypes.c_float(lo), ctypes.c_float(eb),
                              ctypes.byref(o))
    return int(q), bool(o.value)


def quantize_wide(x: float, lo: float, eb: float, out_f32: bool):
    """Grid index and outlier flag with 64-bit intermediates (Sec. 5.3);
    out_f32: the reconstruction is rounded to float32 (float32 fields)."""
    o = ctypes.c_int(0)
    q = lib().oracle_quantize_wide(float(x), float(lo), ctypes.c_float(eb), int(out_f32),
                                   ctypes.byref(o))
    return int(q), bool(o.value)


def sort_rle(keys: Sequence[int]):
    """Stable sort + run-length + delta coding of a key list (Sec. 4.2-4.3).
    Returns (perm, uniques, counts, deltas)."""
    k = np.ascontiguousarray(keys, dtype=np.uint32)
    n = k.size
    perm = np.zeros(max(1, n), np.uint32)
    uniq = np.zeros(max(1, n), np.uint32)
    cnt = np.zeros(max(1, n), np.uint32)
    dl = np.zeros(max(1, n), np.uint32)
    U = lib().oracle_sort_rle(_ptr(k, ctypes.c_uint32), n, _ptr(perm, ctypes.c_uint32),
                              _ptr(uniq, ctypes.c_uint32), _ptr(cnt, ctypes.c_uint32),
                              _ptr(dl, ctypes.c_uint32))
    return perm[:n], uniq[:U], cnt[:U], dl[:U]


def max_bytes(n: int, F: int, B: int = 1024, f64: bool = False) -> int:
    return int(lib().oracle_max_bytes_typed(n, F, B, int(f64)))


# ---------------------------------------------------------------- whole pipeline

def compress(fields: Sequence[np.ndarray], eb, B: int = 1024, K: int = 3,
             KF: Optional[int] = None, want_perm: bool = False):
    """Compress SoA fields (all float32, or all float64: Sec. 5.1's down-cast
    where it meets the bound); returns (stream bytes as np.uint8, perm or None)."""
    f64 = _is_f64(fields)
    fields = [(_f64 if f64 else _f32)(f) for f in fields]
    F = len(fields)
    n = fields[0].size if F else 0
    if KF is None:
        KF = min(F, 3)
    e = _ebs(eb, F)
    cap = max_bytes(n, F, B, f64) if F else 64
    out = np.zeros(max(cap, 4), np.uint8)
    nbytes = ctypes.c_uint64(0)
    perm = np.zeros(max(1, n), np.uint32) if want_perm else None
    fn = lib().oracle_compress_f64 if f64 else lib().oracle_compress
    rc = fn((_field_ptrs64 if f64 else _field_ptrs)(fields), n, F, _ptr(e, ctypes.c_float), B, K,
            KF, _ptr(out, ctypes.c_uint8), out.size, ctypes.byref(nbytes),
            _ptr(perm, ctypes.c_uint32) if want_perm else None)
    if rc != OK:
        raise OracleError(rc, "compress")
    return out[: nbytes.value].copy(), (perm[:n] if want_perm else None)


# ---------------------------------------------------------------- block-parallel framing
# Blocks are encoded independently (Sec. 4: the sort and the codes are local
# to a block), so the stream of a large snapshot is the stream framing
# (header, superblock table, eb table, length table) around the records of
# its blocks in order.  These helpers run the oracle on block-aligned chunks,
# one call per host thread (ctypes releases the GIL), and frame the chunks'
# records into the one stream the whole call would write.  Only the framing
# is done here; every record comes from oracle_compress / oracle_decompress.

_MAGIC, _HEADER, _SUPER = 0x315A5047, 8, 64


def _threads(threads: Optional[int]) -> int:
    if threads:
        return threads
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


def _split(stream: np.ndarray):
    """(header words, eb bits, record lengths, record words) of a stream."""
    w = np.ascontiguousarray(stream, dtype=np.uint8).view(np.uint32)
    nb = int(w[7])
    ns = (nb + _SUPER - 1) // _SUPER
    F = int(w[4])
    eb = w[_HEADER + 2 * ns: _HEADER + 2 * ns + F]
    lens = w[_HEADER + 2 * ns + F: _HEADER + 2 * ns + F + nb]
    return w[:_HEADER], eb, lens, w[_HEADER + 2 * ns + F + nb:]


def _frame(n: int, F: int, B: int, K: int, KF: int, eb_bits: np.ndarray, lens: np.ndarray,
           records: np.ndarray, version_word: int = 1) -> np.ndarray:
    nb = lens.size
    ns = (nb + _SUPER - 1) // _SUPER
    offs = np.concatenate([[0], np.cumsum(lens.astype(np.uint64))[:-1]]).astype(np.uint64) \
        if nb else np.zeros(0, np.uint64)
    sup = np.zeros(2 * ns, np.uint32)
    sup[0::2] = (offs[::_SUPER] & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    sup[1::2] = (offs[::_SUPER] >> np.uint64(32)).astype(np.uint32)
    hdr = np.array([_MAGIC, version_word, n & 0xFFFFFFFF, n >> 32, F, B, K | (KF << 8), nb],
                   np.uint32)
    return np.concatenate([hdr, sup, eb_bits.astype(np.uint32), lens.astype(np.uint32),
                           records.astype(np.uint32)]).view(np.uint8)


def compress_parallel(fields: Sequence[np.ndarray], eb, B: int = 1024, K: int = 3,
                      KF: Optional[int] = None, threads: Optional[int] = None,
                      want_perm: bool = False):
    """(stream, perm or None) as compress() returns them, computed chunk by
    chunk on host threads."""
    from concurrent.futures import ThreadPoolExecutor
    f64 = _is_f64(fields)
    fields = [(_f64 if f64 else _f32)(f) for f in fields]
    F = len(fields)
    n = fields[0].size
    KF = min(F, 3) if KF is None else KF
    nb = (n + B - 1) // B
    T = _threads(threads)
    per = max(1, -(-nb // (4 * T)))  # blocks per chunk: about four chunks per thread
    chunks = [(b0 * B, min(n, (b0 + per) * B)) for b0 in range(0, nb, per)]

    perm = np.zeros(n, np.uint32) if want_perm else None

    def one(c):
        s, pc = compress([f[c[0]:c[1]] for f in fields], eb, B=B, K=K, KF=KF,
                         want_perm=want_perm)
        if want_perm:
            perm[c[0]:c[1]] = pc + np.uint32(c[0])  # chunk-relative input indices
        return _split(s)
    if not chunks:
        return compress(fields, eb, B=B, K=K, KF=KF, want_perm=want_perm)
    with ThreadPoolExecutor(T) as ex:
        parts = list(ex.map(one, chunks))
    lens = np.concatenate([p[2] for p in parts])
    recs = np.concatenate([p[3] for p in parts])
    flags = 0
    for p in parts:  # header flags of the whole stream: any chunk's
        flags |= int(p[0][1]) >> 16
    return _frame(n, F, B, K, KF, parts[0][1], lens, recs, 1 | (flags << 16)), perm


def decompress_parallel(stream: np.ndarray, n: int, F: int,
                        threads: Optional[int] = None) -> List[np.ndarray]:
    """What decompress() returns, computed chunk by chunk on host threads:
    each chunk of blocks is framed as a stream of its own and decoded by the
    oracle.  The whole stream's header and tables are checked first."""
    from concurrent.futures import ThreadPoolExecutor
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    info = inspect(s)
    if info["n"] != n or info["F"] != F or info["bytes"] != s.size:
        raise OracleError(ECORRUPT, "decompress_parallel")
    hdr, eb_bits, lens, recs = _split(s)
    B, K, KF, nb = info["B"], info["K"], info["KF"], info["nblocks"]
    offs = np.concatenate([[0], np.cumsum(lens.astype(np.int64))]).astype(np.int64)
    w = s.view(np.uint32)
    sup = w[_HEADER: _HEADER + 2 * ((nb + _SUPER - 1) // _SUPER)].astype(np.uint64)
    if nb and not ((sup[0::2] | (sup[1::2] << np.uint64(32))) == offs[:-1:_SUPER]).all():
        raise OracleError(ECORRUPT, "decompress_parallel")
    f64 = bool(info["flags"] & 1)
    outs = [np.zeros(n, np.float64 if f64 else np.float32) for _ in range(F)]
    T = _threads(threads)
    per = max(1, -(-nb // (4 * T)))
    ranges = [(b0, min(nb, b0 + per)) for b0 in range(0, nb, per)]

    def one(r):
        b0, b1 = r
        lo, hi = b0 * B, min(n, b1 * B)
        sub = _frame(hi - lo, F, B, K, KF, eb_bits, lens[b0:b1], recs[offs[b0]:offs[b1]],
                     int(hdr[1]))  # the whole stream's flags (a chunk may hold no wide record)
        part = decompress(sub, hi - lo, F)
        for f in range(F):
            outs[f][lo:hi] = part[f]
    if not ranges:
        return decompress(s, n, F)
    with ThreadPoolExecutor(T) as ex:
        list(ex.map(one, ranges))
    return outs


def encode_block(fields: Sequence[np.ndarray], eb, K: int = 3, KF: Optional[int] = None):
    """Record words of one block (all of ``fields``), and its permutation."""
    fields = [_f32(f) for f in fields]
    F = len(fields)
    n = fields[0].size
    if KF is None:
        KF = min(F, 3)
    e = _ebs(eb, F)
    cap = 1 + F * n
    rec = np.zeros(cap, np.uint32)
    rw = ctypes.c_uint32(0)
    perm = np.zeros(n, np.uint32)
    rc = lib().oracle_encode_block(_field_ptrs(fields), n, F, _ptr(e, ctypes.c_float), K, KF,
                                   _ptr(rec, ctypes.c_uint32), cap, ctypes.byref(rw),
                                   _ptr(perm, ctypes.c_uint32))
    if rc != OK:
        raise OracleError(rc, "encode_block")
    return rec[: rw.value].copy(), perm


def block_trace(fields: Sequence[np.ndarray], eb, K: int = 3, KF: Optional[int] = None) -> dict:
    """Intermediate results of stages 1-3 for one block (float32 or float64)."""
    f64 = _is_f64(fields)
    fields = [(_f64 if f64 else _f32)(f) for f in fields]
    F = len(fields)
    n = fields[0].size
    if KF is None:
        KF = min(F, 3)
    e = _ebs(eb, F)
    lo = np.zeros(F, np.float64)
    wide = np.zeros(F, np.uint8)
    s = np.zeros(3, np.uint32)
    q = np.zeros(F * n, np.uint64)
    outl = np.zeros(F * n, np.uint8)
    key = np.zeros(n, np.uint32)
    perm = np.zeros(n, np.uint32)
    uniq = np.zeros(n, np.uint32)
    cnt = np.zeros(n, np.uint32)
    widths = np.zeros(2 + F, np.uint32)
    U = ctypes.c_uint32(0)
    cw = ctypes.c_uint32(0)
    P = lambda a, t=ctypes.c_uint32: _ptr(a, t)
    rc = lib().oracle_block_trace(None if f64 else _field_ptrs(fields),
                                  _field_ptrs64(fields) if f64 else None, n, F,
                                  _ptr(e, ctypes.c_float), K, KF, P(lo, ctypes.c_double),
                                  P(wide, ctypes.c_uint8), P(s), P(q, ctypes.c_uint64),
                                  P(outl, ctypes.c_uint8), P(key), P(perm), P(uniq), P(cnt),
                                  P(widths), ctypes.byref(U), ctypes.byref(cw))
    if rc != OK:
        raise OracleError(rc, "block_trace")
    u = U.value
    return dict(lo=lo if f64 else lo.astype(np.float32), wide=wide.astype(bool), s=s[:KF],
                q=q.reshape(F, n), outlier=outl.reshape(F, n).astype(bool), key=key, perm=perm,
                uniq=uniq[:u], count=cnt[:u], w_gap=int(widths[0]), w_cnt=int(widths[1]),
                w=widths[2:].copy(), U=u, coded_words=cw.value)


def inspect(stream: np.ndarray) -> dict:
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    info = np.zeros(8, np.uint64)
    rc = lib().oracle_inspect(_ptr(s, ctypes.c_uint8), s.size, _ptr(info, ctypes.c_uint64))
    if rc != OK:
        raise OracleError(rc, "inspect")
    keys = ("n", "F", "B", "K", "KF", "nblocks", "bytes", "flags")
    return {k: int(v) for k, v in zip(keys, info)}


def _decode(stream: np.ndarray, n: int, F: int, f64: bool):
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    outs = [np.zeros(max(1, n), np.float64 if f64 else np.float32) for _ in range(F)]
    if f64:
        rc = lib().oracle_decompress_f64(_ptr(s, ctypes.c_uint8), s.size, _field_ptrs64(outs), n, F)
    else:
        rc = lib().oracle_decompress(_ptr(s, ctypes.c_uint8), s.size, _field_ptrs(outs), n, F)
    return int(rc), [o[:n] for o in outs]


def decompress(stream: np.ndarray, n: int, F: int, f64: bool = False) -> List[np.ndarray]:
    """Decoded fields (float64 arrays for a float64 stream, f64=True)."""
    rc, outs = _decode(stream, n, F, f64)
    if rc != OK:
        raise OracleError(rc, "decompress")
    return outs


def decompress_status(stream: np.ndarray, n: int, F: int, f64: bool = False) -> int:
    return _decode(stream, n, F, f64)[0]


def bound_check(orig: Sequence[np.ndarray], recon: Sequence[np.ndarray], eb, perm=None):
    orig = [_f32(f) for f in orig]
    recon = [_f32(f) for f in recon]
    F = len(orig)
    n = orig[0].size
    e = _ebs(eb, F)
    viol = np.zeros(F, np.uint64)
    mx = np.zeros(F, np.float64)
    p = None if perm is None else np.ascontiguousarray(perm, dtype=np.uint32)
    lib().oracle_bound_check(_field_ptrs(orig), _field_ptrs(recon),
                             None if p is None else _ptr(p, ctypes.c_uint32), n, F,
                             _ptr(e, ctypes.c_float), _ptr(viol, ctypes.c_uint64),
                             _ptr(mx, ctypes.c_double))
    return viol, mx


def field_range(fields: Sequence[np.ndarray]) -> np.ndarray:
    fields = [_f32(f) for f in fields]
    F = len(fields)
    mm = np.zeros(2 * F, np.float32)
    lib().oracle_field_range(_field_ptrs(fields), fields[0].size, F, _ptr(mm, ctypes.c_float))
    return mm.reshape(F, 2)


def rel_to_abs(rel: float, lo: float, hi: float) -> float:
    return float(np.float32(lib().oracle_rel_to_abs(rel, lo, hi)))


def rel_ebs(fields: Sequence[np.ndarray], rel: float) -> np.ndarray:
    mm = field_range(fields)
    return np.array([rel_to_abs(rel, float(a), float(b)) for a, b in mm], np.float32)


def error_stats(orig: Sequence[np.ndarray], recon: Sequence[np.ndarray], perm=None) -> dict:
    """Per-field sum of squared errors and NRMSE, and the aggregate PSNR (dB)."""
    orig = [_f32(f) for f in orig]
    recon = [_f32(f) for f in recon]
    F = len(orig)
    n = orig[0].size
    ss = np.zeros(F, np.float64)
    nr = np.zeros(F, np.float64)
    ps = np.zeros(1, np.float64)
    p = None if perm is None else np.ascontiguousarray(perm, dtype=np.uint32)
    lib().oracle_error_stats(_field_ptrs(orig), _field_ptrs(recon),
                             None if p is None else _ptr(p, ctypes.c_uint32), n, F,
                             _ptr(ss, ctypes.c_double), _ptr(nr, ctypes.c_double),
                             _ptr(ps, ctypes.c_double))
    return {"sum_sq": ss, "nrmse": nr, "psnr": float(ps[0])}


def stream_stats(stream: np.ndarray, n: int, F: int):
    """(outliers per field, raw blocks) of a stream."""
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    out = np.zeros(F, np.uint64)
    raw = np.zeros(1, np.uint64)
    rc = lib().oracle_stream_stats(_ptr(s, ctypes.c_uint8), s.size, n, F,
                                   _ptr(out, ctypes.c_uint64), _ptr(raw, ctypes.c_uint64))
    if rc != OK:
        raise OracleError(rc, "stream_stats")
    return out, int(raw[0])
