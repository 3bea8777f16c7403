"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and its host-side helpers and argument checks behave (no GPU work)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpz.h")


@pytest.fixture(scope="module")
def gpz():
    import paper_2508_10305_amd as g
    if not os.path.exists(g.LIB_PATH):
        from paper_2508_10305_amd import build
        build.build_lib()
    return g


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gpz_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gpz_compress", "gpz_decompress", "gpz_bound_check"):
        assert must in names


def test_library_exports_every_declared_symbol(gpz):
    L = gpz.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) == set(gpz.EXPORTS)


def test_sizes_match_oracle(gpz, orc):
    L = gpz.lib()
    for n in [0, 1, 1023, 1024, 1025, 10 ** 6]:
        for F in [1, 3, 6]:
            assert gpz.max_compressed_bytes(n, F) == orc.max_bytes(n, F, 1024)
            assert L.gpz_max_compressed_bytes_f64(n, F, None) == orc.max_bytes(n, F, 1024, True)
    assert gpz.compress_workspace_bytes(10 ** 6, 3) >= 4 * 3 * 10 ** 6


def test_rel_to_abs_matches_oracle(gpz, orc):
    rng = np.random.default_rng(0)
    for _ in range(200):
        lo, hi = sorted(rng.standard_normal(2) * 10.0 ** rng.integers(-3, 6))
        lo, hi = float(np.float32(lo)), float(np.float32(hi))
        for rel in (1e-2, 1e-3, 1e-4):
            assert gpz.rel_to_abs(rel, lo, hi) == orc.rel_to_abs(rel, lo, hi)
    assert gpz.rel_to_abs(1e-3, 2.0, 2.0) == orc.rel_to_abs(1e-3, 2.0, 2.0)


def test_inspect_parses_oracle_stream(gpz, orc):
    x = [np.random.default_rng(1).random(3000).astype(np.float32) for _ in range(4)]
    s, _ = orc.compress(x, 1e-3, K=2, KF=2)
    info = gpz.inspect(s[:32].tobytes())
    assert info == dict(n=3000, nfields=4, block_size=1024, seg_bits=2, key_fields=2, nblocks=3,
                        flags=0)
    bad = bytearray(s[:32].tobytes())
    bad[0] ^= 1
    with pytest.raises(gpz.GpzError):
        gpz.inspect(bytes(bad))


def test_invalid_arguments_rejected_before_device_work(gpz):
    L = gpz.lib()
    eb = np.array([1e-3], np.float32)
    out = ctypes.c_uint64(0)
    fake = (ctypes.c_void_p * 1)(ctypes.c_void_p(16))
    p = gpz.params(1)
    bad = gpz.params(1, block_size=100)
    def args(prm, e, F=1):
        return (ctypes.cast(fake, ctypes.c_void_p), 10, F, e.ctypes.data_as(ctypes.c_void_p),
                ctypes.byref(prm), ctypes.c_void_p(16), 1000, ctypes.byref(out), None,
                ctypes.c_void_p(16), 1 << 20, None)

    assert L.gpz_compress(*args(bad, eb)) == gpz.GPZ_EINVAL
    for e in (0.0, -1.0, np.inf, np.nan, 1e-38):
        assert L.gpz_compress(*args(p, np.array([e], np.float32))) == gpz.GPZ_EINVAL
    assert L.gpz_compress(*args(p, eb, F=0)) == gpz.GPZ_EINVAL
    assert L.gpz_compress(*args(p, eb, F=65)) == gpz.GPZ_EINVAL
    # block sizes outside 256..2048 run the generic kernels, but not the
    # single-pass compaction; float64 fields neither
    p64 = gpz.params(1, block_size=64, single_pass=True)
    assert L.gpz_compress(*args(p64, eb)) == gpz.GPZ_EUNSUPPORTED
    p1 = gpz.params(1, single_pass=True)
    assert L.gpz_compress_f64(*args(p1, eb)) == gpz.GPZ_EUNSUPPORTED
    assert L.gpz_max_compressed_bytes_f64(1000, 3, None) == \
        2 * L.gpz_max_compressed_bytes(1000, 3, None) - 4 * (8 + 2 + 3 + 1 + 1)
    assert L.gpz_decompress(None, 100, None, 10, 1, None, 0, None) == gpz.GPZ_EINVAL


def test_strerror(gpz):
    for c in range(-6, 1):
        assert gpz.lib().gpz_strerror(c)


def test_timing_kinds_mask(gpz):
    L = gpz.lib()
    assert L.gpz_set_timing_kinds(1 << 6) == gpz.GPZ_EINVAL  # no kind 6
    assert L.gpz_set_timing_kinds(0x3F) == gpz.GPZ_OK
    assert L.gpz_set_timing_kinds(0) == gpz.GPZ_OK
    with pytest.raises(ValueError):
        gpz.set_timing(True, kinds=("no such kernel",))
    gpz.set_timing(False)


def test_batch_and_stats_entry_points_reject_bad_arguments(gpz):
    """Host-side argument checks of the batch, statistics and timing entry
    points: every one returns a status before touching the device."""
    L = gpz.lib()
    assert L.gpz_batch_destroy(None) == gpz.GPZ_OK
    assert L.gpz_batch_compress(None, None) == gpz.GPZ_EINVAL
    assert L.gpz_batch_decompress(None, None) == gpz.GPZ_EINVAL
    assert L.gpz_batch_sizes(None) is None and L.gpz_batch_errors(None) is None
    jobs = (gpz.Job * 1)()  # zeroed job: no fields, no eb, no output
    assert L.gpz_batch_workspace_bytes(jobs, 1, None) == 0
    b = ctypes.c_void_p()
    p = gpz.Params()
    L.gpz_default_params(ctypes.byref(p), 3)
    p.block_size = 100  # not a power of two
    assert L.gpz_batch_create(ctypes.byref(b), jobs, 1, ctypes.byref(p), None, None, 0) == \
        gpz.GPZ_EINVAL
    assert L.gpz_batch_create(None, jobs, 1, None, None, None, 0) == gpz.GPZ_EINVAL
    assert L.gpz_error_stats(None, None, None, 10, 0, None, None, None, None, 0, None) == \
        gpz.GPZ_EINVAL
    assert L.gpz_stream_stats(None, 100, 10, 3, None, None, None, 0, None) == gpz.GPZ_EINVAL
    assert L.gpz_stats_workspace_bytes(0) == 0 and L.gpz_stats_workspace_bytes(65) == 0
    assert L.gpz_stats_workspace_bytes(64) >= 32 * 64
    # a workspace smaller than gpz_stats_workspace_bytes is refused before any device work
    small = L.gpz_stats_workspace_bytes(3) - 1
    fake = (ctypes.c_void_p * 3)(0x1000, 0x2000, 0x3000)  # never dereferenced on the host
    ebs = np.full(3, 1e-3, np.float32)
    mm = np.zeros(6, np.float32)
    assert L.gpz_field_range(ctypes.cast(fake, ctypes.c_void_p), 10, 3,
                             mm.ctypes.data_as(ctypes.c_void_p), 0x5000, small, None) == \
        gpz.GPZ_EINVAL
    res = (gpz.FieldError * 3)()
    assert L.gpz_error_stats(ctypes.cast(fake, ctypes.c_void_p), ctypes.cast(fake, ctypes.c_void_p),
                             None, 10, 3, ebs.ctypes.data_as(ctypes.c_void_p), res, None, 0x5000,
                             small, None) == gpz.GPZ_EINVAL
    v = np.zeros(3, np.uint64)
    m = np.zeros(3, np.float64)
    assert L.gpz_bound_check(ctypes.cast(fake, ctypes.c_void_p), ctypes.cast(fake, ctypes.c_void_p),
                             None, 10, 3, ebs.ctypes.data_as(ctypes.c_void_p),
                             v.ctypes.data_as(ctypes.c_void_p), m.ctypes.data_as(ctypes.c_void_p),
                             0x5000, small, None) == gpz.GPZ_EINVAL
    ms = (ctypes.c_double * 5)()
    cnt = (ctypes.c_uint32 * 5)()
    assert L.gpz_timing_collect(None, cnt, 5) == gpz.GPZ_EINVAL
    assert L.gpz_timing_collect(ms, cnt, 0) == gpz.GPZ_EINVAL


def test_flags_select_compaction_only(gpz):
    """Only GPZ_FLAG_SINGLE_PASS is a valid flag; it does not change sizes."""
    L = gpz.lib()
    p = gpz.params(3)
    base = L.gpz_compress_workspace_bytes(100_000, 3, ctypes.byref(p))
    p1 = gpz.params(3, single_pass=True)
    assert p1.flags == gpz.GPZ_FLAG_SINGLE_PASS
    assert L.gpz_compress_workspace_bytes(100_000, 3, ctypes.byref(p1)) == base > 0
    assert L.gpz_max_compressed_bytes(100_000, 3, ctypes.byref(p1)) == \
        L.gpz_max_compressed_bytes(100_000, 3, ctypes.byref(p))
    p.flags = 2
    assert L.gpz_compress_workspace_bytes(100_000, 3, ctypes.byref(p)) == 0


def test_injected_allocation_failure(gpz, monkeypatch):
    """With no caller workspace the library allocates one; an injected
    allocation failure (GPZ_FAULT=alloc) surfaces as GPZ_ENOMEM before any
    device work."""
    L = gpz.lib()
    monkeypatch.setenv("GPZ_FAULT", "alloc")
    p = gpz.params(3)
    fake = (ctypes.c_void_p * 3)(0x1000, 0x2000, 0x3000)  # never dereferenced on the host
    ebs = np.full(3, 1e-3, np.float32)
    nbytes = ctypes.c_uint64(0)
    rc = L.gpz_compress(ctypes.cast(fake, ctypes.c_void_p), 5000, 3,
                        ebs.ctypes.data_as(ctypes.c_void_p), ctypes.byref(p), 0x4000, 1 << 20,
                        ctypes.byref(nbytes), None, None, 0, None)
    assert rc == gpz.GPZ_ENOMEM
    # the reporting calls allocate only when no workspace is given
    mm = np.zeros(6, np.float32)
    assert L.gpz_field_range(ctypes.cast(fake, ctypes.c_void_p), 5000, 3,
                             mm.ctypes.data_as(ctypes.c_void_p), None, 0, None) == gpz.GPZ_ENOMEM
    res = (gpz.FieldError * 3)()
    assert L.gpz_error_stats(ctypes.cast(fake, ctypes.c_void_p), ctypes.cast(fake, ctypes.c_void_p),
                             None, 5000, 3, ebs.ctypes.data_as(ctypes.c_void_p), res, None, None,
                             0, None) == gpz.GPZ_ENOMEM


def test_bandwidth_probes_export_and_check_arguments(gpz):
    """libgpzbench.so (the achievable-bandwidth probes beside the roofline
    peak) exports the probes of include/gpz_bench.h and refuses bad shapes
    before launching anything."""
    from paper_2508_10305_amd import build
    if not os.path.exists(build.BENCH_LIB):
        build.build_lib()
    L = ctypes.CDLL(build.BENCH_LIB)
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "gpz_bench.h")).read(),
                  flags=re.S)
    names = sorted(set(re.findall(r"\b(gpzb_[a-z_0-9]+)\s*\(", text)))
    assert names == ["gpzb_copy", "gpzb_mix", "gpzb_read"]
    for n in names:
        assert hasattr(L, n), n
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    L.gpzb_mix.argtypes = [vp, vp, u64, u32, u32, u32, u32, u32, vp]
    L.gpzb_mix.restype = ctypes.c_int
    fake = 0x10000  # never dereferenced on the host
    assert L.gpzb_mix(None, fake, 65536, 4, 1, 1, 1, 0, None) == -1      # null source
    assert L.gpzb_mix(fake, fake, 65536, 2, 1, 1, 1, 0, None) == -1      # ratio not 4:1 / 1:4
    assert L.gpzb_mix(fake, fake, 65536 + 16, 4, 1, 1, 1, 0, None) == -1  # not whole units
    assert L.gpzb_mix(fake, fake, 65536, 1, 4, 1, 8, 0, None) == -1      # unroll 8
    assert L.gpzb_mix(fake, fake, 65536, 1, 4, 0, 1, 0, None) == -1      # empty grid
