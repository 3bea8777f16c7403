"""The allocation-free field range (gpz_field_range_noalloc) against the
workspace-taking gpz_field_range, through the C ABI: two calls in a row on
one GPU, the second on a smaller input (the library-owned scratch keeps the
first call's keys, so the second must reset them), plus the field limit and
an injected allocation failure that must not affect it."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gpz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_10305_amd as g
    g.lib()
    return g


def fields_of(n, F, seed, specials=False, offset=0):
    rng = np.random.default_rng(seed)
    host = [(rng.standard_normal(n + offset) * 10.0 ** (f % 5)).astype(np.float32)
            for f in range(F)]
    if specials and n > 8:
        host[0][offset + 3] = np.inf
        host[0][offset + 5] = -np.inf
        host[1 % F][offset + 7] = np.nan
        host[F - 1][:] = np.nan
    dev = [torch.from_numpy(h).cuda() for h in host]
    return [d[offset:] for d in dev], host


@pytest.mark.parametrize("shapes", [((1_000_003, 6), (4097, 3)), ((5000, 64), (1, 1)),
                                    ((3, 2), (0, 2))])
def test_noalloc_matches_field_range_twice(gpz, shapes):
    for k, (n, F) in enumerate(shapes):
        print(f"[case] noalloc n={n} F={F} call={k}", flush=True)
        fields, _ = fields_of(n, F, seed=k + n, specials=True, offset=k)
        ref = gpz.field_range(fields, ws=gpz.stats_workspace(F))
        got = gpz.field_range_noalloc(fields)
        torch.cuda.synchronize()
        assert got.view(np.uint32).tolist() == ref.view(np.uint32).tolist(), (n, F, k)


def test_noalloc_large_then_small_after_other_calls(gpz):
    big, hb = fields_of(3_000_000, 4, seed=11)
    small, hs = fields_of(1000, 4, seed=12)
    a = gpz.field_range_noalloc(big)
    b = gpz.field_range_noalloc(small)
    for got, host in ((a, hb), (b, hs)):
        for f, h in enumerate(host):
            fin = h[np.isfinite(h)]
            assert got[f, 0] == fin.min() and got[f, 1] == fin.max()


def test_noalloc_field_limit_and_alloc_fault(gpz):
    import ctypes
    fields, _ = fields_of(100, 1, seed=3)
    ptrs = (ctypes.c_void_p * 65)(*([fields[0].data_ptr()] * 65))
    mm = np.zeros(130, np.float32)
    rc = gpz.lib().gpz_field_range_noalloc(ctypes.cast(ptrs, ctypes.c_void_p), 100, 65,
                                           mm.ctypes.data_as(ctypes.c_void_p), None)
    assert rc == gpz.GPZ_EINVAL  # beyond the scratch's 64 fields
    os.environ["GPZ_FAULT"] = "alloc"
    try:
        with pytest.raises(gpz.GpzError):
            gpz.field_range(fields)  # the allocating path fails as injected
        got = gpz.field_range_noalloc(fields)  # the allocation-free one does not
    finally:
        del os.environ["GPZ_FAULT"]
    ref = gpz.field_range(fields)
    assert got.view(np.uint32).tolist() == ref.view(np.uint32).tolist()
