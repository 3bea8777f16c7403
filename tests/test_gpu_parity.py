"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Compressed streams must be byte-identical, permutations identical,
decompressed floats bit-identical, bound checks identical.  Integer/byte work
has no tolerance; the floating-point steps are fixed to the same IEEE
operations on both sides, so the tolerance is zero everywhere."""
import ctypes
import sys

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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(host):
    return [torch.from_numpy(np.ascontiguousarray(f)).cuda() for f in host]


def check_case(gpz, orc, host, eb, B=1024, K=3, KF=None, label=""):
    say(f"[case] {label} n={host[0].size} F={len(host)} B={B} K={K} KF={KF}")
    F = len(host)
    n = host[0].size
    ref, ref_perm = orc.compress(host, eb, B=B, K=K, KF=KF, want_perm=True)
    dev = to_dev(host)
    got, perm = gpz.compress(dev, eb, block_size=B, seg_bits=K, key_fields=KF, want_perm=True)
    torch.cuda.synchronize()
    g = got.cpu().numpy()
    assert g.size == ref.size, f"{label}: size {g.size} != oracle {ref.size}"
    if not (g == ref).all():
        w1, w2 = g.view(np.uint32), ref.view(np.uint32)
        bad = np.nonzero(w1 != w2)[0]
        raise AssertionError(f"{label}: {bad.size} words differ, first at word {bad[0]}")
    assert (perm.cpu().numpy().astype(np.uint32) == ref_perm).all(), f"{label}: perm"
    # the single-pass (look-back) compaction writes the same stream, except
    # that it stores raw a block needing 64-bit grid steps (stream flag 2);
    # it exists for the wave-per-block encoder's block sizes only
    if B in (256, 512, 1024, 2048):
        got1, perm1 = gpz.compress(dev, eb, block_size=B, seg_bits=K, key_fields=KF,
                                   want_perm=True, single_pass=True)
        if (ref.view(np.uint32)[1] >> 17) & 1:
            out1 = gpz.decompress(got1, n, F)
            v1, _ = gpz.bound_check(dev, out1, eb, perm=perm1)
            assert (v1 == 0).all(), f"{label}: single-pass stream misses the bound"
        else:
            assert torch.equal(got1, got), f"{label}: single-pass compaction stream differs"
            assert torch.equal(perm1, perm), f"{label}: single-pass perm differs"
    out = gpz.decompress(got, n, F)
    ref_out = orc.decompress(ref, n, F)
    for f in range(F):
        a = out[f].cpu().numpy().view(np.uint32)
        assert (a == ref_out[f].view(np.uint32)).all(), f"{label}: decoded field {f}"
    viol, mx = gpz.bound_check(dev, out, eb, perm=perm)
    rviol, rmx = orc.bound_check(host, ref_out, eb, perm=ref_perm)
    assert (viol == rviol).all() and (viol == 0).all(), f"{label}: violations {viol}"
    assert (mx == rmx).all(), f"{label}: max error {mx} vs {rmx}"
    return g


@pytest.mark.parametrize("n", [1, 63, 64, 65, 255, 1000, 1023, 1024, 1025, 5000])
@pytest.mark.parametrize("F", [1, 3, 6])
def test_edge_sizes(gpz, orc, n, F):
    rng = np.random.default_rng(n * 13 + F)
    host = [rng.random(n).astype(np.float32) for _ in range(F)]
    check_case(gpz, orc, host, 1e-4, label="edge")


@pytest.mark.parametrize("B", [256, 512, 1024, 2048])
@pytest.mark.parametrize("K,KF", [(0, 3), (1, 3), (2, 2), (3, 3), (4, 3), (5, 3), (3, 1), (5, 2)])
def test_block_and_segment_parameters(gpz, orc, B, K, KF):
    from paper_2508_10305_amd import synth
    host = synth.clusters(20_000 + 37, seed=B + K, extra_fields=1)
    check_case(gpz, orc, host, 1e-4, B=B, K=K, KF=KF, label=f"params B={B} K={K} KF={KF}")


def test_config_small_clusters(gpz, orc):
    """1,000,000 particles x 3 fields, abs eb 1e-4 (the small parity workload)."""
    from paper_2508_10305_amd import synth
    host = synth.clusters(1_000_000, seed=0)
    check_case(gpz, orc, host, 1e-4, label="clusters 1M")


@pytest.mark.parametrize("rel", [1e-2, 1e-3, 1e-4])
def test_cosmology_md_lidar_scaled(gpz, orc, rel):
    from paper_2508_10305_amd import synth
    sets = {
        "cosmology": synth.cosmology(1_500_000, seed=1, n_halos=256),
        "md": synth.md(48, seed=2),
        "lidar": synth.lidar(800_000, seed=3),
    }
    for name, host in sets.items():
        eb = orc.rel_ebs(host, rel)
        dev = to_dev(host)
        geb = gpz.rel_ebs(dev, rel)
        assert (geb.view(np.uint32) == eb.view(np.uint32)).all(), f"{name}: relative bounds"
        check_case(gpz, orc, host, eb, label=f"{name} rel {rel}")


@pytest.mark.parametrize("K", [3, 5])
def test_local_storage_orders(gpz, orc, K):
    """File-like storage orders (particles stored near their neighbours:
    small blocks, narrow codes, short runs of segment IDs) against the
    oracle, and a shuffled crystal as the opposite case (md's local order is
    its lattice order)."""
    from paper_2508_10305_amd import synth
    sets = [(k, "local") for k in ("clusters", "cosmology", "lidar", "md")] + [("md", "shuffled")]
    for kind, order in sets:
        host = synth.make(kind, 300_000, seed=11, order=order)
        eb = orc.rel_ebs(host, 1e-3)
        check_case(gpz, orc, host, eb, K=K, label=f"{kind} {order} K={K}")


def test_specials_and_outliers(gpz, orc):
    rng = np.random.default_rng(5)
    n = 7000
    host = []
    for f in range(4):
        x = (rng.standard_normal(n) * 100).astype(np.float32)
        idx = rng.choice(n, 300, replace=False)
        sp = np.array([np.nan, np.inf, -np.inf, -0.0, 0.0, 1e-40, -1e-42, 3e38, -3e38], np.float32)
        x[idx] = sp[rng.integers(0, sp.size, idx.size)]
        x[idx[:3]] = np.array([0x7F800001, 0xFF812345, 0x7FC00001], np.uint32).view(np.float32)
        host.append(x)
    for eb in (1e-6, 1e-3, 10.0):
        check_case(gpz, orc, host, eb, label=f"specials eb={eb}")


@pytest.mark.parametrize("B", [256, 512, 1024, 2048])
def test_every_packing_width(gpz, orc, B):
    """Every fixed-length width 1..24 of a field array, in full and partial
    blocks: with eb = 0.5 the grid step is 1, so integer values k are their
    own codes, and block b of field 1 holds codes of exactly 1 + b % 24 bits
    (field 2 the mirror width, field 3 random widths)."""
    rng = np.random.default_rng(B)
    nblocks = 49
    n = nblocks * B - B // 2 - 3
    host = [rng.random(n).astype(np.float32)]  # the key field
    for f in range(3):
        x = np.empty(n, np.float32)
        for b in range(nblocks):
            lo, hi = b * B, min(n, (b + 1) * B)
            w = [1 + b % 24, 24 - b % 24, int(rng.integers(1, 25))][f]
            k = rng.integers(0, 1 << w, hi - lo)
            k[rng.integers(0, hi - lo)] = 0
            k[rng.integers(0, hi - lo)] = (1 << w) - 1
            x[lo:hi] = k.astype(np.float32)
        host.append(x)
    eb = np.array([1e-3, 0.5, 0.5, 0.5], np.float32)
    seen = set()
    for b in range(nblocks):
        tr = orc.block_trace([f[b * B:(b + 1) * B] for f in host], eb, KF=1)
        assert tr["w"][1] == 1 + b % 24 and tr["w"][2] == 24 - b % 24, f"block {b}: {tr['w']}"
        seen.update(int(w) for w in tr["w"])
    assert seen >= set(range(1, 25))
    check_case(gpz, orc, host, eb, B=B, KF=1, label=f"widths B={B}")


def test_quantizer_range_boundary(gpz, orc):
    """Grid indices at the top of the 24-bit range (Sec. 4.1, Sec. 5.3).
    With eb = 0.5 the grid step is 1: 2^24-1 is on the 24-bit grid; a block
    holding 2^24 or 2^24+2 steps above its minimum takes the 64-bit steps for
    that field, which code those values exactly (no outlier); -0.0 in a block
    whose minimum is +0 or -0 is on the grid."""
    B = 1024
    rng = np.random.default_rng(12)
    cases = [
        [0.0, 16777215.0],             # largest 24-bit index: on the grid
        [0.0, 16777216.0],             # t = 2^24: 64-bit steps
        [0.0, 16777216.0, 16777218.0],
        [5.0, 16777220.0],             # t = 2^24-1 after the minimum shift: 24-bit grid
        [4.0, 16777220.0],             # t = 2^24 after the minimum shift: 64-bit steps
        [-0.0, 0.0, 3.0],              # signed zeros
        [-0.0, 7.0],
    ]
    host = [rng.random(B * len(cases)).astype(np.float32)]
    x = np.empty(B * len(cases), np.float32)
    for b, vals in enumerate(cases):
        x[b * B:(b + 1) * B] = np.asarray(vals, np.float32)[rng.integers(0, len(vals), B)]
        x[b * B:b * B + len(vals)] = vals  # every value present
    host.append(x)
    eb = np.array([1e-3, 0.5], np.float32)
    tr = [orc.block_trace([f[b * B:(b + 1) * B] for f in host], eb, KF=1)
          for b in range(len(cases))]
    assert [int(t["outlier"][1].sum()) for t in tr] == [0] * len(cases)
    assert [bool(t["wide"][1]) for t in tr] == [False, True, True, False, True, False, False]
    check_case(gpz, orc, host, eb, B=B, KF=1, label="quantizer range boundary")


def test_block_minimum_non_finite(gpz, orc):
    """The block minimum lo (Sec. 4.1) is taken over finite values only.
    Each block holds one arrangement of non-finite values in an otherwise
    finite field: none, a single NaN of either sign (quiet and signalling),
    a single -inf or +inf, all +inf, all NaN, -inf beside NaN, and a
    negative NaN in the block's first or last position; the partial last
    block holds one too.  A negative NaN is the smallest float under an
    order-preserving integer key, so a minimum that let it through would
    set lo to NaN."""
    B = 1024
    rng = np.random.default_rng(31)
    bits = lambda u: np.array([u], np.uint32).view(np.float32)[0]
    qnan, nqnan, nsnan = bits(0x7FC00000), bits(0xFFC00001), bits(0xFF800001)
    cases = [
        {}, {"r": qnan}, {"r": nqnan}, {"r": nsnan}, {"r": -np.inf}, {"r": np.inf},
        {"all": np.inf}, {"all": nqnan}, {"r": -np.inf, "r2": qnan},
        {0: nqnan}, {B - 1: nqnan}, {"r": nqnan},
    ]
    n = (len(cases) - 1) * B + 517
    host = []
    for f in range(5):
        x = (rng.standard_normal(n) * 10 + 3).astype(np.float32)
        for b in range(len(cases)):
            c = cases[(b + 2 * f) % len(cases)]
            lo, hi = b * B, min(n, (b + 1) * B)
            for key, v in c.items():
                if key == "all":
                    x[lo:hi] = v
                elif key in ("r", "r2"):
                    x[lo + int(rng.integers(0, hi - lo))] = v
                elif lo + key < hi:
                    x[lo + key] = v
        host.append(x)
    for eb in (1e-3, 0.5):
        check_case(gpz, orc, host, eb, KF=3, label=f"non-finite block minimum eb={eb}")


def test_raw_fallback_and_constant(gpz, orc):
    rng = np.random.default_rng(6)
    host = [rng.random(4000).astype(np.float32) for _ in range(2)]
    check_case(gpz, orc, host, 2.0 ** -100, label="raw fallback")
    const = [np.full(3000, np.float32(-4.5)) for _ in range(3)]
    check_case(gpz, orc, const, 1e-3, label="constant")
    grid = [(1.0 + rng.integers(0, 1000, 5000) * 2.0 ** -9).astype(np.float32) for _ in range(3)]
    check_case(gpz, orc, grid, 2.0 ** -10, label="on-grid")
    zeros = [np.zeros(2000, np.float32), -np.zeros(2000, np.float32)]
    check_case(gpz, orc, zeros, 1e-3, label="zeros")


def test_gpu_decodes_oracle_stream_and_rejects_corruption(gpz, orc):
    from paper_2508_10305_amd import synth
    host = synth.clusters(100_000, seed=9)
    ref, _ = orc.compress(host, 1e-4)
    s = torch.from_numpy(ref).cuda()
    out = gpz.decompress(s, 100_000, 3)
    ref_out = orc.decompress(ref, 100_000, 3)
    for a, b in zip(out, ref_out):
        assert (a.cpu().numpy().view(np.uint32) == b.view(np.uint32)).all()
    say("[case] corrupt: truncated")
    with pytest.raises(gpz.GpzError) as e:
        gpz.decompress(s[:-4], 100_000, 3)
    assert e.value.code == gpz.GPZ_ECORRUPT
    rng = np.random.default_rng(1)
    nb = 98
    pre = 8 + 2 * 2 + 3 + nb
    for t in range(40):
        bad = ref.copy()
        pos = int(rng.integers(4 * pre, ref.size))
        bad[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        rc_ref = orc.decompress_status(bad, 100_000, 3)
        try:
            gpz.decompress(torch.from_numpy(bad).cuda(), 100_000, 3)
            rc = 0
        except gpz.GpzError as err:
            rc = err.code
        assert rc == rc_ref, f"flip at byte {pos}: gpu {rc} oracle {rc_ref}"
    bad = ref.copy().view(np.uint32)
    bad[8 + 4 + 3 + 5] += 1  # a record length
    with pytest.raises(gpz.GpzError):
        gpz.decompress(torch.from_numpy(bad.view(np.uint8)).cuda(), 100_000, 3)


def test_corrupt_tables_are_rejected(gpz, orc):
    """Damaged superblock and length tables (entries near 2^64 or 2^32,
    whose sums would wrap in 64 or 32 bits) must be reported as corrupt by
    the synchronous decoder, flagged by the asynchronous one, and agree with
    the oracle's verdict."""
    from paper_2508_10305_amd import synth
    n = 200_000
    host = synth.clusters(n, seed=12)
    ref, _ = orc.compress(host, 1e-4)
    nb = (n + 1023) // 1024
    ns = (nb + 63) // 64
    lt = 8 + 2 * ns + 3
    p = gpz.params(3)
    out = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3)]
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    cases = {
        "superblock 1 near 2^64": [(8 + 2, 0xFFFFFF00), (8 + 3, 0xFFFFFFFF)],
        "superblock 1 high word": [(8 + 3, 1)],
        "superblock 0 nonzero": [(8, 5)],
        "length near 2^32": [(lt + 5, 0xFFFFFFF0)],
        "length near 2^32, first of superblock": [(lt + 64, 0xFFFFFFF0)],
        "two lengths summing past 2^32": [(lt + 1, 0x80000000), (lt + 2, 0x80000010)],
        "last length": [(lt + nb - 1, 7)],
    }
    for label, edits in cases.items():
        bad = ref.copy().view(np.uint32)
        for at, v in edits:
            bad[at] = np.uint32(v)
        bad8 = bad.view(np.uint8)
        say(f"[case] corrupt tables: {label}")
        assert orc.decompress_status(bad8, n, 3) == orc.ECORRUPT, label
        d = torch.from_numpy(bad8.copy()).cuda()
        with pytest.raises(gpz.GpzError) as e:
            gpz.decompress(d, n, 3, out=out)
        assert e.value.code == gpz.GPZ_ECORRUPT, label
        gpz.decompress_async(d, n, 3, out, err, p)
        torch.cuda.synchronize()
        assert int(err.item()) != 0, f"{label}: async decoder did not flag the stream"


def test_empty_snapshot_stream(gpz, orc):
    """A snapshot with no particles: header and eb table only, checked on
    the device by both decoders (the asynchronous one never waits)."""
    host = [np.zeros(0, np.float32) for _ in range(3)]
    ref, _ = orc.compress(host, 1e-3)
    s, _ = gpz.compress(to_dev(host), 1e-3)
    assert (s.cpu().numpy() == ref).all()
    gpz.decompress(s, 0, 3)
    p = gpz.params(3)
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    gpz.decompress_async(s, 0, 3, [torch.empty(1, device="cuda")[:0] for _ in range(3)], err, p)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    bad = ref.copy().view(np.uint32)
    bad[8 + 1] = 0x7FC00000  # an eb that is not a valid bound
    d = torch.from_numpy(bad.view(np.uint8).copy()).cuda()
    assert orc.decompress_status(bad.view(np.uint8), 0, 3) == orc.ECORRUPT
    with pytest.raises(gpz.GpzError) as e:
        gpz.decompress(d, 0, 3)
    assert e.value.code == gpz.GPZ_ECORRUPT
    gpz.decompress_async(d, 0, 3, [torch.empty(1, device="cuda")[:0] for _ in range(3)], err, p)
    torch.cuda.synchronize()
    assert int(err.item()) != 0


def test_golden_four_field_block(gpz, orc):
    """The hand-derived four-field block (half-way outlier in a key field, a
    NaN in an attribute field): the GPU writes the derived words."""
    import json
    import os
    from test_oracle_pins import golden_fields
    with open(os.path.join(os.path.dirname(__file__), "golden", "four_field_block.json")) as f:
        g = json.load(f)
    fields = golden_fields(g)
    s, perm = gpz.compress(to_dev(fields), g["eb"], block_size=g["B"], seg_bits=g["K"],
                           key_fields=g["KF"], want_perm=True)
    assert s.cpu().numpy().view(np.uint32).tolist() == g["stream_words"]
    assert perm.cpu().numpy().tolist() == g["perm"]
    out = gpz.decompress(s, 20, 4)
    for got, want in zip(out, golden_fields(g, "decompressed")):
        assert (got.cpu().numpy().view(np.uint32) == want.view(np.uint32)).all()


@pytest.mark.parametrize("single_pass", [False, True])
@pytest.mark.parametrize("short", [1, 4097, None])
def test_enospc_reports_size(gpz, orc, single_pass, short):
    """Too small an output buffer: GPZ_ENOSPC with the size needed, and not a
    byte written past the capacity (sentinel bytes behind it stay intact)."""
    n = 10_000
    host = [np.random.default_rng(2).random(n).astype(np.float32) for _ in range(3)]
    dev = to_dev(host)
    ref, _ = orc.compress(host, 1e-3)
    L = gpz.lib()
    p = gpz.params(3, single_pass=single_pass)
    cap = ref.size - short if short else 40  # None: not even the header fits
    buf = torch.full((cap + 8192,), 0xA5, dtype=torch.uint8, device="cuda")
    ws = torch.empty(gpz.compress_workspace_bytes(n, 3, p), dtype=torch.uint8, device="cuda")
    nbytes = ctypes.c_uint64(0)
    ptrs = (ctypes.c_void_p * 3)(*[t.data_ptr() for t in dev])
    ebs = np.full(3, 1e-3, np.float32)
    say(f"[case] enospc single_pass={single_pass} cap={cap}")
    rc = L.gpz_compress(ctypes.cast(ptrs, ctypes.c_void_p), n, 3,
                        ebs.ctypes.data_as(ctypes.c_void_p), ctypes.byref(p), buf.data_ptr(),
                        cap, ctypes.byref(nbytes), None, ws.data_ptr(), ws.numel(),
                        torch.cuda.current_stream().cuda_stream)
    assert rc == gpz.GPZ_ENOSPC and nbytes.value == ref.size
    assert (buf[cap:].cpu().numpy() == 0xA5).all(), "bytes written past the capacity"


def test_field_range_parity(gpz, orc):
    rng = np.random.default_rng(3)
    host = [(rng.standard_normal(300_001) * 10 ** k).astype(np.float32) for k in range(-2, 3)]
    host[0][[5, 6, 7]] = [np.nan, np.inf, -np.inf]
    host.append(np.full(300_001, np.nan, np.float32))
    host.append(np.where(rng.random(300_001) < 0.5, -0.0, 0.0).astype(np.float32))
    dev = to_dev(host)
    g = gpz.field_range(dev)
    r = orc.field_range(host)
    assert (g.view(np.uint32) == r.view(np.uint32)).all()


@pytest.mark.parametrize("offset", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [1, 3, 7, 64, 1001, 262_147])
def test_field_range_unaligned_views(gpz, orc, offset, n):
    """Views that start off a 16-byte boundary, with the extremes placed in
    the unaligned head and the tail."""
    rng = np.random.default_rng(n + offset)
    host = [rng.standard_normal(n + offset).astype(np.float32) for _ in range(2)]
    host[0][offset] = 1e30  # first element of the view: head when offset != 0
    host[1][-1] = -1e30     # last element: tail
    dev = [t[offset:] for t in to_dev(host)]
    g = gpz.field_range(dev)
    r = orc.field_range([h[offset:].copy() for h in host])
    assert (g.view(np.uint32) == r.view(np.uint32)).all()


@pytest.mark.parametrize("kind", ["identity", "block", "global", "bad"])
def test_bound_check_permutations(gpz, orc, kind):
    """The bound check against the oracle's for identity, block-local, global
    and invalid permutations, with violations, NaNs and a ragged tail."""
    rng = np.random.default_rng(11)
    n, F = 5000, 4
    orig = [rng.standard_normal(n).astype(np.float32) for _ in range(F)]
    eb = np.array([1e-3, 1e-2, 1e-4, 1e-3], np.float32)
    if kind == "identity":
        perm = None
    elif kind == "global":
        perm = rng.permutation(n).astype(np.uint32)
    else:
        perm = np.concatenate([1024 * b + rng.permutation(min(1024, n - 1024 * b))
                               for b in range((n + 1023) // 1024)]).astype(np.uint32)
        if kind == "bad":
            perm[[3, 4000]] = [n, 0xFFFFFFFF]
    src = np.arange(n) if perm is None else np.minimum(perm, n - 1)
    recon = [(o[src] + rng.uniform(-1.2, 1.2, n).astype(np.float32) * e).astype(np.float32)
             for o, e in zip(orig, eb)]
    recon[2][[10, 20]] = np.nan
    dev_o, dev_r = to_dev(orig), to_dev(recon)
    dperm = torch.from_numpy(perm.view(np.int32)).cuda() if perm is not None else None
    viol, mx = gpz.bound_check(dev_o, dev_r, eb, perm=dperm)
    rviol, rmx = orc.bound_check(orig, recon, eb, perm=perm)
    assert (viol == rviol).all(), f"{kind}: {viol} vs {rviol}"
    assert (mx == rmx).all(), f"{kind}: {mx} vs {rmx}"
    assert viol.sum() > 0


def test_error_stats_parity(gpz, orc):
    """Rate-distortion figures of a round trip: violations and maximum error
    exactly; sums of squares (summation order differs: each d*d is exact to
    within one rounding, so n * 2^-52 relative bounds the difference) and the
    aggregate PSNR to 1e-9 relative."""
    from paper_2508_10305_amd import synth
    host = synth.clusters(200_003, seed=21, extra_fields=2)
    eb = np.array([1e-4, 1e-3, 1e-2, 1e-3, 1e-4], np.float32)
    dev = to_dev(host)
    s, perm = gpz.compress(dev, eb, want_perm=True)
    out = gpz.decompress(s, host[0].size, len(host))
    st = gpz.error_stats(dev, out, eb, perm=perm)
    ref_out = orc.decompress(s.cpu().numpy(), host[0].size, len(host))
    ref = orc.error_stats(host, ref_out, perm=perm.cpu().numpy().astype(np.uint32))
    rv, rm = orc.bound_check(host, ref_out, eb, perm=perm.cpu().numpy().astype(np.uint32))
    assert (st["violations"] == rv).all() and (st["max_abs_err"] == rm).all()
    assert np.allclose(st["sum_sq"], ref["sum_sq"], rtol=1e-9, atol=0)
    assert np.allclose(st["nrmse"], ref["nrmse"], rtol=1e-9, atol=0)
    assert abs(st["psnr"] - ref["psnr"]) <= 1e-9 * abs(ref["psnr"])
    assert (st["range"].view(np.uint32) == orc.field_range(host).view(np.uint32)).all()


def test_reporting_calls_allocate_nothing_with_a_workspace(gpz, orc, monkeypatch):
    """With a caller workspace the field range, error statistics, bound check
    and stream statistics make no allocation: they succeed while every
    library allocation is made to fail (GPZ_FAULT=alloc), and give the
    oracle's results; without one they report GPZ_ENOMEM."""
    from paper_2508_10305_amd import synth
    host = synth.clusters(150_001, seed=31, extra_fields=1)
    dev = to_dev(host)
    n, F = host[0].size, len(host)
    eb = orc.rel_ebs(host, 1e-3)
    s, perm = gpz.compress(dev, eb, want_perm=True)
    out = gpz.decompress(s, n, F)
    ws = gpz.stats_workspace(F)
    monkeypatch.setenv("GPZ_FAULT", "alloc")
    say("[case] reporting calls with GPZ_FAULT=alloc")
    assert (gpz.rel_ebs(dev, 1e-3, ws=ws).view(np.uint32) == eb.view(np.uint32)).all()
    st = gpz.error_stats(dev, out, eb, perm=perm, ws=ws)
    v, m = gpz.bound_check(dev, out, eb, perm=perm, ws=ws)
    pp = perm.cpu().numpy().astype(np.uint32)
    ref_out = orc.decompress(s.cpu().numpy(), n, F)
    rv, rm = orc.bound_check(host, ref_out, eb, perm=pp)
    assert (v == rv).all() and (m == rm).all()
    assert (st["violations"] == rv).all() and (st["max_abs_err"] == rm).all()
    got = gpz.stream_stats(s, n, F, ws=ws)
    ref = orc.stream_stats(s.cpu().numpy(), n, F)
    assert got[0].tolist() == ref[0].tolist() and got[1] == ref[1]
    for call in (lambda: gpz.field_range(dev), lambda: gpz.error_stats(dev, out, eb, perm=perm),
                 lambda: gpz.bound_check(dev, out, eb), lambda: gpz.stream_stats(s, n, F)):
        with pytest.raises(gpz.GpzError) as e:
            call()
        assert e.value.code == gpz.GPZ_ENOMEM


def test_stream_stats_parity(gpz, orc):
    """Outlier and raw-block counts of GPU streams equal the oracle's; a
    broken record length is reported as corrupt."""
    rng = np.random.default_rng(5)
    n = 50_000
    smooth = [np.linspace(0, 1, n).astype(np.float32) for _ in range(3)]
    for f in range(3):
        smooth[f][rng.integers(0, n, 40 * (f + 1))] = np.nan
    noise = [rng.random(n).astype(np.float32) for _ in range(3)]
    mixed = [np.concatenate([a[: n // 2], b[n // 2:]]) for a, b in zip(smooth, noise)]
    for label, host, eb in (("smooth", smooth, 1e-3), ("noise", noise, 1e-9), ("mixed", mixed, 1e-7)):
        s, _ = gpz.compress(to_dev(host), eb)
        got = gpz.stream_stats(s, n, 3)
        ref = orc.stream_stats(s.cpu().numpy(), n, 3)
        say(f"[case] stream stats {label}: {got}")
        assert got[0].tolist() == ref[0].tolist() and got[1] == ref[1], label
    bad = s.clone().view(torch.int32)
    bad[8 + 2 * 1 + 3 + 2] += 1  # length of block 2
    with pytest.raises(gpz.GpzError) as e:
        gpz.stream_stats(bad.view(torch.uint8), n, 3)
    assert e.value.code == gpz.GPZ_ECORRUPT


@pytest.mark.parametrize("single_pass", [False, True])
def test_kernel_timing_log(gpz, single_pass):
    """The event log records one entry per kernel of each call: clearing,
    encoder, scan and copy (three-step) or clearing and encoder (single
    pass), and the decoder."""
    from paper_2508_10305_amd import synth
    host = synth.clusters(300_000, seed=4)
    dev = to_dev(host)
    gpz.set_timing(True)
    gpz.timing_collect()
    s, _ = gpz.compress(dev, 1e-4, single_pass=single_pass)
    s, _ = gpz.compress(dev, 1e-4, single_pass=single_pass)
    gpz.decompress(s, 300_000, 3)
    kt = gpz.timing_collect()
    gpz.set_timing(False)
    counts = {k: v[1] for k, v in kt.items()}
    # the walk over the blocks the encoder left for 64-bit steps shares the
    # scan's launch; the decoder's walk for wide records ("generic") is not
    # launched when the header announces none
    want = {"prepare": 2, "encode": 2, "decode": 1, "scan": 0 if single_pass else 2,
            "copy": 0 if single_pass else 2, "generic": 0}
    assert counts == want, counts
    assert all(kt[k][0] > 0 for k in want if want[k])
    assert gpz.timing_collect()["encode"][1] == 0  # the log was cleared
    # timing a subset of the kinds: only those launches are logged
    gpz.set_timing(True, kinds=("encode", "decode"))
    s, _ = gpz.compress(dev, 1e-4, single_pass=single_pass)
    gpz.decompress(s, 300_000, 3)
    kt = gpz.timing_collect()
    gpz.set_timing(False)
    assert {k: v[1] for k, v in kt.items()} == {"encode": 1, "prepare": 0, "decode": 1,
                                                "scan": 0, "copy": 0, "generic": 0}


def test_random_parameters_match_oracle(gpz, orc):
    """Random block sizes, segment bits, key-field counts, bounds and value
    mixes (the property-test generator of the oracle): GPU stream, permutation
    and decompressed bits equal the oracle's in every case."""
    from hypothesis import HealthCheck, given, settings
    from hypothesis import strategies as st
    from test_oracle_properties import KINDS, make_fields

    @settings(max_examples=40, deadline=None, derandomize=True,
              suppress_health_check=[HealthCheck.too_slow])
    @given(B=st.sampled_from([256, 512, 1024, 2048]), n=st.integers(1, 9000),
           F=st.integers(1, 8), K=st.integers(0, 5), kf=st.integers(1, 3),
           e=st.floats(-6.0, -1.0), seed=st.integers(0, 2**32 - 1), kind=st.sampled_from(KINDS))
    def one(B, n, F, K, kf, e, seed, kind):
        KF = min(kf, F)
        eb = float(np.float32(10.0 ** e))
        host = make_fields(n, F, eb, seed, kind)
        check_case(gpz, orc, host, eb, B=B, K=K, KF=KF, label=f"random {kind}")

    one()
