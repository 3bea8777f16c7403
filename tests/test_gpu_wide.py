"""GPU parity for the 64-bit grid steps (Sec. 5.3), float64 fields (Sec. 5.1)
and the block sizes outside 256..2048, all through the C ABI, against the
CPU oracle: stream bytes, permutations and decoded bits must be identical
(no tolerance: both sides take the same IEEE float and double operations).
The wave-per-block kernels hand the blocks that need 64-bit steps to the
generic ones, so mixed snapshots cover the hand-off in both directions."""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden")


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


def widegrid(n, F, seed, frac=0.02):
    """Values in [0, 1) with a few multiples of 2^22 in some blocks: those
    blocks span more than 2^24 grid steps at small bounds."""
    rng = np.random.default_rng(seed)
    out = []
    for f in range(F):
        x = rng.random(n)
        blk = (np.arange(n) // 1024) % 3 == f % 3  # every third block of this field
        m = (rng.random(n) < frac) & blk
        x[m] = rng.integers(1, 9, int(m.sum())) * 2.0 ** 22
        out.append(x.astype(np.float32))
    return out


def check_f64(gpz, orc, host, eb, B=1024, K=3, KF=None, label=""):
    n, F = host[0].size, len(host)
    say(f"[case] f64 {label} n={n} F={F} B={B} K={K} KF={KF}")
    ref, ref_perm = orc.compress(host, eb, B=B, K=K, KF=KF, want_perm=True)
    dev = [torch.from_numpy(np.ascontiguousarray(h)).cuda() for h in host]
    got, perm = gpz.compress_f64(dev, eb, block_size=B, seg_bits=K, key_fields=KF,
                                 want_perm=True)
    g = got.cpu().numpy()
    assert g.size == ref.size, f"{label}: size {g.size} != oracle {ref.size}"
    if not (g == ref).all():
        bad = np.nonzero(g.view(np.uint32) != ref.view(np.uint32))[0]
        raise AssertionError(f"{label}: {bad.size} words differ, first at word {bad[0]}")
    assert (perm.cpu().numpy().astype(np.uint32) == ref_perm).all(), f"{label}: perm"
    ref_out = orc.decompress(ref, n, F, f64=True)
    out = gpz.decompress_f64(got, n, F)
    for f in range(F):
        a = out[f].cpu().numpy().view(np.uint64)
        assert (a == ref_out[f].view(np.uint64)).all(), f"{label}: decoded field {f}"
    outl, raw = gpz.stream_stats(got, n, F)
    routl, rraw = orc.stream_stats(ref, n, F)
    assert outl.tolist() == routl.tolist() and raw == rraw, f"{label}: stream stats"
    return ref


@pytest.mark.parametrize("B", [256, 1024, 2048])
def test_wide_range_blocks_f32(gpz, orc, B):
    """Blocks whose grid needs more than 24 bits, mixed with blocks that do
    not, key and attribute fields, a partial last block: the wave-per-block
    encoder leaves the wide ones to the generic encoder and the decoder
    leaves their records to the generic decoder."""
    from test_gpu_parity import check_case
    n = 9 * 1024 + 517
    # seven fields: three key axes, the three attribute fields the encoder
    # quantizes with the keys, and one it quantizes in its field loop
    host = widegrid(n, 7, seed=B)
    eb = np.array([2.0 ** -12, 2.0 ** -11, 1e-4, 2.0 ** -10, 3e-5, 1e-4, 2.0 ** -12], np.float32)
    ref = check_case(gpz, orc, host, eb, B=B, KF=3, label=f"wide B={B}")
    assert (ref.view(np.uint32)[1] >> 17) & 1, "no wide record in the case"


@pytest.mark.parametrize("B", [64, 128, 4096])
def test_generic_block_sizes(gpz, orc, B):
    """Block sizes outside 256..2048 run the generic kernels whole: clusters,
    special values and wide blocks, ragged sizes."""
    from paper_2508_10305_amd import synth
    from test_gpu_parity import check_case
    for n in (1, B - 1, 3 * B + 5):
        host = synth.clusters(max(n, 1), seed=n + B)
        host[1][::97] = np.nan
        host[2][5::131] = np.inf
        check_case(gpz, orc, host, 1e-4, B=B, label=f"generic B={B} n={n}")
    host = widegrid(5 * B + 3, 3, seed=B)
    check_case(gpz, orc, host, 2.0 ** -12, B=B, label=f"generic wide B={B}")


@pytest.mark.parametrize("B", [256, 1024, 4096])
def test_f64_downcast_and_wide(gpz, orc, B):
    """Float64 fields: float32 values (down-cast meets the bound), values
    below float32 resolution at a bound float32 cannot meet (64-bit steps),
    special values with NaN payloads, and a per-block mix of both regimes."""
    rng = np.random.default_rng(B)
    n = 7 * B + 301
    f32vals = (rng.random(n) * 100.0).astype(np.float32).astype(np.float64)
    fine = 1.0 + rng.integers(0, 2 ** 20, n) * 2.0 ** -35 + rng.random(n) * 2.0 ** -40
    spec = rng.normal(0, 1, n)
    spec[::53] = np.nan
    spec.view(np.uint64)[7::211] = 0x7FF0000000000ABC  # signalling NaN payload
    spec[11::97] = -np.inf
    spec[13::89] = -0.0
    mix = np.where((np.arange(n) // B) % 2 == 0, f32vals, fine)
    check_f64(gpz, orc, [f32vals, fine, spec, mix], np.array([1e-3, 2.0 ** -38, 1e-6, 2.0 ** -38],
                                                            np.float32), B=B, label="mix")
    # one field only, K and KF variations
    check_f64(gpz, orc, [fine], 2.0 ** -30, B=B, K=5, KF=1, label="one field")
    check_f64(gpz, orc, [f32vals, spec], 1e-2, B=B, K=0, KF=2, label="K=0")


def test_f64_wide_range(gpz, orc):
    """Float64 values spanning more than 2^24 grid steps and values beyond
    2^53 steps (outliers), at the default block size."""
    rng = np.random.default_rng(77)
    n = 3 * 1024 + 9
    x = rng.random(n) * 1e6
    y = rng.random(n)
    y[::101] = 1e30  # beyond 2^53 steps above the block minimum: outliers
    check_f64(gpz, orc, [x, y, x * -3.0], 1e-6, label="wide range")


def test_golden_wide_blocks_decode_on_gpu(gpz, orc):
    """The hand-derived wide and float64 blocks (tests/golden/wide_blocks.json)
    decode on the GPU to the hand-derived values, and the GPU writes the
    hand-derived stream for each."""
    with open(os.path.join(GOLD, "wide_blocks.json")) as fh:
        blocks = json.load(fh)["blocks"]
    for blk in blocks:
        f64 = blk["dtype"] == "float64"
        dt = np.float64 if f64 else np.float32
        fields = []
        for v in blk["fields"]:
            a = np.array([np.nan if x == "nan" else x for x in v], dt)
            if f64 and "nan_bits64" in blk:
                a.view(np.uint64)[np.isnan(a)] = blk["nan_bits64"]
            fields.append(a)
        want = np.array(blk["stream_words"], np.uint32)
        dev = [torch.from_numpy(a).cuda() for a in fields]
        n = fields[0].size
        if f64:
            got, _ = gpz.compress_f64(dev, blk["eb"], block_size=blk["B"], seg_bits=blk["K"],
                                      key_fields=blk["KF"])
        else:
            got, _ = gpz.compress(dev, blk["eb"], block_size=blk["B"], seg_bits=blk["K"],
                                  key_fields=blk["KF"])
        assert got.cpu().numpy().view(np.uint32).tolist() == want.tolist(), blk["name"]
        s = torch.from_numpy(want.view(np.uint8).copy()).cuda()
        out = (gpz.decompress_f64 if f64 else gpz.decompress)(s, n, len(fields))
        ref = orc.decompress(want.view(np.uint8), n, len(fields), f64=f64)
        ut = np.uint64 if f64 else np.uint32
        for o, r in zip(out, ref):
            assert (o.cpu().numpy().view(ut) == r.view(ut)).all(), blk["name"]


def test_wide_record_without_header_flag_is_corrupt(gpz, orc):
    """A record with a wide field in a stream whose header does not announce
    one is corrupt: the synchronous decoder returns GPZ_ECORRUPT, the
    asynchronous one raises its error flag, as the oracle rejects it.  A
    float64 stream handed to the float32 decoder (and the reverse) is an
    argument error."""
    host = widegrid(4 * 1024, 3, seed=5)
    s, _ = orc.compress(host, 2.0 ** -12)
    w = s.view(np.uint32).copy()
    assert (w[1] >> 17) & 1
    w[1] &= ~np.uint32(2 << 16)
    assert orc.decompress_status(w.view(np.uint8), host[0].size, 3) == orc.ECORRUPT
    d = torch.from_numpy(w.view(np.uint8).copy()).cuda()
    with pytest.raises(gpz.GpzError) as e:
        gpz.decompress(d, host[0].size, 3)
    assert e.value.code == gpz.GPZ_ECORRUPT
    out = [torch.empty(host[0].size, dtype=torch.float32, device="cuda") for _ in range(3)]
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    gpz.decompress_async(d, host[0].size, 3, out, err, gpz.params(3))
    torch.cuda.synchronize()
    assert int(err.item()) != 0
    # the intact stream decodes through the asynchronous path too
    d2 = torch.from_numpy(s.copy()).cuda()
    gpz.decompress_async(d2, host[0].size, 3, out, err, gpz.params(3))
    ref = orc.decompress(s, host[0].size, 3)
    assert int(err.item()) == 0
    for o, r in zip(out, ref):
        assert (o.cpu().numpy().view(np.uint32) == r.view(np.uint32)).all()
    # value type mismatches
    x64 = [torch.from_numpy(h.astype(np.float64)).cuda() for h in host]
    s64, _ = gpz.compress_f64(x64, 1e-3)
    with pytest.raises(gpz.GpzError) as e:
        gpz.decompress(s64, host[0].size, 3)
    assert e.value.code == gpz.GPZ_EINVAL
    with pytest.raises(gpz.GpzError) as e:
        gpz.decompress_f64(d2, host[0].size, 3)
    assert e.value.code == gpz.GPZ_EINVAL


def test_batch_with_wide_jobs(gpz, orc):
    """A batch whose jobs mix wide-range snapshots with ordinary ones: the
    batched generic walks code and decode the wide blocks; every job's
    stream and decoded bits equal the oracle's."""
    from paper_2508_10305_amd import synth
    from test_gpu_batch import build_batch, check_batch, oracle_results
    jobs = [(widegrid(5 * 1024 + 3, 3, seed=1), 2.0 ** -12),
            (synth.clusters(7000, seed=3), 1e-4),
            (widegrid(2 * 1024, 4, seed=2), 2.0 ** -11)]
    ref = oracle_results(orc, jobs)
    assert sum(int((r[0].view(np.uint32)[1] >> 17) & 1) for r in ref) == 2
    for grid in (97, 0):
        from paper_2508_10305_amd.batch import default_config
        cfg = default_config()
        cfg.grid = grid
        say(f"[case] batch wide grid={grid}")
        b, fields, outs, decs, ebs = build_batch(gpz, jobs, cfg)
        b.compress()
        b.decompress()
        check_batch(b, outs, decs, ref, f"wide batch grid={grid}")
        b.close()


def test_batch_wide_jobs_beyond_the_first_256(gpz, orc):
    """300 jobs, wide ones among the first 256 and past them: the batched
    walk over blocks left to the generic encoder reads the jobs' deferred
    counts 256 at a time, and every group must be walked."""
    from paper_2508_10305_amd import synth
    from test_gpu_batch import build_batch, check_batch, oracle_results
    rng = np.random.default_rng(7)
    jobs = []
    for j in range(300):
        if j in (3, 255, 256, 290):
            jobs.append((widegrid(2 * 1024 + 5 * j % 97, 3, seed=100 + j), 2.0 ** -12))
        else:
            n = int(rng.integers(100, 3000))
            jobs.append((synth.clusters(n, seed=1000 + j), float(rng.choice([1e-3, 1e-4]))))
    ref = oracle_results(orc, jobs)
    wide = [j for j, r in enumerate(ref) if (r[0].view(np.uint32)[1] >> 17) & 1]
    assert wide == [3, 255, 256, 290]
    from paper_2508_10305_amd.batch import default_config
    for grid in (97, 0):
        cfg = default_config()
        cfg.grid = grid
        say(f"[case] batch of 300 with wide jobs grid={grid}")
        b, fields, outs, decs, ebs = build_batch(gpz, jobs, cfg)
        b.compress()
        b.decompress()
        check_batch(b, outs, decs, ref, f"300 jobs grid={grid}")
        b.close()
