"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle against something the paper or mathematics fixes:
the Sec. 4.2 worked example, streams derived by hand from the format rules,
closed forms (constant and on-grid fields), exact rational arithmetic, and
invariants (error bound, permutation, stream accounting)."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _words(stream):
    return np.frombuffer(np.ascontiguousarray(stream).tobytes(), dtype="<u4")


# ----------------------------------------------------------- worked example


def test_sort_rle_worked_example(orc):
    g = _gold("sort_example.json")
    seg = [p[0] for p in g["input_pairs"]]
    off = [p[1] for p in g["input_pairs"]]
    perm, uniq, cnt, dl = orc.sort_rle(seg)
    assert [[seg[i], off[i]] for i in perm] == g["sorted_pairs"]
    assert perm.tolist() == g["perm"]
    assert uniq.tolist() == g["uniques"]
    assert cnt.tolist() == g["counts"]
    assert dl.tolist() == g["deltas"]


def test_example_stream_by_hand(orc):
    g = _gold("example_stream.json")
    x = np.array(g["x"], np.float32)
    s, perm = orc.compress([x], g["eb"], B=g["B"], K=g["K"], KF=g["KF"], want_perm=True)
    assert _words(s).tolist() == g["stream_words"]
    assert perm.tolist() == g["perm"]
    y = orc.decompress(s, x.size, 1)[0]
    assert y.tolist() == g["decompressed"]
    tr = orc.block_trace([x], g["eb"], K=g["K"], KF=g["KF"])
    assert tr["s"].tolist() == [1]
    assert tr["key"].tolist() == [3, 1, 4, 3, 0] * 3
    assert tr["uniq"].tolist() == [0, 1, 3, 4]
    assert tr["count"].tolist() == [3, 3, 6, 3]


def golden_fields(g, key="fields"):
    """Float32 arrays of a golden file; "nan" entries take the file's NaN bits."""
    out = []
    for v in g[key]:
        a = np.array([np.nan if x == "nan" else x for x in v], np.float32)
        a.view(np.uint32)[np.isnan(a)] = g["nan_bits"]
        out.append(a)
    return out


def test_four_field_block_by_hand(orc):
    """Three key axes and an attribute field, with an exactly half-way value
    (an outlier of a key field) and a NaN (an outlier of an attribute field):
    every stream word, the permutation and the decoded bits were derived by
    hand (tests/golden/four_field_block.json)."""
    g = _gold("four_field_block.json")
    fields = golden_fields(g)
    s, perm = orc.compress(fields, g["eb"], B=g["B"], K=g["K"], KF=g["KF"], want_perm=True)
    assert _words(s).tolist() == g["stream_words"]
    assert perm.tolist() == g["perm"]
    out = orc.decompress(s, fields[0].size, len(fields))
    for got, want in zip(out, golden_fields(g, "decompressed")):
        assert (got.view(np.uint32) == want.view(np.uint32)).all()
    tr = orc.block_trace(fields, g["eb"], K=g["K"], KF=g["KF"])
    assert tr["s"].tolist() == [1, 1, 0]
    assert tr["outlier"][2].nonzero()[0].tolist() == [7]
    assert tr["outlier"][3].nonzero()[0].tolist() == [13]
    assert tr["uniq"].tolist() == [0, 34, 211, 448, 482]
    assert tr["count"].tolist() == [6, 2, 4, 6, 2]


def test_constant_block_by_hand(orc):
    g = _gold("constant_block.json")
    x = np.full(4, 3.0, np.float32)
    s, perm = orc.compress([x], 0.5, B=1024, K=3, KF=1, want_perm=True)
    assert _words(s).tolist() == g["stream_words"]
    assert perm.tolist() == [0, 1, 2, 3]
    tr = orc.block_trace([x], 0.5, K=3, KF=1)
    assert tr["coded_words"] == len(g["coded_record_words"])
    y = orc.decompress(s, 4, 1)[0]
    assert (y == 3.0).all()


# ----------------------------------------------------------- closed forms


@pytest.mark.parametrize("F", [1, 3, 6])
@pytest.mark.parametrize("n", [2, 33, 1024])
def test_constant_field_closed_form(orc, F, n):
    """Constant fields: grid index 0 everywhere, one run, zero-width payloads.
    Coded record = 2 + ceil(bw(n-1)/32) + 2F words; reconstruction exact."""
    c = np.float32(-17.25)
    xs = [np.full(n, c, np.float32) for _ in range(F)]
    tr = orc.block_trace(xs, 1e-3)
    assert tr["U"] == 1 and tr["uniq"].tolist() == [0] and tr["count"].tolist() == [n]
    assert tr["w_gap"] == 0 and tr["w_cnt"] == int(n - 1).bit_length()
    assert (tr["w"] == 0).all() and (tr["q"] == 0).all() and not tr["outlier"].any()
    coded = 2 + (1 if n > 1 else 0) + 2 * F
    assert tr["coded_words"] == coded
    s, perm = orc.compress(xs, 1e-3, want_perm=True)
    w = _words(s)
    rec_len = min(coded, 1 + F * n)
    assert s.size == 4 * (8 + 2 + F + 1 + rec_len)
    ys = orc.decompress(s, n, F)
    for y in ys:
        assert (y.view(np.uint32) == np.float32(c).view(np.uint32)).all()
    assert w[8 + 2 + F] == rec_len


def test_on_grid_field_exact(orc):
    """x = 1 + k * 2^-9 with integer k and eb = 2^-10: every step is exact, so
    there are no outliers and the decompressed bits equal the input bits at
    the permuted positions."""
    rng = np.random.default_rng(7)
    n = 5000
    xs = [(1.0 + rng.integers(0, 1000, n) * 2.0 ** -9).astype(np.float32) for _ in range(3)]
    eb = 2.0 ** -10
    s, perm = orc.compress(xs, eb, want_perm=True)
    ys = orc.decompress(s, n, 3)
    for x, y in zip(xs, ys):
        assert (y.view(np.uint32) == x[perm].view(np.uint32)).all()
    for b in range(0, n, 1024):
        tr = orc.block_trace([x[b:b + 1024] for x in xs], eb)
        assert not tr["outlier"].any()


def test_all_zero_and_negative_zero(orc):
    x = np.array([0.0, -0.0, 0.0, -0.0] * 40, np.float32)
    assert np.float32(orc.block_min(x)).view(np.uint32) == 0  # +0.0
    s, perm = orc.compress([x], 1e-3, want_perm=True)
    y = orc.decompress(s, x.size, 1)[0]
    assert (y == 0).all()


# ----------------------------------------------------------- block minimum rules


def test_block_min_rules(orc):
    nan, inf = np.float32(np.nan), np.float32(np.inf)
    assert orc.block_min(np.array([nan, inf, -inf], np.float32)) == 0.0
    assert orc.block_min(np.array([nan, 5.0, -inf, 2.5, inf], np.float32)) == 2.5
    v = np.float32(orc.block_min(np.array([-0.0, 1.0], np.float32)))
    assert v.view(np.uint32) == 0
    tiny = np.float32(1e-45)  # smallest subnormal
    assert orc.block_min(np.array([1.0, -tiny, 0.0], np.float32)) == -tiny


# ----------------------------------------------------------- quantizer vs exact arithmetic


def _round_f32(fr: Fraction) -> float:
    """Exact round-to-nearest-even of a rational to float32 (normal range)."""
    if fr == 0:
        return 0.0
    sign = -1 if fr < 0 else 1
    a = abs(fr)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -126)
    ulp = Fraction(2) ** (e - 23)
    m = round(a / ulp)  # Fraction round: ties to even
    return sign * float(m * ulp)


@pytest.mark.parametrize("eb", [2.0 ** -14, 1e-6, 3.3e-5])
def test_quantizer_against_exact_rationals(orc, eb):
    """Every third float32 in [1, 1 + 2^-10]: the float32 grid index is within
    1 of the exact nearest index; a value kept on the grid is reconstructed
    (exact fma, one rounding) strictly within eb; a value flagged as an
    outlier has a float32-rounded error of at least eb."""
    eb32 = float(np.float32(eb))
    lo = 1.0
    start = np.float32(1.0).view(np.uint32)
    stop = np.float32(1.0 + 2.0 ** -10).view(np.uint32)
    xs = np.arange(start, stop + 1, dtype=np.uint32).view(np.float32)
    twoeb = Fraction(2) * Fraction(eb32)
    n_out = 0
    for x in xs[::3]:
        x = float(x)
        q, outl = orc.quantize(x, lo, eb32)
        exact = round((Fraction(x) - Fraction(lo)) / twoeb)
        assert abs(q - exact) <= 1
        xr = _round_f32(Fraction(q) * twoeb + Fraction(lo))
        err = abs(Fraction(xr) - Fraction(x))
        if outl:
            assert _round_f32(err) >= eb32
        else:
            assert err < Fraction(eb32)
        n_out += outl
    if eb == 2.0 ** -14:
        # all arithmetic is exact at a power-of-two bound: only exact
        # half-way values (error exactly eb) become outliers
        assert n_out <= xs[::3].size // 16 + 1


def test_quantizer_half_way_value_is_outlier(orc):
    """A value exactly half-way between two grid points has error exactly
    eb: the strict bound stores it verbatim."""
    q, o = orc.quantize(1.0 + 2.0 ** -14, 1.0, 2.0 ** -14)
    assert o


def test_quantizer_range_limit(orc):
    """Grid indices stop at 2^24 - 1 (32-bit intermediates); beyond, the value
    is an outlier with index 0."""
    q, o = orc.quantize(float(2 ** 24 - 1), 0.0, 0.5)
    assert q == 2 ** 24 - 1 and not o
    q, o = orc.quantize(float(2 ** 24), 0.0, 0.5)
    assert q == 0 and o
    for bad in (np.nan, np.inf, -np.inf):
        q, o = orc.quantize(float(bad), 0.0, 0.5)
        assert q == 0 and o


def test_mask_equals_modulo():
    """Table modular_sass: a % 2^s == a & (2^s - 1)."""
    rng = np.random.default_rng(1)
    a = rng.integers(0, 2 ** 24, 10000, dtype=np.uint64)
    for s in range(0, 25):
        assert ((a % (1 << s)) == (a & ((1 << s) - 1))).all()


# ----------------------------------------------------------- invariants


def _specials_field(rng, n):
    x = rng.standard_normal(n).astype(np.float32) * np.float32(10)
    idx = rng.choice(n, 40, replace=False)
    specials = np.array([np.nan, np.inf, -np.inf, -0.0, 0.0, 1e-40, -1e-42, 3e38, -3e38,
                         np.float32(1e-45)], np.float32)
    x[idx] = specials[rng.integers(0, specials.size, idx.size)]
    snan = np.array([0x7F800001, 0xFF812345], np.uint32).view(np.float32)
    x[idx[:2]] = snan
    return x


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_error_bound_invariant_with_specials(orc, seed):
    rng = np.random.default_rng(seed)
    for n, F, eb in [(3000, 3, 1e-3), (1500, 5, 0.25), (2049, 1, 1e-6)]:
        xs = [_specials_field(rng, n) for _ in range(F)]
        s, perm = orc.compress(xs, eb, want_perm=True)
        ys = orc.decompress(s, n, F)
        for x, y in zip(xs, ys):
            xo = x[perm]
            same = xo.view(np.uint32) == y.view(np.uint32)
            with np.errstate(invalid="ignore"):
                err = np.abs(y.astype(np.float64) - xo.astype(np.float64))
            ok = same | (err <= np.float64(np.float32(eb)))
            assert ok.all()
            nonfinite = ~np.isfinite(xo)
            assert same[nonfinite].all()  # non-finite values kept bit-exact


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 1023, 1024, 1025, 3000])
@pytest.mark.parametrize("F", [1, 3, 6])
def test_edge_sizes_and_accounting(orc, n, F):
    rng = np.random.default_rng(n + 7 * F)
    xs = [rng.random(n).astype(np.float32) for _ in range(F)]
    s, perm = orc.compress(xs, 1e-4, want_perm=True)
    w = _words(s)
    nb = (n + 1023) // 1024
    ns = (nb + 63) // 64
    info = orc.inspect(s)
    assert info["n"] == n and info["F"] == F and info["nblocks"] == nb and info["bytes"] == s.size
    lens = w[8 + 2 * ns + F: 8 + 2 * ns + F + nb].astype(np.int64)
    assert s.size == 4 * (8 + 2 * ns + F + nb + int(lens.sum()))
    for b in range(nb):
        nn = min(1024, n - b * 1024)
        assert 1 <= lens[b] <= 1 + F * nn
    assert sorted(perm.tolist()) == list(range(n))
    for b in range(nb):
        blk = perm[b * 1024:(b + 1) * 1024]
        assert ((blk >= b * 1024) & (blk < (b + 1) * 1024)).all()
    ys = orc.decompress(s, n, F)
    for x, y in zip(xs, ys):
        assert (np.abs(y.astype(np.float64) - x[perm].astype(np.float64)) <= np.float32(1e-4)).all()


def test_superblock_offsets_are_prefix_sums(orc):
    rng = np.random.default_rng(3)
    n = 64 * 1024 * 2 + 5000  # > two superblocks
    xs = [rng.random(n).astype(np.float32) for _ in range(3)]
    s, _ = orc.compress(xs, 1e-2)
    w = _words(s)
    nb = (n + 1023) // 1024
    ns = (nb + 63) // 64
    sup = w[8:8 + 2 * ns].astype(np.uint64)
    sup = sup[0::2] | (sup[1::2] << np.uint64(32))
    lens = w[8 + 2 * ns + 3: 8 + 2 * ns + 3 + nb].astype(np.uint64)
    pref = np.concatenate([[0], np.cumsum(lens)])
    assert sup.tolist() == [int(pref[64 * j]) for j in range(ns)]


def test_sort_is_stable_by_segment(orc):
    rng = np.random.default_rng(11)
    pts = [(rng.random(1024) * 0.3).astype(np.float32) for _ in range(3)]
    tr = orc.block_trace(pts, 1e-3)
    order = np.argsort(tr["key"], kind="stable")
    assert (tr["perm"] == order).all()
    sk = tr["key"][tr["perm"]]
    assert (np.diff(sk.astype(np.int64)) >= 0).all()
    assert tr["count"].sum() == 1024
    assert (np.diff(tr["uniq"].astype(np.int64)) > 0).all()
    assert tr["U"] <= min(1024, 2 ** 9)
    # Run-length coding: counts are the histogram of the keys
    h = np.bincount(tr["key"], minlength=512)
    assert (h[tr["uniq"]] == tr["count"]).all() and h.sum() == tr["count"].sum()


def test_segments_partition_range(orc):
    """Each key axis is cut into 2^K power-of-two segments covering the
    block's grid range: segment shift = max(0, bw(qmax) - K)."""
    rng = np.random.default_rng(5)
    for K in range(0, 6):
        pts = [(rng.random(1024) * 10).astype(np.float32) for _ in range(3)]
        tr = orc.block_trace(pts, 1e-3, K=K)
        for a in range(3):
            qmax = int(tr["q"][a].max())
            seg = tr["q"][a] >> tr["s"][a]
            assert int(seg.max()) < 2 ** K or (K == 0 and int(seg.max()) == 0)
            if K >= 1 and qmax >= 2 ** K:
                assert qmax >> int(tr["s"][a]) >= 2 ** (K - 1)  # top segment in use


def test_raw_fallback(orc):
    """Values that are all outliers (grid range far beyond 2^24) cannot be
    coded smaller than raw: blocks are stored verbatim, in input order."""
    rng = np.random.default_rng(9)
    x = [rng.random(2000).astype(np.float32) for _ in range(2)]
    eb = 2.0 ** -100
    s, perm = orc.compress(x, eb, want_perm=True)
    assert (perm == np.arange(2000)).all()
    w = _words(s)
    lens = w[8 + 2 + 2: 8 + 2 + 2 + 2]
    assert lens.tolist() == [1 + 2 * 1024, 1 + 2 * 976]
    ys = orc.decompress(s, 2000, 2)
    for a, b in zip(x, ys):
        assert (a.view(np.uint32) == b.view(np.uint32)).all()


# ----------------------------------------------------------- decoder robustness


def test_decoder_rejects_corruption(orc):
    rng = np.random.default_rng(4)
    n = 5000
    xs = [rng.random(n).astype(np.float32) for _ in range(3)]
    s, _ = orc.compress(xs, 1e-3)
    assert orc.decompress_status(s, n, 3) == 0
    assert orc.decompress_status(s[:-4], n, 3) == orc.ECORRUPT
    bad = s.copy()
    bad[0] ^= 1
    assert orc.decompress_status(bad, n, 3) == orc.ECORRUPT
    bad = s.copy().view(np.uint32)
    bad[8 + 2 + 3] += 1  # first record length
    assert orc.decompress_status(bad.view(np.uint8), n, 3) == orc.ECORRUPT
    assert orc.decompress_status(s, n + 1, 3) == orc.EINVAL
    # random bit flips in the records: either detected or decoded, never a crash
    for t in range(200):
        bad = s.copy()
        pos = rng.integers(4 * (8 + 2 + 3 + 5), s.size)
        bad[pos] ^= np.uint8(1 << rng.integers(0, 8))
        assert orc.decompress_status(bad, n, 3) in (0, orc.ECORRUPT)


def test_invalid_parameters(orc):
    x = [np.zeros(10, np.float32)]
    for kw in [dict(B=100), dict(B=32), dict(K=6), dict(KF=2)]:
        with pytest.raises(orc.OracleError):
            orc.compress(x, 1e-3, **kw)
    for eb in [0.0, -1.0, np.inf, np.nan, 1e-38, 2.0 ** 121]:
        with pytest.raises(orc.OracleError):
            orc.compress(x, eb)


# ----------------------------------------------------------- ranges and relative bounds


def test_field_range_and_relative_bound(orc):
    rng = np.random.default_rng(2)
    x = rng.standard_normal(1000).astype(np.float32)
    x[[3, 9, 77]] = [np.nan, np.inf, -np.inf]
    mm = orc.field_range([x])
    fin = x[np.isfinite(x)]
    assert mm[0, 0] == fin.min() and mm[0, 1] == fin.max()
    e = orc.rel_to_abs(1e-3, float(mm[0, 0]), float(mm[0, 1]))
    rel32 = float(np.float32(1e-3))  # the relative bound is a float32 argument
    assert e == float(np.float32(rel32 * (float(fin.max()) - float(fin.min()))))
    assert orc.rel_to_abs(1e-3, 5.0, 5.0) == float(np.float32(1e-3))


def test_field_range_zero_extremes_are_positive(orc):
    for order in ([-0.0, 0.0], [0.0, -0.0]):
        x = np.array(order * 3 + [np.nan], np.float32)
        mm = orc.field_range([x])
        assert mm.view(np.uint32).tolist() == [[0, 0]]


def test_bound_check_counts_violations(orc):
    x = np.linspace(0, 1, 100).astype(np.float32)
    y = x.copy()
    y[5] += np.float32(0.01)
    y[7] = np.nan
    v, m = orc.bound_check([x], [y], 1e-3)
    assert v.tolist() == [2]
    assert abs(m[0] - abs(float(y[5]) - float(x[5]))) < 1e-12


def test_bound_check_permutation_and_invalid_entries(orc):
    """A reversal permutation pairs recon[j] with orig[n-1-j]; entries outside
    [0, n) count as violations without being read."""
    x = np.arange(8, dtype=np.float32)
    y = x[::-1].copy()
    perm = np.arange(8, dtype=np.uint32)[::-1].copy()
    v, m = orc.bound_check([x], [y], 1e-3, perm=perm)
    assert v.tolist() == [0] and m.tolist() == [0.0]
    v, _ = orc.bound_check([x], [x], 1e-3, perm=perm)  # wrong pairing: 8 pairs off by >= 1
    assert v.tolist() == [8]
    bad = perm.copy()
    bad[[0, 3]] = [8, 0xFFFFFFFF]
    v, m = orc.bound_check([x], [y], 1e-3, perm=bad)
    assert v.tolist() == [2] and m.tolist() == [0.0]


def test_error_stats_closed_form(orc):
    """Every value off by exactly 0.5 over a range of 100: sum of squares
    n/4, NRMSE 0.005, aggregate PSNR 20 log10(200) dB (Sec. 3.1 definition)."""
    n = 101
    x = [np.arange(n, dtype=np.float32), np.linspace(-50, 50, n).astype(np.float32)]
    y = [a + np.float32(0.5) for a in x]
    st = orc.error_stats(x, y)
    assert st["sum_sq"].tolist() == [n * 0.25, n * 0.25]
    assert st["nrmse"].tolist() == [0.005, 0.005]
    assert abs(st["psnr"] - 20 * np.log10(200.0)) < 1e-12
    # one exact field and one off by 0.5: mean NRMSE^2 halves (+3.01 dB)
    st = orc.error_stats(x, [x[0], y[1]])
    assert abs(st["psnr"] - (20 * np.log10(200.0) + 10 * np.log10(2.0))) < 1e-12


def test_error_stats_pairs_like_the_bound_check(orc):
    """Pairs follow the permutation; NaN differences and entries outside
    [0, n) are left out of the sum."""
    x = np.arange(8, dtype=np.float32)
    y = x[::-1] + np.float32(0.25)
    perm = np.arange(8, dtype=np.uint32)[::-1].copy()
    assert orc.error_stats([x], [y], perm=perm)["sum_sq"].tolist() == [8 * 0.0625]
    y2 = y.copy()
    y2[2] = np.nan
    bad = perm.copy()
    bad[5] = 99
    assert orc.error_stats([x], [y2], perm=bad)["sum_sq"].tolist() == [6 * 0.0625]


def test_stream_stats_counts(orc):
    """Non-finite values are outliers of coded blocks (one per value);
    incompressible blocks are raw and count no outliers."""
    n = 3000
    smooth = [np.linspace(0, 1, n).astype(np.float32) for _ in range(3)]
    smooth[1][[5, 1500, 2999]] = [np.nan, np.inf, -np.inf]
    smooth[2][[7]] = [np.nan]
    s, _ = orc.compress(smooth, 1e-3)
    out, raw = orc.stream_stats(s, n, 3)
    assert out.tolist() == [0, 3, 1] and raw == 0
    # a grid finer than 2^53 steps over the block range: every index is out
    # of range even for 64-bit intermediates, every value an outlier, every
    # block raw
    noise = [np.random.default_rng(f).random(n).astype(np.float32) for f in range(3)]
    s, _ = orc.compress(noise, 1e-30)
    out, raw = orc.stream_stats(s, n, 3)
    assert raw == 3 and out.tolist() == [0, 0, 0]


# ----------------------------------------------------------- 64-bit intermediates and float64


def _wide_gold_fields(blk, key):
    """Arrays of one wide_blocks.json block; "nan" entries take its NaN bits."""
    dt = np.float64 if blk["dtype"] == "float64" else np.float32
    out = []
    for v in blk[key]:
        a = np.array([np.nan if x == "nan" else x for x in v], dt)
        if dt == np.float64 and "nan_bits64" in blk:
            a.view(np.uint64)[np.isnan(a)] = blk["nan_bits64"]
        out.append(a)
    return out


@pytest.mark.parametrize("name", ["f32_wide_range", "f64_wide_shift_32", "f64_downcast",
                                  "f64_precision"])
def test_wide_and_float64_blocks_by_hand(orc, name):
    """Sec. 5.3 / Sec. 5.1 extension of the record layout: every stream word,
    the permutation, the field mode and the decoded bits of four blocks were
    derived by hand (tests/golden/wide_blocks.json)."""
    blk = {b["name"]: b for b in _gold("wide_blocks.json")["blocks"]}[name]
    fields = _wide_gold_fields(blk, "fields")
    f64 = blk["dtype"] == "float64"
    if name == "f64_downcast":
        assert fields[0][1] == 0.25 + 2.0 ** -40
    if name == "f64_precision":
        assert fields[0][1] == 1.0 + 2.0 ** -30 and np.float32(blk["eb"]) == 2.0 ** -40
    s, perm = orc.compress(fields, blk["eb"], B=blk["B"], K=blk["K"], KF=blk["KF"],
                           want_perm=True)
    assert _words(s).tolist() == blk["stream_words"]
    assert perm.tolist() == blk["perm"]
    assert orc.inspect(s)["flags"] == int(f64) | (2 if any(blk["wide"]) else 0)
    out = orc.decompress(s, fields[0].size, len(fields), f64=f64)
    want = _wide_gold_fields(blk, "decompressed")
    ut = np.uint64 if f64 else np.uint32
    for got, w in zip(out, want):
        assert got.dtype == w.dtype and (got.view(ut) == w.view(ut)).all()
    tr = orc.block_trace(fields, blk["eb"], K=blk["K"], KF=blk["KF"])
    assert tr["wide"].tolist() == blk["wide"]
    if any(blk["wide"]):
        # a wide record in a stream that does not announce one is corrupt
        bad = _words(s).copy()
        bad[1] &= ~np.uint32(2 << 16)
        assert orc.decompress_status(bad.view(np.uint8), fields[0].size, len(fields),
                                     f64=f64) == orc.ECORRUPT


@pytest.mark.parametrize("eb", [1.3e-5, 2.0 ** -18, 7.7e-7])
def test_wide_quantizer_against_exact_rationals(orc, eb):
    """A grid wider than 2^24 steps (float32 values up to 1000 over the block
    minimum 0): the 64-bit grid index is within 1 of the exact nearest index,
    and the outlier flag is exactly "the float32 value nearest to the exact
    reconstruction q * 2eb + lo (rounded to double, then to float32) is not
    strictly within eb of x" -- evaluated here in exact rationals."""
    eb32 = float(np.float32(eb))
    twoeb = Fraction(2) * Fraction(eb32)
    rng = np.random.default_rng(5)
    xs = np.concatenate([rng.random(1500) * 1000.0, rng.random(500)]).astype(np.float32)
    assert float(xs.max()) / (2 * eb32) > 2 ** 24
    n_out = 0
    for x in xs:
        x = float(x)
        q, outl = orc.quantize_wide(x, 0.0, eb32, True)
        exact = round(Fraction(x) / twoeb)
        assert abs(q - exact) <= 1
        y_exact = Fraction(q) * twoeb
        y64 = float(y_exact)  # correctly rounded to double (int / int division)
        y32 = float(np.float32(y64))  # then to float32 (round to nearest even)
        within = abs(Fraction(y32) - Fraction(x)) < Fraction(eb32)
        assert outl == (not within)
        n_out += outl
    # the small values are resolved by float32; only the large ones may miss
    assert n_out < 1500


def test_wide_range_block_is_coded_not_outliers(orc):
    """A block whose values near its minimum need a grid finer than 2^-24 of
    its range: the 32-bit steps would store every value beyond 2^24 - 1
    steps verbatim (index 0, outlier), the wide steps code them.  Here the
    large values lie exactly on the grid, so none is an outlier and all are
    reconstructed exactly; the small ones are within the bound."""
    eb = 2.0 ** -10
    rng = np.random.default_rng(9)
    x = rng.random(1024).astype(np.float32)
    big = np.arange(1, 17, dtype=np.float64) * 2.0 ** 20
    x[::64] = big.astype(np.float32)
    # under 32-bit steps alone the large values would be outliers
    assert all(orc.quantize(float(v), 0.0, eb)[1] for v in big)
    tr = orc.block_trace([x], eb, K=3, KF=1)
    assert tr["wide"].tolist() == [True]
    assert not tr["outlier"].any()
    s, perm = orc.compress([x], eb, K=3, KF=1, want_perm=True)
    y = orc.decompress(s, x.size, 1)[0]
    src = x[perm]
    d = np.abs(y.astype(np.float64) - src.astype(np.float64))
    assert (d < eb).all()
    assert (y[src >= 2.0 ** 20] == src[src >= 2.0 ** 20]).all()
    outl, raw = orc.stream_stats(s, x.size, 1)
    assert outl.tolist() == [0] and raw == 0


def test_float64_downcast_when_bound_allows(orc):
    """Float64 values that are float32 values.  In a block where the float32
    steps leave no outlier, the down-cast meets the bound: the float64
    stream takes the 32-bit steps there, keeps the block's permutation and
    decodes to the float32 stream's values widened.  In a block where some
    value misses the bound in float32 (near half-way values), the float64
    field goes wide and every value stays within the bound."""
    rng = np.random.default_rng(3)
    B, n = 1024, 5 * 1024
    # blocks 0-2 in [0, 1) (float32 spacing far below eb), 3-4 in [0, 100)
    scale = np.repeat([1.0, 1.0, 1.0, 100.0, 100.0], B)
    x32 = [(rng.random(n) * scale).astype(np.float32) for _ in range(4)]
    x64 = [a.astype(np.float64) for a in x32]
    eb = 1e-3
    s32, p32 = orc.compress(x32, eb, want_perm=True)
    s64, p64 = orc.compress(x64, eb, want_perm=True)
    y32 = orc.decompress(s32, n, 4)
    y64 = orc.decompress(s64, n, 4, f64=True)
    kinds = set()
    for b in range(n // B):
        sl = slice(b * B, (b + 1) * B)
        t32 = orc.block_trace([a[sl] for a in x32], eb)
        t64 = orc.block_trace([a[sl] for a in x64], eb)
        for f in range(4):
            if not t32["outlier"][f].any():
                assert not t64["wide"][f]
                kinds.add("down-cast")
            else:
                assert t64["wide"][f]
                kinds.add("wide")
        if not t64["wide"].any():
            assert (p32[sl] == p64[sl]).all()
            for a, c in zip(y32, y64):
                assert (a[sl].astype(np.float64) == c[sl]).all()
    assert kinds == {"down-cast", "wide"}
    for f in range(4):
        assert (np.abs(y64[f] - x64[f][p64]) < eb).all()


def test_float64_wide_when_float32_cannot_meet_bound(orc):
    """Float64 values spaced below float32 resolution with a bound below it:
    every block takes the wide steps, nothing is an outlier, and every
    decoded value is within the bound of its float64 original (where the
    float32 down-cast alone misses by up to 2^-24 relative)."""
    rng = np.random.default_rng(4)
    n = 3000
    x = [1.0 + rng.integers(0, 2 ** 20, n) * 2.0 ** -35 + rng.random(n) * 2.0 ** -40
         for _ in range(3)]
    eb = 2.0 ** -38
    assert max(abs(float(np.float32(v)) - v) for v in x[0][:200]) > eb
    s, perm = orc.compress(x, eb, want_perm=True)
    for b in range(-(-n // 1024)):
        tr = orc.block_trace([a[b * 1024:(b + 1) * 1024] for a in x], eb)
        assert tr["wide"].all() and not tr["outlier"].any()
    y = orc.decompress(s, n, 3, f64=True)
    for f in range(3):
        assert (np.abs(y[f] - x[f][perm]) < eb).all()
    outl, raw = orc.stream_stats(s, n, 3)
    assert outl.tolist() == [0, 0, 0] and raw == 0


def test_float64_non_finite_bit_exact_and_type_checked(orc):
    """Non-finite float64 values (any NaN payload, +-inf) are outliers stored
    as their 64-bit patterns; a float64 stream read as float32 (or the
    reverse) is refused as an argument error."""
    x = np.linspace(-1, 1, 300)
    bits = x.view(np.uint64)
    bits[[3, 77, 150]] = [0x7FF0000000000001, 0xFFF8DEADBEEF0000, 0x7FF0000000000000]
    x[200] = -np.inf
    s, perm = orc.compress([x, x[::-1].copy()], 1e-4, want_perm=True)
    y = orc.decompress(s, x.size, 2, f64=True)
    src = x[perm]
    nf = ~np.isfinite(src)
    assert nf.sum() == 4
    assert (y[0][nf].view(np.uint64) == src[nf].view(np.uint64)).all()
    assert orc.decompress_status(s, x.size, 2, f64=False) == orc.EINVAL
    s32, _ = orc.compress([x.astype(np.float32)], 1e-4)
    assert orc.decompress_status(s32, x.size, 1, f64=True) == orc.EINVAL
