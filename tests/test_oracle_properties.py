"""Property tests of the oracle on random small inputs (hypothesis): for any
block size, segment bits, key-field count, bound and value mix, every
invariant the method fixes must hold -- the header describes the input,
the stream never exceeds the all-raw size, decompression respects the bound
(non-finite values bit-exact), the permutation stays inside its block, each
coded block comes out stably sorted by segment ID (Sec. 4.2, checked with
numpy's stable argsort on IDs recomputed from the quantized values), raw
blocks keep input order, and compression is deterministic.  Inputs are
float32 or float64 (Sec. 5.1), and the value mixes include ranges that need
64-bit grid indices (Sec. 5.3) and float64 values finer than float32."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

KINDS = ("uniform", "clustered", "specials", "constant", "wide", "ongrid", "widegrid")


@st.composite
def cases(draw):
    B = draw(st.sampled_from([64, 128, 256, 512, 1024, 2048, 4096]))
    n = draw(st.integers(0, min(5000, 3 * B + 7)))
    F = draw(st.integers(1, 8))
    K = draw(st.integers(0, 5))
    KF = draw(st.integers(1, min(F, 3)))
    eb = float(np.float32(10.0 ** draw(st.floats(-6.0, -1.0))))
    seed = draw(st.integers(0, 2**32 - 1))
    kind = draw(st.sampled_from(KINDS))
    f64 = draw(st.booleans())
    if f64 and draw(st.booleans()):
        eb = float(np.float32(10.0 ** draw(st.floats(-12.0, -7.0))))  # below float32 spacing
    return B, n, F, K, KF, eb, seed, kind, f64


def make_fields(n, F, eb, seed, kind, f64=False):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(F):
        if kind == "uniform":
            x = rng.random(n)
        elif kind == "clustered":
            c = rng.random(8)
            x = c[rng.integers(0, 8, n)] + rng.normal(0, 1e-3, n)
        elif kind == "specials":
            x = rng.normal(0, 1, n)
            m = rng.random(n)
            x[m < 0.05] = np.nan
            x[(m >= 0.05) & (m < 0.08)] = np.inf
            x[(m >= 0.08) & (m < 0.1)] = -np.inf
            x[(m >= 0.1) & (m < 0.15)] = 0.0
            x[(m >= 0.15) & (m < 0.2)] = -0.0
            x[(m >= 0.2) & (m < 0.22)] = 1e-42  # denormal
        elif kind == "constant":
            x = np.full(n, rng.normal())
        elif kind == "wide":
            x = rng.normal(0, 1, n) * 10.0 ** rng.integers(-3, 30, n)
        elif kind == "widegrid":  # small values beside a few far ones: > 2^24 grid steps
            x = rng.random(n)
            m = rng.random(n) < 0.02
            x[m] = rng.integers(1, 9, int(m.sum())) * 2.0 ** 22
        else:  # (near) the grid of the bound
            k = rng.integers(0, 4000, n).astype(np.float64)
            x = k * (2.0 * float(np.float32(eb))) + rng.normal()
        if f64:
            x = np.asarray(x, dtype=np.float64) * (1.0 + rng.random(n) * 2.0 ** -30)
            out.append(np.asarray(x, dtype=np.float64))
        else:
            out.append(np.asarray(x, dtype=np.float32))
    return out


def record_modes(stream, n, F, B):
    w = stream.view(np.uint32)
    nb = -(-n // B)
    ns = -(-nb // 64)
    lens = w[8 + 2 * ns + F: 8 + 2 * ns + F + nb]
    off = 8 + 2 * ns + F + nb
    modes = []
    for L in lens:
        modes.append(int(w[off]) & 3)
        off += int(L)
    return modes


@settings(max_examples=400, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(cases())
def test_oracle_invariants(orc, case):
    B, n, F, K, KF, eb, seed, kind, f64 = case
    fields = make_fields(n, F, eb, seed, kind, f64)
    s, perm = orc.compress(fields, eb, B=B, K=K, KF=KF, want_perm=True)
    s2, _ = orc.compress(fields, eb, B=B, K=K, KF=KF, want_perm=True)
    assert (s == s2).all(), "compression is not deterministic"
    info = orc.inspect(s)
    assert (info["n"], info["F"], info["B"], info["K"], info["KF"]) == (n, F, B, K, KF)
    assert info["nblocks"] == -(-n // B) and info["bytes"] == s.size
    assert info["flags"] & 1 == int(f64)
    assert s.size <= orc.max_bytes(n, F, B, f64)
    out = orc.decompress(s, n, F, f64=f64)
    if f64:
        for f in range(F):
            x = fields[f][perm.astype(np.int64)]
            same = out[f].view(np.uint64) == x.view(np.uint64)
            with np.errstate(invalid="ignore"):
                assert (same | (np.abs(out[f] - x) <= float(np.float32(eb)))).all()
    else:
        viol, _ = orc.bound_check(fields, out, eb, perm=perm)
        assert int(viol.sum()) == 0
    if n == 0:
        return
    perm = perm.astype(np.int64)
    j = np.arange(n)
    assert (perm // B == j // B).all(), "permutation leaves its block"
    ut = np.uint64 if f64 else np.uint32
    for f in range(F):
        src = fields[f][perm]
        nf = ~np.isfinite(src)
        assert (out[f][nf].view(ut) == src[nf].view(ut)).all()
    modes = record_modes(s, n, F, B)
    for b, mode in enumerate(modes):
        lo, hi = b * B, min(n, (b + 1) * B)
        p = perm[lo:hi] - lo
        assert sorted(p.tolist()) == list(range(hi - lo))
        if mode == 1:
            assert (p == np.arange(hi - lo)).all(), "raw block not in input order"
            continue
        tr = orc.block_trace([f[lo:hi] for f in fields], eb, K=K, KF=KF)
        ids = np.zeros(hi - lo, np.int64)
        for ax in range(KF):
            seg = tr["q"][ax].astype(np.int64) >> int(tr["s"][ax])
            ids = (ids << K) | seg
        assert (p == np.argsort(ids, kind="stable")).all(), f"block {b} not stably sorted"
