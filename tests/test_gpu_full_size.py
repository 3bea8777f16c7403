"""GPU parity at the benchmark sizes, whole streams: the cosmology-like
snapshot (64,000,000 x 6, rel eb 1e-3), the molecular-dynamics-like crystal
(32,000,000 x 6) and the LiDAR-like tile (100,000,000 x 3) at rel eb 1e-2,
1e-3 and 1e-4, compressed in the launch configuration the benchmark times.

Every byte of the GPU stream and the permutation must equal the CPU
oracle's, and every decoded float must equal the oracle's decompression bit
for bit.  The oracle runs block-parallel on the host's cores (blocks are
independent, so chunks of blocks framed into one stream give exactly the
stream of one call; the framing is pinned on the CPU)."""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_10305_amd as g
    g.lib()
    return g


_SETS = {}


def workload(kind):
    """Host arrays of one benchmark workload, generated once per module."""
    from paper_2508_10305_amd import synth
    if kind not in _SETS:
        _SETS.clear()  # one large set in host memory at a time
        t0 = time.time()
        if kind == "cosmology":
            _SETS[kind] = synth.cosmology(64_000_000, seed=1)
        elif kind == "md":
            _SETS[kind] = synth.md(200, seed=2)
        else:
            _SETS[kind] = synth.lidar(100_000_000, seed=3)
        say(f"[gen] {kind} {_SETS[kind][0].size} x {len(_SETS[kind])} in "
            f"{time.time() - t0:.1f}s")
    return _SETS[kind]


def full_parity(gpz, orc, kind, rel):
    host = workload(kind)
    n, F = host[0].size, len(host)
    say(f"[case] full {kind} n={n} F={F} rel={rel}")
    dev = [torch.from_numpy(f).cuda() for f in host]
    eb = gpz.rel_ebs(dev, rel)
    assert (eb.view(np.uint32) == orc.rel_ebs(host, rel).view(np.uint32)).all(), "bounds"
    comp = gpz.Compressor(n, F)  # the benchmark's parameters and launches
    stream, perm = comp.compress(dev, eb, want_perm=True)
    got = stream.cpu().numpy()
    gperm = perm.cpu().numpy().astype(np.uint32)
    t0 = time.time()
    ref, ref_perm = orc.compress_parallel(host, eb, want_perm=True)
    say(f"[oracle] compress {time.time() - t0:.1f}s, CR {4 * n * F / ref.size:.3f}")
    assert got.size == ref.size, f"{kind} {rel}: size {got.size} != oracle {ref.size}"
    if not (got == ref).all():
        bad = np.nonzero(got.view(np.uint32) != ref.view(np.uint32))[0]
        raise AssertionError(f"{kind} {rel}: {bad.size} words differ, first at word {bad[0]}")
    assert (gperm == ref_perm).all(), f"{kind} {rel}: permutation"
    del comp, perm
    out = gpz.decompress(stream, n, F)
    t0 = time.time()
    ref_out = orc.decompress_parallel(ref, n, F)
    say(f"[oracle] decompress {time.time() - t0:.1f}s")
    for f in range(F):
        a = out[f].cpu().numpy().view(np.uint32)
        assert (a == ref_out[f].view(np.uint32)).all(), f"{kind} {rel}: decoded field {f}"
    viol, mx = gpz.bound_check(dev, out, eb, perm=torch.from_numpy(ref_perm.view(np.int32)).cuda())
    assert (viol == 0).all() and (mx < eb.astype(np.float64)).all(), f"{kind} {rel}: bound"
    del dev, out, stream
    torch.cuda.empty_cache()


def test_full_size_cosmology(gpz, orc):
    full_parity(gpz, orc, "cosmology", 1e-3)


@pytest.mark.parametrize("rel", [1e-2, 1e-3, 1e-4])
def test_full_size_md(gpz, orc, rel):
    full_parity(gpz, orc, "md", rel)


@pytest.mark.parametrize("rel", [1e-2, 1e-3, 1e-4])
def test_full_size_lidar(gpz, orc, rel):
    full_parity(gpz, orc, "lidar", rel)
