"""The block-parallel oracle helpers only frame chunks of blocks: their
stream, permutation and decoded fields must equal one whole oracle call, for
snapshots with a ragged last block, several superblocks, every chunking and
a snapshot smaller than one block."""
import numpy as np
import pytest


@pytest.mark.parametrize("n,B,threads", [(300_077, 1024, 7), (70_001, 256, 3), (10, 1024, 4),
                                         (64 * 1024 * 3, 1024, 16)])
def test_parallel_framing_equals_one_call(orc, n, B, threads):
    from paper_2508_10305_amd import synth
    host = synth.clusters(n, seed=n % 97, extra_fields=2)
    host[3][::1000] = np.nan
    ref, ref_perm = orc.compress(host, 1e-4, B=B, want_perm=True)
    got, perm = orc.compress_parallel(host, 1e-4, B=B, threads=threads, want_perm=True)
    assert got.size == ref.size and (got == ref).all()
    assert (perm == ref_perm).all()
    a = orc.decompress(ref, n, len(host))
    b = orc.decompress_parallel(ref, n, len(host), threads=threads)
    for x, y in zip(a, b):
        assert (x.view(np.uint32) == y.view(np.uint32)).all()


def test_parallel_decompress_rejects_bad_superblock_table(orc):
    from paper_2508_10305_amd import synth
    host = synth.clusters(200_000, seed=3)
    s, _ = orc.compress(host, 1e-4)
    bad = s.copy().view(np.uint32)
    bad[8 + 2] += 1  # the second superblock's offset
    with pytest.raises(orc.OracleError):
        orc.decompress_parallel(bad.view(np.uint8), 200_000, 3)
