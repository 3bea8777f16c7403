"""Storage orders of the synthetic workloads: the local orders are
permutations of the drawn sets that group each cluster (halo) together with
the background last, or sweep LiDAR strips serpentine; md's other order is a
seeded shuffle.  Pure input generation (no GPU)."""
import numpy as np
import pytest

from paper_2508_10305_amd import synth


@pytest.mark.parametrize("kind", ["clusters", "cosmology", "md", "lidar"])
@pytest.mark.parametrize("order", ["local", "shuffled"])
def test_orders_are_permutations(kind, order):
    n = 50_000
    a = synth.make(kind, n, 3)
    b = synth.make(kind, n, 3, order=order)
    assert len(a) == len(b)
    # the same particles: sort the rows of (field 0, field 1, ...) records
    ra = np.rec.fromarrays(a)
    rb = np.rec.fromarrays(b)
    assert np.array_equal(np.sort(ra), np.sort(rb))
    assert synth.make(kind, n, 3, order=order)[0].tobytes() == b[0].tobytes()  # seeded


def test_cluster_major_order_groups_labels():
    n = 40_000
    lab = np.empty(n, np.int32)
    f = synth.cosmology(n, seed=5, n_halos=32, labels=lab)
    perm = synth.local_order("cosmology", f, lab)
    s = lab[perm]
    assert (np.diff(s) >= 0).all() and s[-1] == 32  # halo-major, background last
    # each halo keeps its draw order
    for h in (0, 7, 31):
        idx = perm[s == h]
        assert (np.diff(idx) > 0).all()


def test_lidar_strips_serpentine():
    f = synth.lidar(30_000, seed=4)
    perm = synth.local_order("lidar", f)
    x, y = f[0][perm], f[1][perm]
    strip = np.floor(y.astype(np.float64) / 10.0).astype(np.int64)
    assert (np.diff(strip) >= 0).all()
    for k in np.unique(strip)[:20]:
        xs = x[strip == k]
        d = np.diff(xs)
        assert (d >= 0).all() if k % 2 == 0 else (d <= 0).all()
