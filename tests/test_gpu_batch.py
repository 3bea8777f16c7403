"""Batched form: every job of a batch must produce exactly the stream (and
decompressed floats) the CPU oracle computes for that snapshot alone, with or
without graph capture, on every graph replay, and after rebinding to new
jobs."""
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


def make_jobs(seed, sizes, fields_per_job=None):
    from paper_2508_10305_amd import synth
    rng = np.random.default_rng(seed)
    jobs = []
    for i, n in enumerate(sizes):
        F = fields_per_job[i] if fields_per_job else int(rng.integers(3, 7))
        host = synth.clusters(n, seed=seed * 1000 + i, n_clusters=int(rng.integers(8, 1025)),
                              extra_fields=F - 3) if n else [np.zeros(0, np.float32)] * F
        eb = float(np.exp(rng.uniform(np.log(1e-5), np.log(1e-2))))
        jobs.append((host, eb))
    return jobs


def oracle_results(orc, jobs):
    """Each job's stream and decoded fields from the CPU oracle: the batched
    form is compared with what the method computes (Sec. 4.1-4.4, and the
    reverse of Sec. 3.2), not with another GPU path."""
    ref = []
    for host, eb in jobs:
        n = host[0].size
        s, _ = orc.compress(host, eb)
        out = orc.decompress(s, n, len(host))
        ref.append((s, out))
    return ref


def build_batch(gpz, jobs, config=None, **kw):
    from paper_2508_10305_amd.batch import Batch
    fields, outs, decs, ebs = [], [], [], []
    for host, eb in jobs:
        n, F = host[0].size, len(host)
        fields.append([torch.from_numpy(np.ascontiguousarray(f)).cuda() for f in host])
        outs.append(torch.zeros(gpz.max_compressed_bytes(n, F, kw.get("p")), dtype=torch.uint8,
                                device="cuda"))
        decs.append([torch.full((max(n, 1),), np.nan, dtype=torch.float32, device="cuda")[:n]
                     for _ in range(F)])
        ebs.append(eb)
    b = Batch(fields, ebs, outs, dec=decs, config=config, **kw)
    return b, fields, outs, decs, ebs


def check_batch(b, outs, decs, ref, label):
    sizes = b.sizes()
    assert (b.errors() == 0).all(), label
    for j, (rs, rout) in enumerate(ref):
        assert int(sizes[j]) == rs.size, f"{label}: job {j} size"
        got = outs[j][: rs.size].cpu().numpy()
        assert (got == rs).all(), f"{label}: job {j} stream bytes differ"
        for f, ro in enumerate(rout):
            d = decs[j][f].cpu().numpy()
            assert (d.view(np.uint32) == ro.view(np.uint32)).all(), f"{label}: job {j} field {f}"


@pytest.mark.parametrize("use_graph", [0, 1])
@pytest.mark.parametrize("grid,tile", [(97, 1), (97, 3), (0, 1)])
def test_batch_equals_plain(gpz, orc, use_graph, grid, tile):
    """grid 97: an odd persistent grid, blocks shared unevenly between waves;
    grid 0: one workgroup per block."""
    from paper_2508_10305_amd.batch import default_config
    sizes = [1, 1023, 1024, 1025, 5000, 0, 70_000, 200_001, 64 * 1024 + 7, 3]
    jobs = make_jobs(7, sizes)
    ref = oracle_results(orc, jobs)
    cfg = default_config()
    cfg.use_graph = use_graph
    cfg.tile = tile
    cfg.grid = grid
    say(f"[case] batch graph={use_graph} grid={grid} tile={tile}")
    b, fields, outs, decs, ebs = build_batch(gpz, jobs, cfg)
    b.compress()
    b.decompress()
    check_batch(b, outs, decs, ref, f"graph={use_graph} grid={grid} tile={tile}")
    b.close()


def test_batch_matches_oracle(gpz, orc):
    """Batched compression and decompression, each job against the oracle:
    stream bytes and size, then decoded bits, with no error flag."""
    jobs = make_jobs(11, [3000, 10_000, 1024 * 5], fields_per_job=[3, 5, 6])
    b, fields, outs, decs, ebs = build_batch(gpz, jobs)
    b.compress()
    b.decompress()
    check_batch(b, outs, decs, oracle_results(orc, jobs), "oracle")
    b.close()


@pytest.mark.parametrize("grid,tile", [(97, 3), (0, 1)])
def test_batch_non_finite_blocks(gpz, orc, grid, tile):
    """The batched encoders share the plain one's block minimum over finite
    values (Sec. 4.1).  Jobs whose blocks each hold one arrangement of
    non-finite values (a single NaN of either sign, -inf, +inf, all NaN, a
    negative NaN in the first or last position) must give the oracle's
    stream, in the persistent and the one-workgroup-per-block launches."""
    from paper_2508_10305_amd.batch import default_config
    bits = lambda u: np.array([u], np.uint32).view(np.float32)[0]
    specials = [None, bits(0x7FC00000), bits(0xFFC00001), bits(0xFF800001), -np.inf, np.inf,
                "all", 0, 1023]
    rng = np.random.default_rng(41)
    jobs = []
    for n, F in [(9 * 1024, 6), (5 * 1024 + 300, 4), (2000, 3)]:
        host = []
        for f in range(F):
            x = (rng.standard_normal(n) * 5 - 2).astype(np.float32)
            for b in range(-(-n // 1024)):
                lo, hi = b * 1024, min(n, (b + 1) * 1024)
                c = specials[(b + f) % len(specials)]
                if c is None:
                    continue
                if isinstance(c, str):
                    x[lo:hi] = bits(0xFFC00001)
                elif isinstance(c, int):
                    if lo + c < hi:
                        x[lo + c] = bits(0xFFC00001)
                else:
                    x[lo + int(rng.integers(0, hi - lo))] = c
            host.append(x)
        jobs.append((host, 1e-3))
    cfg = default_config()
    cfg.grid = grid
    cfg.tile = tile
    say(f"[case] batch non-finite blocks grid={grid} tile={tile}")
    b, fields, outs, decs, ebs = build_batch(gpz, jobs, cfg)
    b.compress()
    sizes = b.sizes()
    assert (b.errors() == 0).all()
    for j, (host, eb) in enumerate(jobs):
        ref, _ = orc.compress(host, eb)
        got = outs[j][: int(sizes[j])].cpu().numpy()
        assert got.size == ref.size and (got == ref).all(), f"job {j} differs from the oracle"
    b.close()


def test_graph_replays_with_eager_work_between(gpz, orc):
    jobs = make_jobs(13, [50_000, 8_000, 120_000])
    ref = oracle_results(orc, jobs)
    b, fields, outs, decs, ebs = build_batch(gpz, jobs)
    for rep in range(4):
        for o in outs:
            o.zero_()
        for d in decs:
            for t in d:
                t.fill_(float("nan"))
        say(f"[case] graph replay {rep}")
        b.compress()
        # eager work of the program between replays
        x = torch.randn(1 << 20, device="cuda")
        torch.cuda.synchronize()
        _ = (x * 2).sum().item()
        gpz.compress([t for t in fields[1]], ebs[1])
        b.decompress()
        check_batch(b, outs, decs, ref, f"replay {rep}")
    b.close()


@pytest.mark.parametrize("grid", [2048, 0])
def test_rebind_keeps_graphs_valid(gpz, orc, grid):
    from paper_2508_10305_amd.batch import default_config
    jobs_a = make_jobs(17, [30_000, 2_000, 9_000])
    jobs_b = make_jobs(19, [100_000, 1_500])
    ref_b = oracle_results(orc, jobs_b)
    total_blocks = sum((h[0].size + 1023) // 1024 for h, _ in jobs_a + jobs_b)
    cfg = default_config()
    cfg.grid = grid
    # the capacity exceeds both job lists: direct launches exit past them
    b, *_ = build_batch(gpz, jobs_a, cfg, max_jobs=8, max_blocks=total_blocks + 37)
    b.compress()
    b.decompress()
    torch.cuda.synchronize()
    # new jobs, same batch object and captured graphs
    fields, outs, decs, ebs = [], [], [], []
    for host, eb in jobs_b:
        n, F = host[0].size, len(host)
        fields.append([torch.from_numpy(np.ascontiguousarray(f)).cuda() for f in host])
        outs.append(torch.zeros(gpz.max_compressed_bytes(n, F), dtype=torch.uint8, device="cuda"))
        decs.append([torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(F)])
        ebs.append(eb)
    ws = torch.empty(b.workspace_bytes(fields, ebs, outs, decs), dtype=torch.uint8, device="cuda")
    say(f"[case] rebind grid={grid}")
    b.rebind(fields, ebs, outs, dec=decs, workspace=ws)
    b.compress()
    b.decompress()
    check_batch(b, outs, decs, ref_b, "rebind")
    b.close()


def test_rebinds_back_to_back_on_one_stream(gpz, orc):
    """Rebinds queue their table upload on the caller's stream and return
    without waiting for it: three job lists bound, compressed and decompressed
    in a row on one side stream, with no host synchronization of our own,
    must each give the plain results."""
    from paper_2508_10305_amd.batch import Batch, default_config
    lists = [make_jobs(31 + k, sizes) for k, sizes in
             enumerate([[40_000, 3_000], [1_025, 90_000, 7], [64 * 1024, 12_345, 2_048]])]
    refs = [oracle_results(orc, jobs) for jobs in lists]
    cfg = default_config()
    b = Batch.empty(8, 256, config=cfg)
    s = torch.cuda.Stream()
    bound = []
    for k, jobs in enumerate(lists):
        fields, outs, decs, ebs = [], [], [], []
        for host, eb in jobs:
            n, F = host[0].size, len(host)
            fields.append([torch.from_numpy(np.ascontiguousarray(f)).cuda() for f in host])
            outs.append(torch.zeros(gpz.max_compressed_bytes(n, F), dtype=torch.uint8,
                                    device="cuda"))
            decs.append([torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(F)])
            ebs.append(eb)
        ws = torch.empty(Batch.workspace_bytes(fields, ebs, outs, decs), dtype=torch.uint8,
                         device="cuda")
        torch.cuda.synchronize()  # inputs are in place before the side stream starts
        say(f"[case] back-to-back rebind {k}")
        with torch.cuda.stream(s):
            b.rebind(fields, ebs, outs, dec=decs, workspace=ws, stream=s)
            b.compress(stream=s)
            b.decompress(stream=s)
            # this list's results leave the batch's size table before the next rebind
            sizes = b.sizes_device().clone()
        bound.append((outs, decs, sizes, fields, ws))
    torch.cuda.synchronize()
    for k, ((outs, decs, sizes, _, _), ref) in enumerate(zip(bound, refs)):
        sz = sizes.cpu().numpy()
        for j, (rs, rout) in enumerate(ref):
            assert int(sz[j]) == rs.size, f"list {k} job {j} size"
            assert (outs[j][: rs.size].cpu().numpy() == rs).all(), f"list {k} job {j} stream"
            for f, ro in enumerate(rout):
                d = decs[j][f].cpu().numpy()
                assert (d.view(np.uint32) == ro.view(np.uint32)).all(), f"list {k} job {j} f {f}"
    b.close()


def test_batch_reports_corrupt_stream(gpz):
    jobs = make_jobs(23, [20_000, 20_000])
    b, fields, outs, decs, ebs = build_batch(gpz, jobs)
    b.compress()
    sizes = b.sizes()
    # corrupt a record length of job 1 only
    w = outs[1].view(torch.int32)
    nb = (20_000 + 1023) // 1024
    lt = 8 + 2 + len(fields[1])
    w[lt + 3] += 1
    b.decompress()
    err = b.errors()
    assert err[0] == 0 and err[1] != 0
    b.close()


@pytest.mark.parametrize("B", [256, 512, 2048])
@pytest.mark.parametrize("grid", [300, 0])
def test_batch_other_block_sizes(gpz, orc, B, grid):
    """Batched streams and decoded fields equal the oracle's at other block
    sizes too (full and partial blocks, persistent and direct launches)."""
    from paper_2508_10305_amd.batch import default_config
    jobs = make_jobs(29 + B, [B - 1, B, 3 * B + 5, 40_000, 0, 7])
    p = gpz.params(3, block_size=B)
    ref = []
    for host, eb in jobs:
        n = host[0].size
        s, _ = orc.compress(host, eb, B=B)
        ref.append((s, orc.decompress(s, n, len(host))))
    cfg = default_config()
    cfg.grid = grid
    say(f"[case] batch B={B} grid={grid}")
    b, fields, outs, decs, ebs = build_batch(gpz, jobs, cfg, p=p)
    b.compress()
    b.decompress()
    check_batch(b, outs, decs, ref, f"B={B} grid={grid}")
    b.close()
