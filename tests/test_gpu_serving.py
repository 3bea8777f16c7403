"""Serving form: continuous batching must give every request exactly the
result the CPU oracle computes for it alone (the relative bound of a
compression's own slice, its stream bytes and size; decoded bits and a
clean status of a decompression), and admission must respect the HBM
budget."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_10305_amd as gpz
    from paper_2508_10305_amd import serve
    gpz.lib()
    pools = serve.build_pools(200_000, seed=3)
    sizes = serve.template_sizes(2_000, 200_000, count=4)
    templates = serve.build_templates(pools, sizes)
    reqs = serve.make_requests(pools, templates, sizes, 80, seed=9, rate=40_000.0, n_min=2_000,
                               n_max=200_000)
    return gpz, serve, reqs


def oracle_result(orc, r):
    """What the request computes, by the CPU oracle on host copies of its
    input: the stream of its slice (compress) or the decoded template
    (decompress)."""
    if r.op == "compress":
        host = [f.cpu().numpy() for f in r.fields]
        # the relative bound of the request's own slice, by the oracle
        eb = orc.rel_ebs(host, r.rel) if r.rel else r.eb
        assert (eb.view(np.uint32) == r.eb.view(np.uint32)).all(), f"request {r.rid}: bound"
        s, _ = orc.compress(host, eb)
        return s
    return orc.decompress(r.stream.cpu().numpy(), r.n, r.F)


def snapshot(results):
    """on_done callback: keep a host copy of each result, with the size and
    status the server recorded, before its buffer is reused."""
    def keep(r):
        if r.op == "compress":
            results[r.rid] = (r.out.cpu().numpy().copy(), r.nbytes, r.status)
        else:
            results[r.rid] = ([o.cpu().numpy().copy() for o in r.out], r.nbytes, r.status)
    return keep


def check_same(orc, reqs, results):
    for r in reqs:
        ref = oracle_result(orc, r)
        got, nbytes, status = results[r.rid]
        if r.op == "compress":
            assert nbytes == ref.size, f"request {r.rid}: size {nbytes} != oracle {ref.size}"
            assert (got[: ref.size] == ref).all(), f"request {r.rid}: stream differs in the mix"
        else:
            assert status == 0, f"request {r.rid}: decoder flagged the stream"
            for f in range(r.F):
                assert (got[f].view(np.uint32) == ref[f].view(np.uint32)).all(), f"request {r.rid}"


@pytest.mark.parametrize("mode", ["batched", "per_request"])
def test_each_result_same_alone_and_in_the_mix(setup, orc, mode):
    gpz, serve, reqs = setup
    srv = serve.Server(4 << 30, nstreams=3, max_jobs=16, max_blocks=1 << 14)
    rs = serve.fresh(reqs)
    print(f"[case] serving {mode}", flush=True)
    results = {}
    st = srv.run(rs, mode=mode, on_done=snapshot(results))
    torch.cuda.synchronize()
    check_same(orc, rs, results)
    assert st["requests"] == len(reqs)
    if mode == "batched":
        assert max(srv.batch_sizes) > 1, "no request was batched with another"
    srv.close()


def test_admission_respects_budget_and_queues(setup):
    gpz, serve, reqs = setup
    # a budget that holds only a few requests at a time
    budget = 24 << 20
    srv = serve.Server(budget, nstreams=2, max_jobs=8, max_blocks=1 << 12)
    rs = serve.fresh(reqs)
    print("[case] serving overload", flush=True)
    st = srv.run(rs, mode="batched")
    assert st["arena_peak_bytes"] <= srv.arena.size
    queued = [r for r in rs if r.t_admit > r.t + 1e-4]
    assert queued, "a small budget must make admission wait"
    assert st["requests"] == len(reqs)
    srv.close()
