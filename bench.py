#!/usr/bin/env python3
"""Compress + decompress throughput of the GPZ hot path on one MI355X.

Workload: a cosmology-like snapshot, 64,000,000 particles x 6 float32 SoA
fields (x, y, z, vx, vy, vz), error bound 1e-3 of each field's value range.
A step is one full compression (encode, length scan, record copy) followed by
one full decompression (decode) of the snapshot, inputs resident in HBM.

Prints one JSON line.  ``value`` = 2 * S / step time (original bytes moved
through both directions per second).  ``roofline`` is for the kernel with the
largest share of the step, the encoder, timed with HIP events on its launch
stream during the timed steps (only its launches carry events there); the
other kernels' times come from a second run of the same steps with every
kernel timed.  ``cpu_baseline`` is the CPU oracle on a bounded sample of the
same snapshot, on this host's cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_encode_cosmology64M.md")
ENCODER_SOURCES = ("paper_2508_10305_amd/csrc/encode.hip", "paper_2508_10305_amd/csrc/gpz_internal.h")


def encoder_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in ENCODER_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per encoder launch from the committed counter summary, when
    it was taken on the encoder source as it is now (else None)."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            kv = dict(line[2:].split(": ", 1) for line in f.read().splitlines()
                      if line.startswith("- ") and ": " in line)
        if kv.get("encoder_source_sha256", "").strip() != encoder_source_hash():
            return None
        return int(kv["traffic_bytes_per_launch"].strip())
    except (OSError, KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def kernel_times(gpz, torch, fn, steps):
    """Average per-launch ms of every kernel kind over `steps` calls of fn()."""
    gpz.set_timing(True)
    gpz.timing_collect()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    gpz.set_timing(False)
    return {k: (v[0] / v[1] if v[1] else 0.0) for k, v in gpz.timing_collect().items()}


def workload_figures(gpz, torch, kind, n, seed, rel, steps, warmup):
    """Plain-form figures of one more workload (molecular-dynamics-like or
    LiDAR-like) at a relative bound: step time, compress / decompress rates,
    the encoder's and decoder's HBM roofline fractions, ratio, largest error
    relative to the bound (checked below 1 for every field)."""
    from paper_2508_10305_amd import synth
    host = synth.make(kind, n, seed)
    fields = [torch.from_numpy(f).cuda() for f in host]
    del host
    n, F = fields[0].numel(), len(fields)
    S = 4 * n * F
    eb = gpz.rel_ebs(fields, rel)
    p = gpz.params(F)
    comp = gpz.Compressor(n, F, p)
    outs = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(F)]
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream, perm = comp.compress(fields, eb, want_perm=True)
    C = int(stream.numel())
    gpz.decompress(stream, n, F, out=outs)
    est = gpz.error_stats(fields, outs, eb, perm=perm)
    assert int(est["violations"].sum()) == 0, f"{kind}: bound violated"
    del perm

    def step():
        comp.compress_async(fields, eb)
        gpz.decompress_async(comp.out, n, F, outs, err, p)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    ms = e0.elapsed_time(e1) / steps
    kt = kernel_times(gpz, torch, step, steps)
    nb = (n + p.block_size - 1) // p.block_size
    rec = C - 4 * (8 + 2 * ((nb + 63) // 64) + F + nb)
    t_c = kt["prepare"] + kt["encode"] + kt["scan"] + kt["copy"]
    t_d = kt["decode"] + kt["generic"]
    out = {"n": n, "fields": F, "rel_eb": rel, "ms_per_step": round(ms, 4),
           "GBps": round(2 * S / (ms * 1e-3) / 1e9, 1),
           "compress_GBps": round(S / (t_c * 1e-3) / 1e9, 1),
           "decompress_GBps": round(S / (t_d * 1e-3) / 1e9, 1),
           "encoder_ms": round(kt["encode"], 4), "decoder_ms": round(kt["decode"], 4),
           "encoder_roofline_frac": round((S + rec) / (kt["encode"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
           "decoder_roofline_frac": round((C + S) / (kt["decode"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
           "compression_ratio": round(S / C, 4),
           "max_abs_err_over_eb": float((est["max_abs_err"] / eb.astype(np.float64)).max()),
           "aggregate_psnr_db": round(est["psnr"], 3)}
    del comp, fields, outs, stream
    torch.cuda.empty_cache()
    return out


def batched_figures(gpz, torch, steps):
    """Batched form (256 snapshots, as bench.py --form batched) at the launch
    shape the autotuner picked on this GPU: round time and rate beside the
    loop of plain per-snapshot launches of the same jobs; every stream is
    compared with the plain one."""
    from paper_2508_10305_amd import synth
    from paper_2508_10305_amd.batch import Batch, default_config
    specs = synth.batch_specs(256, seed=4)
    fields = [synth.clusters_device(sp["n"], sp["seed"], sp["clusters"],
                                    extra_fields=sp["fields"] - 3) for sp in specs]
    S = sum(4 * sp["n"] * sp["fields"] for sp in specs)
    ebs = [sp["eb"] for sp in specs]
    p = gpz.params(3)
    outs = [torch.empty(gpz.max_compressed_bytes(sp["n"], sp["fields"], p), dtype=torch.uint8,
                        device="cuda") for sp in specs]
    decs = [[torch.empty(sp["n"], dtype=torch.float32, device="cuda") for _ in range(sp["fields"])]
            for sp in specs]
    comps = [gpz.Compressor(sp["n"], sp["fields"], p) for sp in specs]
    err = torch.zeros(1, dtype=torch.int32, device="cuda")

    def plain_round():
        for j, sp in enumerate(specs):
            comps[j].compress_async(fields[j], ebs[j])
            gpz.decompress_async(comps[j].out, sp["n"], sp["fields"], decs[j], err, p)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    ms_plain = timed(plain_round, 3)
    # the same plain calls captured once in a HIP graph and replayed: the
    # plain form's kernels without the host's launch gaps, the per-byte
    # rate the batched form is compared with
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plain_round()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        plain_round()
    ms_plain_graph = timed(graph.replay, 3)
    ref = []
    for j, sp in enumerate(specs):
        s_, _ = comps[j].compress(fields[j], ebs[j])
        ref.append(s_.clone())
    # every replayed stream is the one the eager call writes
    graph.replay()
    torch.cuda.synchronize()
    graph_same = all(int(comps[j].nbytes_dev.item()) == ref[j].numel() and
                     bool(torch.equal(comps[j].out[: ref[j].numel()], ref[j]))
                     for j in range(len(specs)))
    del graph, comps
    ws = torch.empty(Batch.workspace_bytes(fields, ebs, outs, decs, p), dtype=torch.uint8,
                     device="cuda")
    # launch shape: the autotuner's cached pick for this device and batch
    # shape, else one workgroup per block (its pick on MI355X)
    from paper_2508_10305_amd import autotune
    total_blocks = sum((sp["n"] + 1023) // 1024 for sp in specs)
    key = autotune.shape_key(torch.cuda.get_device_name(0), 1024, total_blocks, len(specs))
    pick = autotune.load_cache().get(key, {"grid": 0, "tile": 1})
    cfg = default_config()
    cfg.grid, cfg.tile, cfg.use_graph = pick["grid"], pick["tile"], 1
    b = Batch(fields, ebs, outs, dec=decs, p=p, config=cfg, workspace=ws)

    def rnd():
        b.compress()
        b.decompress()
    ms = timed(rnd, steps)
    sizes = b.sizes()
    assert (b.errors() == 0).all()
    same = all(int(sizes[j]) == ref[j].numel() and
               bool(torch.equal(outs[j][: ref[j].numel()], ref[j])) for j in range(len(specs)))
    C = int(sizes.sum())
    b.close()
    out = {"snapshots": len(specs), "bytes": S, "ms_per_round": round(ms, 4),
           "GBps": round(2 * S / (ms * 1e-3) / 1e9, 1),
           "roofline_frac": round(2 * (S + C) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
           "plain_loop_ms": round(ms_plain, 4), "speedup_vs_plain_loop": round(ms_plain / ms, 3),
           "plain_graph_ms": round(ms_plain_graph, 4),
           "per_byte_vs_plain_graph": round(ms_plain_graph / ms, 3),
           "plain_graph_streams_identical": graph_same,
           "streams_identical_to_plain": same,
           "launch": {"grid": pick["grid"], "tile": pick["tile"], "graph": 1,
                      "cached_pick": key in autotune.load_cache()}}
    del fields, outs, decs, ws, ref
    torch.cuda.empty_cache()
    return out


def f64_figures(gpz, torch, host, rel, steps):
    """Float64 fields (Sec. 5.1) through the generic kernels: the cosmology
    snapshot's values widened to float64, bounds from the float32 field
    range; compress and decompress rates of the original (float64) bytes."""
    fields = [torch.from_numpy(f).cuda().double() for f in host]
    n, F = fields[0].numel(), len(fields)
    S = 8 * n * F
    eb = gpz.rel_ebs([f.float() for f in fields], rel)
    s, _ = gpz.compress_f64(fields, eb)
    out = gpz.decompress_f64(s, n, F)
    C = int(s.numel())
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(steps):
        gpz.compress_f64(fields, eb)
    e[1].record()
    for _ in range(steps):
        gpz.decompress_f64(s, n, F, out=out)
    e[2].record()
    torch.cuda.synchronize()
    tc, td = e[0].elapsed_time(e[1]) / steps, e[1].elapsed_time(e[2]) / steps
    res = {"n": n, "fields": F, "rel_eb": rel, "compression_ratio": round(S / C, 4),
           "compress_ms": round(tc, 3), "decompress_ms": round(td, 3),
           "compress_GBps": round(S / (tc * 1e-3) / 1e9, 1),
           "decompress_GBps": round(S / (td * 1e-3) / 1e9, 1),
           "note": "host-synchronous calls, each allocating its output and workspace"}
    del fields, out, s
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=64_000_000)
    ap.add_argument("--rel", type=float, default=1e-3)
    ap.add_argument("--cpu-sample-blocks", type=int, default=40000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the extra workloads (md, lidar, float64, batched) and the HBM probes")
    ap.add_argument("--form", choices=["plain", "batched", "serving", "copy", "rd"],
                    default="plain",
                    help="plain per-snapshot launch (default), batched snapshots, serving loop, "
                         "a plain device copy of the snapshot's bytes (HBM reference), or a "
                         "rate-distortion sweep over the synthetic workloads")
    ap.add_argument("--rd-drawn-only", action="store_true",
                    help="rate-distortion form: drawn storage order only")
    ap.add_argument("--batch-grid", type=int, default=0,
                    help="batched form: persistent grid, 0 = one workgroup per block (with "
                         "--batch-tile, skips the autotuner)")
    ap.add_argument("--batch-tile", type=int, default=0)
    ap.add_argument("--jobs", type=int, default=256, help="snapshots of the batched form")
    ap.add_argument("--requests", type=int, default=20_000, help="requests of the serving form")
    ap.add_argument("--serve-streams", type=int, default=3,
                    help="serving form: HIP streams running launches (one more runs the "
                         "field ranges of relative-bound requests)")
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="scales the serving request sizes (1.0: 100K-32M particles)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the compressor is single-GPU (blocks are independent; "
              "see the sharding notes in DESIGN.md). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.form == "batched":
        return bench_batched(args)
    if args.form == "serving":
        from paper_2508_10305_amd import serve
        return serve.bench_main(args, log=log)
    if args.form == "copy":
        return bench_copy(args)
    if args.form == "rd":
        return bench_rd(args)

    import torch

    import paper_2508_10305_amd as gpz
    from paper_2508_10305_amd import synth

    dev = torch.device("cuda:0")
    t0 = time.time()
    host = synth.cosmology(args.n, seed=1)
    log(f"[bench] generated {args.n} x 6 in {time.time() - t0:.1f}s")
    F = len(host)
    n = args.n
    S = 4 * n * F
    fields = [torch.from_numpy(f).to(dev) for f in host]
    torch.cuda.synchronize()

    # value-range-relative bound -> absolute bounds (field range kernel),
    # timed with HIP events over warm calls (a separate pass over the input,
    # not part of the step)
    eb = gpz.rel_ebs(fields, args.rel)
    torch.cuda.synchronize()
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    r0.record()
    for _ in range(5):
        eb2 = gpz.rel_ebs(fields, args.rel)
    r1.record()
    torch.cuda.synchronize()
    range_ms = r0.elapsed_time(r1) / 5
    assert (eb2 == eb).all()

    p = gpz.params(F)
    comp = gpz.Compressor(n, F, p, device=dev)
    outs = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(F)]
    err = torch.zeros(1, dtype=torch.int32, device=dev)

    # correctness gate (untimed): full round trip, bound check
    stream, perm = comp.compress(fields, eb, want_perm=True)
    C = int(stream.numel())
    gpz.decompress(stream, n, F, out=outs)
    est = gpz.error_stats(fields, outs, eb, perm=perm)
    viol, maxerr = est["violations"], est["max_abs_err"]
    assert int(viol.sum()) == 0, f"bound violated: {viol}"
    outl, raw_blocks = gpz.stream_stats(stream, n, F)
    log(f"[bench] S={S} C={C} CR={S / C:.3f} max_err/eb={(maxerr / eb).max():.4f}")
    nb = (n + p.block_size - 1) // p.block_size

    def step():
        comp.compress_async(fields, eb)
        gpz.decompress_async(comp.out, n, F, outs, err, p)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # plain-form per-call latency (host-synchronous compress + decompress)
    lat = []
    for _ in range(max(5, min(args.steps, 20))):
        t0 = time.perf_counter()
        comp.compress(fields, eb)
        gpz.decompress(comp.out[:C], n, F, out=outs)
        lat.append(1e3 * (time.perf_counter() - t0))
    torch.cuda.synchronize()

    # timed region: only the dominant kernel (the encoder) records an event
    # pair, every other launch is as in production
    gpz.set_timing(True, kinds=("encode",))
    gpz.timing_collect()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    gpz.set_timing(False)
    kt = gpz.timing_collect()
    assert int(err.item()) == 0, "decoder flagged the stream"
    ms_step = e0.elapsed_time(e1) / args.steps
    avg = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kt.items()}
    # every kernel's time, in the same steps repeated with all kinds timed
    gpz.set_timing(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    gpz.set_timing(False)
    for k, v in gpz.timing_collect().items():
        if k != "encode" and v[1]:
            avg[k] = v[0] / v[1]
    # "generic": the decoder's walk for records with 64-bit-step fields (it
    # finds none in this snapshot and returns at once); the encoder's walk
    # for such blocks shares the scan's launch
    t_c = avg["prepare"] + avg["encode"] + avg["scan"] + avg["copy"]
    t_d = avg["decode"] + avg["generic"]
    value = 2 * S / (ms_step * 1e-3) / 1e9

    # algorithmic bytes per launch: what each kernel must read and write.  The
    # encoder reads the snapshot and writes the records (C minus the stream's
    # tables) to their slots; the copy reads and writes the records once more.
    rec = C - 4 * (8 + 2 * ((nb + 63) // 64) + F + nb)
    nsup = (nb + 63) // 64
    algo = {"encode": S + rec, "decode": C + S, "prepare": 4 * (2 * nb + 7 + nsup),
            "scan": 12 * nsup, "copy": 2 * rec, "generic": 0}
    dominant = max(avg, key=lambda k: avg[k])
    ach = algo[dominant] / (avg[dominant] * 1e-3) / 1e9
    traffic = None
    if dominant == "encode" and n == 64_000_000 and F == 6 and args.rel == 1e-3:
        traffic = measured_traffic()
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBPS, 4), "traffic": traffic, "kernel": dominant,
                "algorithmic_bytes": algo[dominant]}
    kernels = {k: {"ms": round(avg[k], 4),
                   "algorithmic_GBps": round(algo[k] / (avg[k] * 1e-3) / 1e9, 1)
                   if avg[k] and algo[k] else None}
               for k in avg}

    # The same step captured once in a HIP graph and replayed: the plain
    # calls' launches without the host between them (the async calls are
    # capturable).  Reported beside the eager step, which stays the headline;
    # every replay's stream and decoded fields must equal the eager ones.
    ref_stream = stream.clone()
    ref_outs = [o.clone() for o in outs]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()

    def replay_matches():
        torch.cuda.synchronize()
        return (int(err.item()) == 0 and int(comp.nbytes_dev.item()) == C and
                torch.equal(comp.out[:C], ref_stream) and
                all(torch.equal(o, r) for o, r in zip(outs, ref_outs)))
    graph.replay()
    graph_same = replay_matches()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record()
    for _ in range(args.steps):
        graph.replay()
    g1.record()
    torch.cuda.synchronize()
    graph_ms = g0.elapsed_time(g1) / args.steps
    graph_same = graph_same and replay_matches()
    del graph, ref_outs

    # A/B: single-pass look-back compaction (encoder places its own record)
    # against the default three launches (encode, scan, copy); same stream
    p1 = gpz.params(F, single_pass=True)
    comp1 = gpz.Compressor(n, F, p1, device=dev)
    s1, _ = comp1.compress(fields, eb)
    assert torch.equal(s1, stream), "single-pass compaction wrote a different stream"
    del s1
    for _ in range(args.warmup):
        comp1.compress_async(fields, eb)
    torch.cuda.synchronize()
    gpz.set_timing(True)
    gpz.timing_collect()
    for _ in range(args.steps):
        comp1.compress_async(fields, eb)
    torch.cuda.synchronize()
    gpz.set_timing(False)
    kt1 = gpz.timing_collect()
    avg1 = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kt1.items()}
    t_c1 = avg1["prepare"] + avg1["encode"]
    del comp1
    compaction_ab = {
        "three_step_compress_ms": round(t_c, 4),
        "three_step_kernels_ms": {k: round(avg[k], 4) for k in ("prepare", "encode", "scan",
                                                                 "copy")},
        "single_pass_compress_ms": round(t_c1, 4),
        "single_pass_kernels_ms": {k: round(avg1[k], 4) for k in ("prepare", "encode")},
    }

    cpu = cpu_parallel = None
    if not args.no_cpu_baseline:
        import oracle
        m = min(n, args.cpu_sample_blocks * p.block_size)
        sample = [np.ascontiguousarray(f[:m]) for f in host]
        t0 = time.perf_counter()
        s_ref, _ = oracle.compress(sample, eb)
        t1 = time.perf_counter()
        oracle.decompress(s_ref, m, F)
        t2 = time.perf_counter()
        cpu = {"value": round(2 * 4 * m * F / (t2 - t0) / 1e9, 5), "unit": "GB/s", "cores": 1,
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"first {m} particles ({m // p.block_size} blocks) x {F} fields of the "
                         f"snapshot; compress {t1 - t0:.2f}s + decompress {t2 - t1:.2f}s, "
                         f"single-threaded C"}
        # the same sample split into block-aligned chunks, one oracle call per
        # host thread (blocks are independent; ctypes releases the GIL)
        from concurrent.futures import ThreadPoolExecutor
        # the GPU machine's CPU share for one GPU is 16 threads, whatever nproc shows
        T = max(1, min(16, len(os.sched_getaffinity(0))))
        cb = (m // p.block_size + T - 1) // T * p.block_size
        chunks = [(lo, min(m, lo + cb)) for lo in range(0, m, cb)]

        def one(c):
            part = [np.ascontiguousarray(f[c[0]:c[1]]) for f in sample]
            s_, _ = oracle.compress(part, eb)
            oracle.decompress(s_, c[1] - c[0], F)
        t0 = time.perf_counter()
        with ThreadPoolExecutor(len(chunks)) as ex:
            list(ex.map(one, chunks))
        t3 = time.perf_counter()
        cpu_parallel = {"value": round(2 * 4 * m * F / (t3 - t0) / 1e9, 5), "unit": "GB/s",
                        "cores": len(chunks), "kind": "oracle", "cpu_model": cpu_model(),
                        "nproc": os.cpu_count(),
                        "sample": f"the same {m} particles in {len(chunks)} block-aligned chunks, "
                                  f"one oracle compress + decompress per thread, {t3 - t0:.2f}s"}

    # whole job for a value-range-relative bound: the field range (the bound
    # must reach the host), then compress and decompress, host-synchronous
    for _ in range(2):
        gpz.rel_ebs(fields, args.rel)
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ebx = gpz.rel_ebs(fields, args.rel)
        comp.compress_async(fields, ebx)
        gpz.decompress_async(comp.out, n, F, outs, err, p)
    torch.cuda.synchronize()
    rel_eb_step_ms = 1e3 * (time.perf_counter() - t0) / args.steps

    extra = {}
    if not args.no_extras:
        # achievable HBM rates on this GPU (streaming read and copy probes)
        best, _ = hbm_reference(S, reps=5)
        extra["hbm_reference"] = {"read_GBps": best["read"]["GBps"],
                                  "copy_GBps": best["copy"]["GBps"],
                                  "read4_write1_GBps": best["mix_4r1w"]["GBps"],
                                  "read1_write4_GBps": best["mix_1r4w"]["GBps"],
                                  "read_shape": {k: best["read"][k] for k in ("wg_per_cu", "unroll", "nt")},
                                  "copy_shape": {k: best["copy"][k] for k in ("wg_per_cu", "unroll", "nt")}}
        # the dominant kernels against the probe of their own traffic mix
        extra["vs_mix_probe"] = {
            "encoder": round(kernels["encode"]["algorithmic_GBps"] / best["mix_4r1w"]["GBps"], 4),
            "decoder": round(kernels["decode"]["algorithmic_GBps"] / best["mix_1r4w"]["GBps"], 4)}
        extra["f64_cosmology"] = f64_figures(gpz, torch, host, args.rel, max(3, args.steps // 4))
        del fields, outs, comp, stream, perm
        torch.cuda.empty_cache()
        for key, kind, nn, seed in (("md_32M_x6", "md", 32_000_000, 2),
                                    ("lidar_100M_x3", "lidar", 100_000_000, 3)):
            extra[key] = workload_figures(gpz, torch, kind, nn, seed, args.rel, args.steps,
                                          args.warmup)
            log(f"[bench] {key}: {extra[key]}")
        extra["batched_256"] = batched_figures(gpz, torch, args.steps)
        log(f"[bench] batched: {extra['batched_256']}")

    lat.sort()
    rec = {
        "metric": "compress+decompress GB/s and % HBM roofline at rel eb 1e-3; ratio; p99 latency",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cosmology-like snapshot, 64,000,000 particles x 6 float32 fields, "
                               "rel eb 1e-3 of each field's range, one plain per-snapshot launch",
                   "n": n, "fields": F, "block_size": p.block_size, "seg_bits": p.seg_bits,
                   "rel_eb": args.rel},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_baseline_parallel": cpu_parallel,
        "compress_GBps": round(S / (t_c * 1e-3) / 1e9, 2),
        "decompress_GBps": round(S / (t_d * 1e-3) / 1e9, 2),
        "compression_ratio": round(S / C, 4),
        "max_abs_err_over_eb": float((maxerr / eb.astype(np.float64)).max()),
        "bit_rate_bits_per_value": round(8 * C / (n * F), 4),
        "aggregate_psnr_db": round(est["psnr"], 3),
        "outlier_fraction": float(outl.sum()) / (n * F),
        "raw_blocks": raw_blocks,
        "kernels": kernels,
        "compaction_ab": compaction_ab,
        "graph_replayed_step": {"ms_per_step": round(graph_ms, 4),
                                "GBps": round(2 * S / (graph_ms * 1e-3) / 1e9, 2),
                                "streams_identical_to_eager": graph_same},
        "field_range_ms": round(range_ms, 3),
        "rel_eb_step_ms": round(rel_eb_step_ms, 4),
        **extra,
        "plain_latency_ms": {"p50": round(lat[len(lat) // 2], 3),
                             "p99": round(lat[min(len(lat) - 1, int(0.99 * len(lat)))], 3)},
    }
    print(json.dumps(rec), flush=True)


def bench_rd(args):
    """Rate-distortion sweep (Sec. 3.1's analysis: bit rate against aggregate
    PSNR) over the four synthetic workloads at their full sizes and relative
    bounds 1e-2 ... 1e-5, with compression ratio, outliers and GPU rates."""
    import torch

    import paper_2508_10305_amd as gpz
    from paper_2508_10305_amd import synth
    # drawn storage order (primary), then the other order of each workload
    # (file-like locality; for md, whose drawn order is the lattice order, a
    # shuffle), for compression ratio
    workloads = (("cosmology", 64_000_000, "drawn"), ("md", 32_000_000, "drawn"),
                 ("lidar", 100_000_000, "drawn"), ("clusters", 1_000_000, "drawn"),
                 ("cosmology", 64_000_000, "local"), ("md", 32_000_000, "shuffled"),
                 ("lidar", 100_000_000, "local"), ("clusters", 1_000_000, "local"))
    if args.rd_drawn_only:
        workloads = tuple(w for w in workloads if w[2] == "drawn")
    rels = (1e-2, 1e-3, 1e-4, 1e-5)
    rows = []
    for kind, n, order in workloads:
        t0 = time.time()
        host = synth.make(kind, n, {"clusters": 0, "cosmology": 1, "md": 2, "lidar": 3}[kind],
                          order=order)
        fields = [torch.from_numpy(f).cuda() for f in host]
        del host
        n, F = fields[0].numel(), len(fields)
        S = 4 * n * F
        log(f"[rd] {kind}: {n} x {F} generated in {time.time() - t0:.1f}s")
        p = gpz.params(F)
        comp = gpz.Compressor(n, F, p)
        outs = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(F)]
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        for rel in rels:
            eb = gpz.rel_ebs(fields, rel)
            stream, perm = comp.compress(fields, eb, want_perm=True)
            C = int(stream.numel())
            gpz.decompress(stream, n, F, out=outs)
            st = gpz.error_stats(fields, outs, eb, perm=perm)
            outl, raw_blocks = gpz.stream_stats(stream, n, F)
            assert int(st["violations"].sum()) == 0
            del perm
            reps = 5
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record()
            for _ in range(reps):
                comp.compress_async(fields, eb)
            e[1].record()
            for _ in range(reps):
                gpz.decompress_async(comp.out, n, F, outs, err, p)
            e[2].record()
            torch.cuda.synchronize()
            tc, td = e[0].elapsed_time(e[1]) / reps, e[1].elapsed_time(e[2]) / reps
            row = {"workload": kind, "order": order, "n": n, "fields": F, "rel_eb": rel,
                   "compression_ratio": round(S / C, 3),
                   "bit_rate_bits_per_value": round(8 * C / (n * F), 4),
                   "aggregate_psnr_db": round(st["psnr"], 3),
                   "nrmse": [float(f"{v:.4g}") for v in st["nrmse"]],
                   "outlier_fraction": float(outl.sum()) / (n * F), "raw_blocks": raw_blocks,
                   "compress_GBps": round(S / (tc * 1e-3) / 1e9, 1),
                   "decompress_GBps": round(S / (td * 1e-3) / 1e9, 1)}
            rows.append(row)
            log(f"[rd] {kind} ({order}) rel {rel:g}: CR {row['compression_ratio']} "
                f"{row['bit_rate_bits_per_value']} bits/value PSNR {row['aggregate_psnr_db']} dB")
        del comp, fields, outs
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "rate-distortion: bit rate vs aggregate PSNR", "form": "rd",
                      "data": "synthetic", "rows": rows}), flush=True)


def membench_lib():
    import ctypes
    from paper_2508_10305_amd import build
    L = ctypes.CDLL(build.BENCH_LIB)
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    L.gpzb_read.argtypes = [vp, u64, u32, u32, u32, vp, vp]
    L.gpzb_read.restype = ctypes.c_int
    L.gpzb_copy.argtypes = [vp, vp, u64, u32, u32, u32, vp]
    L.gpzb_copy.restype = ctypes.c_int
    L.gpzb_mix.argtypes = [vp, vp, u64, u32, u32, u32, u32, u32, vp]
    L.gpzb_mix.restype = ctypes.c_int
    return L


def hbm_reference(nbytes: int, reps: int = 10, full: bool = False):
    """Achievable HBM rates on this GPU: the streaming read and copy probes
    (libgpzbench.so) over a buffer of `nbytes`, swept over launch shapes
    (workgroups per CU, loads in flight per lane, cache policy); the best
    shape of each is the reference beside the 8 TB/s peak."""
    import torch
    L = membench_lib()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    x = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").random_()
    y = torch.empty_like(x)
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    per_cu = (1, 2, 4, 8, 16, 32) if full else (2, 4, 8, 16)
    unrolls = (1, 2, 4, 8, 16) if full else (2, 4, 8)
    table = []
    # the encoder's mix (read 4 : write 1) over the whole buffer, the
    # decoder's (read 1 : write 4) writing the whole buffer
    enc_read = nbytes // 65536 * 65536
    dec_read = nbytes // 4 // 65536 * 65536
    for kind in ("read", "copy", "mix_4r1w", "mix_1r4w"):
        for k in per_cu:
            for u in (unrolls if kind in ("read", "copy") else (1, 2, 4)):
                for nt in (0, 1):
                    def call():
                        if kind == "read":
                            rc = L.gpzb_read(x.data_ptr(), nbytes, cus * k, u, nt, sink.data_ptr(), s)
                        elif kind == "copy":
                            rc = L.gpzb_copy(x.data_ptr(), y.data_ptr(), nbytes, cus * k, u, nt, s)
                        elif kind == "mix_4r1w":
                            rc = L.gpzb_mix(x.data_ptr(), y.data_ptr(), enc_read, 4, 1, cus * k, u, nt, s)
                        else:
                            rc = L.gpzb_mix(x.data_ptr(), y.data_ptr(), dec_read, 1, 4, cus * k, u, nt, s)
                        assert rc == 0, rc
                    call()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(reps):
                        call()
                    e1.record()
                    torch.cuda.synchronize()
                    ms = e0.elapsed_time(e1) / reps
                    moved = {"read": nbytes, "copy": 2 * nbytes, "mix_4r1w": enc_read * 5 // 4,
                             "mix_1r4w": dec_read * 5}[kind]
                    table.append({"kind": kind, "wg_per_cu": k, "unroll": u, "nt": nt,
                                  "ms": round(ms, 4), "GBps": round(moved / (ms * 1e-3) / 1e9, 1)})
    best = {kind: max((r for r in table if r["kind"] == kind), key=lambda r: r["GBps"])
            for kind in ("read", "copy", "mix_4r1w", "mix_1r4w")}
    del x, y
    torch.cuda.empty_cache()
    return best, table


def bench_copy(args):
    """Achievable-bandwidth reference: the read and copy probes over the
    snapshot's byte count (6 float32 fields of --n particles), every launch
    shape of the sweep, and a torch device copy for comparison."""
    import torch
    S = 4 * args.n * 6
    best, table = hbm_reference(S, reps=max(5, args.steps), full=True)
    x = torch.empty(S // 4, dtype=torch.float32, device="cuda").uniform_()
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    print(json.dumps({"metric": "achievable HBM GB/s (read; copy = read + write)", "form": "copy",
                      "bytes": S, "best_read": best["read"], "best_copy": best["copy"],
                      "best_read4_write1": best["mix_4r1w"], "best_read1_write4": best["mix_1r4w"],
                      "torch_copy_GBps": round(2 * S / (ms * 1e-3) / 1e9, 2),
                      "sweep": table}), flush=True)


def bench_batched(args):
    """Batched form: snapshots of uneven sizes (log-uniform 10K..8M particles,
    3-6 fields, 8-1024 clusters, abs eb log-uniform 1e-5..1e-2) compressed and
    decompressed by the persistent batched kernels under a HIP graph, with the
    launch geometry picked by the autotuner, against a loop of plain
    per-snapshot launches of the same jobs."""
    import torch

    import paper_2508_10305_amd as gpz
    from paper_2508_10305_amd import autotune, synth
    from paper_2508_10305_amd.batch import Batch, default_config

    specs = synth.batch_specs(args.jobs, seed=4)
    t0 = time.time()
    fields = [synth.clusters_device(sp["n"], sp["seed"], sp["clusters"],
                                    extra_fields=sp["fields"] - 3) for sp in specs]
    torch.cuda.synchronize()
    S = sum(4 * sp["n"] * sp["fields"] for sp in specs)
    log(f"[bench] batched: {len(specs)} snapshots, {sum(sp['n'] for sp in specs)} particles, "
        f"{S / 1e9:.2f} GB, generated in {time.time() - t0:.1f}s")
    ebs = [sp["eb"] for sp in specs]
    p = gpz.params(3)
    outs = [torch.empty(gpz.max_compressed_bytes(sp["n"], sp["fields"], p), dtype=torch.uint8,
                        device="cuda") for sp in specs]
    decs = [[torch.empty(sp["n"], dtype=torch.float32, device="cuda") for _ in range(sp["fields"])]
            for sp in specs]

    # plain per-snapshot loop on the same jobs
    comps = [gpz.Compressor(sp["n"], sp["fields"], p) for sp in specs]
    err = torch.zeros(1, dtype=torch.int32, device="cuda")

    def plain_round():
        for j, sp in enumerate(specs):
            comps[j].compress_async(fields[j], ebs[j])
            gpz.decompress_async(comps[j].out, sp["n"], sp["fields"], decs[j], err, p)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_plain = timed(plain_round, max(1, args.steps // 4))
    ref = [c.out for c in comps]
    ref_sizes = []
    for j, sp in enumerate(specs):
        s_, _ = comps[j].compress(fields[j], ebs[j])
        ref_sizes.append(int(s_.numel()))
    del comps

    ws = torch.empty(Batch.workspace_bytes(fields, ebs, outs, decs, p), dtype=torch.uint8,
                     device="cuda")
    cus = torch.cuda.get_device_properties(0).multi_processor_count

    def run(grid, tile):
        cfg = default_config()
        cfg.grid, cfg.tile, cfg.use_graph = grid, tile, 1
        b = Batch(fields, ebs, outs, dec=decs, p=p, config=cfg, workspace=ws)

        def rnd():
            b.compress()
            b.decompress()
        ms = timed(rnd, 3)
        b.close()
        return ms

    total_blocks = sum((sp["n"] + 1023) // 1024 for sp in specs)
    key = autotune.shape_key(torch.cuda.get_device_name(0), 1024, total_blocks, len(specs))
    if args.batch_tile:  # fixed launch shape (grid 0: one workgroup per block)
        tuned = {"grid": args.batch_grid, "tile": args.batch_tile, "table": []}
    else:
        tuned = autotune.tune(run, cus, key, use_cache=False, log=log)
    cfg = default_config()
    cfg.grid, cfg.tile, cfg.use_graph = tuned["grid"], tuned["tile"], 1
    b = Batch(fields, ebs, outs, dec=decs, p=p, config=cfg, workspace=ws)

    def rnd():
        b.compress()
        b.decompress()
    ms_batch = timed(rnd, args.steps)
    sizes = b.sizes()
    assert (b.errors() == 0).all()
    same = all(int(sizes[j]) == ref_sizes[j] and
               bool(torch.equal(outs[j][: ref_sizes[j]], ref[j][: ref_sizes[j]]))
               for j in range(len(specs)))
    C = int(sizes.sum())
    rec = {
        "metric": "batched compress+decompress GB/s (one launch per stage for all snapshots, replayed from a HIP graph)",
        "form": "batched",
        "value": round(2 * S / (ms_batch * 1e-3) / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "ms_per_step": round(ms_batch, 4),
        "plain_loop_ms": round(ms_plain, 4),
        "plain_loop_GBps": round(2 * S / (ms_plain * 1e-3) / 1e9, 2),
        "speedup_vs_plain_loop": round(ms_plain / ms_batch, 3),
        "streams_identical_to_plain": same,
        "compression_ratio": round(S / C, 4),
        "autotune": {"key": key, "grid": tuned["grid"], "tile": tuned["tile"],
                     "ms": tuned.get("ms"), "table": tuned["table"]},
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(specs)} snapshots, particles log-uniform 10K-8M, 3-6 float32 "
                               "fields, abs eb log-uniform 1e-5..1e-2", "bytes": S},
    }
    print(json.dumps(rec), flush=True)
    b.close()


if __name__ == "__main__":
    main()
