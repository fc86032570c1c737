"""Benchmark: train + merge + classify throughput on one MI355X.

One step = the whole hot path over one batch of synthetic frames already
resident in HBM: per-frame trees of the T training frames (obg_train_frame),
the merge (obg_merge) and foreground detection of the test frames
(obg_classify).  The default workload is one 1920x1080 RGB8 stream, depth 5,
T = 50 training + 1000 test frames, merge threshold 1/2.

Prints one JSON line (see the fields below).  `value` counts every pixel the
step touches (training and test frames) per second.  The classify kernel is
also timed on its own with HIP events on the stream it runs on; `roofline`
relates its algorithmic bytes (3 B of RGB read + 1/8 B of mask written per
pixel) to MI355X's 8 TB/s.  `cpu_baseline` times the CPU oracle on a bounded
sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="plain1080",
                   choices=["plain1080", "region4k", "small", "batched", "served"])
    p.add_argument("--streams", type=int, default=64, help="streams of the batched workload")
    p.add_argument("--n-test", type=int, default=None, help="override the number of test frames")
    p.add_argument("--depth", type=int, default=None, choices=range(1, 9), metavar="1..8",
                   help="one-stream workloads: override the tree depth (the timed step and the roofline line "
                        "then describe that depth)")
    p.add_argument("--serve-seconds", type=float, default=60.0,
                   help="simulated seconds of arrivals in the real-time served run")
    p.add_argument("--serve-capacity-seconds", type=float, default=10.0,
                   help="seconds of arrivals offered all at once to measure the served capacity")
    p.add_argument("--serve-budget-gib", type=float, default=32.0)
    p.add_argument("--serve-regions", type=int, default=0,
                   help="serve this many 3840x2160 streams with 32x32 regions (d=4, T=30) instead of the mix")
    p.add_argument("--serve-inflight", type=int, default=3,
                   help="batches on the device at once in the real-time served run")
    p.add_argument("--serve-capacity-inflight", type=int, default=1,
                   help="batches on the device at once in the capacity run (1: the path kernels' time is not "
                        "shared with the frame source)")
    p.add_argument("--serve-batch", type=int, default=1024,
                   help="most frames per batch (served); the capacity run's path rate rises with it up to "
                        "1024-2048 frames (256: 51 %% of 8 TB/s, 1024: 54 %%), real-time batches stay small")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extra-legs", action="store_true",
                   help="plain workloads: skip the batched and served legs that the default run appends")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="time budget of the oracle's timed sample (all training frames, then test frames)")
    p.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "classify_traffic.json"),
                   help="HBM traffic of the classify kernel measured with rocprofv3 counters")
    p.add_argument("--probe", action="store_true",
                   help="only run the streaming probes (read, read+write, 1 GiB copy) and print them")
    p.add_argument("--knob-sweep", action="store_true",
                   help="only time classify and the fused classify + occupancy pass on 1000 frames of the 1080p "
                        "workload over their launch knobs (every setting checked against the default's output)")
    p.add_argument("--probe-sweep", action="store_true",
                   help="only sweep the shaped read and read+write probes over 1000 frames' bytes of the 1080p "
                        "workload (grid, block, groups in flight, item size, phased writes) and print the table")
    return p.parse_args()


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "device.h", "internal.h", "strip_core.h", "api.hip"):
        with open(os.path.join(ROOT, "paper_1412_1945_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def run_probes(obg, torch, src, nbytes, reps=5):
    """Achievable streaming rates for the classify access pattern (TB/s)."""
    dst = torch.empty(max(nbytes // 24, 1 << 30) + 4096, dtype=torch.uint8, device=src.device)
    sink = torch.empty(512 * 512, dtype=torch.int32, device=src.device)
    out = {}
    big = src if src.numel() >= (1 << 30) else torch.empty(1 << 30, dtype=torch.uint8, device=src.device).fill_(7)
    for name, kind, n in [("read", obg.PROBE_READ, nbytes), ("read_write", obg.PROBE_READ_WRITE, nbytes),
                          ("copy_1gib", obg.PROBE_COPY, 1 << 30)]:
        s_in = big if kind == obg.PROBE_COPY else src
        times = []
        for r in range(reps + 1):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            obg.obg_probe(kind, s_in, dst, n, sink, 512)
            b.record()
            torch.cuda.synchronize()
            if r:
                times.append(a.elapsed_time(b))
        ms = min(times)
        moved = n * (2 if kind == obg.PROBE_COPY else 1) + (n // 24 if kind == obg.PROBE_READ_WRITE else 0)
        out[name] = {"ms": round(ms, 4), "tb_s": round(moved / (ms * 1e-3) / 1e12, 3)}
    return out


def probe_sweep(reps=3):
    """The classify access pattern's ceiling: the shaped probes over the bytes
    of 1000 1920x1080 frames (6.22 GB), every launch shape of the sweep, best
    of `reps` timed runs each.  Rates count the bytes read plus, for
    read+write, the 1/24 as many written."""
    import torch
    from paper_1412_1945_amd import obg
    obg.load()
    nbytes = (1000 * 1080 * 5760 // (48 * 4096)) * (48 * 4096)
    src = torch.arange(nbytes // 4, dtype=torch.int32, device="cuda").view(torch.uint8)
    dst = torch.empty(nbytes // 24 + 4096, dtype=torch.uint8, device="cuda")
    sink = torch.empty(4096 * 1024 + 1, dtype=torch.int32, device="cuda")
    ev = lambda: torch.cuda.Event(enable_timing=True)
    rows = []

    def timed(**kw):
        best = None
        for r in range(reps + 1):
            a, b = ev(), ev()
            a.record()
            obg.obg_probe_shaped(src=src, dst=dst, nbytes=nbytes, sink=sink, **kw)
            b.record()
            torch.cuda.synchronize()
            if r:
                t = a.elapsed_time(b)
                best = t if best is None else min(best, t)
        return best

    shapes = []
    for kind in (obg.PROBE_READ, obg.PROBE_READ_WRITE):
        for block in (256, 512, 1024):
            for grid in (256, 512, 1024, 2048, 4096):
                for inflight in (1, 2, 4):
                    for span in (832, 4096):
                        shapes.append(dict(kind=kind, grid=grid, block=block, inflight=inflight, span=span))
    for block, grid in ((512, 256), (512, 512), (256, 512), (256, 1024)):
        for span, phase in ((832, 4), (832, 8), (832, 16), (832, 24), (4096, 2), (4096, 4)):
            shapes.append(dict(kind=obg.PROBE_READ_WRITE, grid=grid, block=block, inflight=1, span=span,
                               phase_items=phase))
    for sh in shapes:
        n = sh["span"] * 48
        used = (nbytes // n) * n
        try:
            ms = timed(**sh)
        except obg.ObgError as e:
            rows.append(dict(sh, error=str(e)))
            continue
        moved = used + (used // 24 if sh["kind"] == obg.PROBE_READ_WRITE else 0)
        rows.append(dict(sh, ms=round(ms, 4), tb_s=round(moved / (ms * 1e-3) / 1e12, 3)))
        print(f"# {rows[-1]}", file=sys.stderr, flush=True)
    best = {k: max((r for r in rows if r.get("kind") == k and "tb_s" in r), key=lambda r: r["tb_s"])
            for k in (obg.PROBE_READ, obg.PROBE_READ_WRITE)}
    print(json.dumps({"probe_sweep": rows, "bytes": nbytes, "best_read": best[obg.PROBE_READ],
                      "best_read_write": best[obg.PROBE_READ_WRITE]}), flush=True)


def knob_sweep(reps=5):
    """Classify and the fused pass (classify + each frame's tree) on 1000 test
    frames of the 1080p d=5 stream, over their launch knobs.  The leaf set is
    the merged one with every other word cleared, so the masks hold both
    classes; every setting's outputs must equal the default's."""
    import itertools
    import torch
    from paper_1412_1945_amd import obg
    from synth import frames as S
    from synth.fast import make_frames_gpu
    obg.load()
    wl = S.cfg1(n_test=1000)
    spec, d, (num, den) = wl.streams[0], wl.depth[0], wl.thr[0]
    g = obg.FrameGeom(spec.width, spec.height, d)
    T, N = spec.n_train, spec.n_test
    fr = torch.empty((T + N, spec.height, spec.row_pitch), dtype=torch.uint8, device="cuda")
    for i in range(0, T + N, 100):
        ids = list(range(i, min(T + N, i + 100)))
        make_frames_gpu(spec, ids, fr[ids[0]: ids[-1] + 1])
    occ, leaf = obg.empty_occ(g, T), obg.empty_leafset(g)
    obg.obg_train_frame(g, fr[:T], T, occ)
    obg.obg_merge(g, occ, T, 0, T, num, den, leaf)
    leaf[:, ::2] = 0
    test = fr[T:]
    ref_m, ref_o = obg.empty_mask(g, N), obg.empty_occ(g, N)
    obg.obg_classify(g, test, N, leaf, ref_m, ref_o)
    mask, occ_out = obg.empty_mask(g, N), obg.empty_occ(g, N)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    nbytes = N * spec.pixels * 3 + N * spec.height * g.mask_row_words * 8

    def run(knobs, fused):
        for k, v in knobs.items():
            obg.obg_tune_set(k, v)
        ts = []
        for r in range(reps + 1):
            a, b = ev(), ev()
            a.record()
            obg.obg_classify(g, test, N, leaf, mask, occ_out if fused else None)
            b.record()
            torch.cuda.synchronize()
            if r:
                ts.append(a.elapsed_time(b))
        for k in knobs:
            obg.obg_tune_set(k, 0)
        same = torch.equal(mask, ref_m) and (not fused or torch.equal(occ_out, ref_o))
        ms = sorted(ts)[len(ts) // 2]
        extra = N * g.words * 4 if fused else 0
        row = dict(knobs, pass_="fused" if fused else "classify", med_ms=round(ms, 4),
                   tb_s=round((nbytes + extra) / (ms * 1e-3) / 1e12, 3), same=same)
        print(f"# {row}", file=sys.stderr, flush=True)
        return row

    rows = []
    for block, wpc, span, inter, stage in itertools.product((256, 512), (1, 2, 3, 4), (512, 832, 1024, 1664),
                                                            (1, 2), (1, 2)):
        if block == 512 and wpc > 2:
            continue
        rows.append(run(dict(classify_block=block, classify_wg_per_cu=wpc, classify_span=span, interleave=inter,
                             mask_stage=stage), False))
    for layout, wpc, span, inter, stage in itertools.product((1, 2), (2, 4), (1024, 2048, 4096, 8192, 32768),
                                                             (1, 2), (1, 2)):
        if layout == 1 and wpc == 4:
            continue
        rows.append(run(dict(layout=layout, occ_wg_per_cu=wpc, fused_span=span, interleave=inter, mask_stage=stage),
                        True))
    print(json.dumps({"knob_sweep": rows}), flush=True)


def workload(name, n_test, depth=None):
    """The one-stream workload; `depth` replaces its tree depth (and the
    depth in its name)."""
    from dataclasses import replace
    from synth import frames as S
    if name == "plain1080":
        wl = S.cfg1(n_test=n_test or 1000)
    elif name == "region4k":
        wl = S.cfg2(n_test=n_test or 500)
    else:
        wl = S.cfg0()
    if depth is None or depth == wl.depth[0]:
        return wl
    return replace(wl, name=wl.name.replace(f"-d{wl.depth[0]}", f"-d{depth}"), depth=[depth] * len(wl.streams))


def host_cpu():
    """Threads the host gives this process (capped by OMP_NUM_THREADS) and the
    CPU's model name."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS", n)))
    except ValueError:
        pass
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return max(n, 1), model


def cpu_baseline(host_train, test_frame, n_test, spec, depth, num, den, region, budget_s,
                 gpu_leaf=None, gpu_mask=None, gpu_classify=None):
    """The oracle as it is, single-threaded: trees of every training frame, the
    merge, then test frames (fetched one at a time) until `budget_s` seconds
    have passed or `n_test` frames are classified.  Two more legs use all the
    host's threads (the oracle's C calls release the GIL): up to 8 test frames
    per thread classified with the same model, and the training frames' trees
    built with the frames dealt to the threads.  They are reported beside the
    single-threaded figure.  With gpu_leaf (the GPU's merged leaf set) and
    gpu_mask(i) (the GPU's mask of test frame i), the oracle's leaf set and
    every mask it computed are compared with them, outside the timed calls.
    With gpu_classify(leaf) (the same classify launch over all test frames
    against another leaf set; returns the GPU's mask of test frame i), the
    oracle's merged tree of another seed's small stream is the model, whose
    masks hold both classes, and 16 test frames are compared whole."""
    from oracle import octree
    t0 = time.perf_counter()
    f = octree.Forest(spec.width, spec.height, depth, region[0], region[1])
    idx = f.add_frames(host_train)
    model = f.merge(idx, num, den)
    t_train = time.perf_counter() - t0
    done = 0
    t_cls = 0.0
    masks_equal = True
    fg_own = 0
    while done < n_test and t_train + t_cls < budget_s:
        fr = test_frame(done)
        t1 = time.perf_counter()
        m = model.classify(fr)
        t_cls += time.perf_counter() - t1
        if gpu_mask is not None:
            masks_equal = masks_equal and bool(np.array_equal(m, gpu_mask(done).reshape(m.shape)))
            fg_own += int(np.unpackbits(m.view(np.uint8)).sum())
        done += 1
    dt = t_train + t_cls
    px = (len(host_train) + done) * spec.pixels
    threads, cpu_model = host_cpu()
    out = {"value": px / dt / 1e9, "unit": "Gpixel/s", "cores": 1, "kind": "oracle",
           "sample": f"{len(host_train)} training frames (trees + merge, {t_train:.1f} s) and {done} test "
                     f"frames (classify, {t_cls:.1f} s) of the same stream, {spec.width}x{spec.height}, "
                     f"single-threaded",
           "train_gpixel_s": round(len(host_train) * spec.pixels / t_train / 1e9, 5),
           "classify_gpixel_s": round(done * spec.pixels / t_cls / 1e9, 5) if done else None,
           "cpu_model": cpu_model, "host_threads": threads}
    if gpu_leaf is not None:
        want = model.leafset()
        out["verified"] = {"leaf_set_equal": bool(np.array_equal(want, gpu_leaf.reshape(want.shape))),
                           "test_frames": done, "masks_equal": masks_equal, "foreground_bits_compared": fg_own}
    if gpu_classify is not None:
        from oracle import models
        other = models.foreign_model(spec.width, spec.height, depth, region[0], region[1])
        g_mask = gpu_classify(models.foreign_leafset(depth, other.n_regions))
        k = min(16, n_test)
        eq, fg = True, 0
        for j in range(k):
            i = j * n_test // k
            want = other.classify(test_frame(i))
            eq = eq and bool(np.array_equal(want, g_mask(i).reshape(want.shape)))
            fg += int(np.unpackbits(want.view(np.uint8)).sum())
        out.setdefault("verified", {})["discriminating"] = {
            "model": f"merged tree of a {models.MODEL_SIDE[depth]}x{models.MODEL_SIDE[depth]} stream of another "
                     f"seed (oracle), same classify launch over all {n_test} test frames",
            "test_frames": k, "masks_equal": eq, "foreground_bits_compared": fg,
            "foreground_fraction": round(fg / (k * spec.pixels), 4)}
    if threads > 1 and done:
        from concurrent.futures import ThreadPoolExecutor
        frames = [test_frame(i) for i in range(min(done, 8 * threads))]
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(model.classify, frames[:threads]))
            t1 = time.perf_counter()
            list(ex.map(model.classify, frames))
            t_mt = time.perf_counter() - t1
            out["threaded_classify"] = {"threads": threads, "frames": len(frames),
                                        "seconds": round(t_mt, 3),
                                        "gpixel_s": round(len(frames) * spec.pixels / t_mt / 1e9, 5)}
            # the training frames' trees, the frames dealt to the threads, each
            # thread building into a forest of its own (the merge needs them in
            # one forest and stays single-threaded)
            parts = [host_train[i::threads] for i in range(threads) if host_train[i::threads]]

            def build(part):
                forest = octree.Forest(spec.width, spec.height, depth, region[0], region[1])
                forest.add_frames(part)
                return forest

            t1 = time.perf_counter()
            forests = list(ex.map(build, parts))
            t_mt = time.perf_counter() - t1
            del forests
            out["threaded_trees"] = {"threads": len(parts), "frames": len(host_train),
                                     "seconds": round(t_mt, 3),
                                     "gpixel_s": round(len(host_train) * spec.pixels / t_mt / 1e9, 5)}
    return out


def batched_leg(a, steps, warmup, verify_oracle=False):
    """64 streams of mixed resolution, depth, T and threshold: the batched form
    (one plan: a persistent launch per step, graph-captured, autotuned on the
    work) against the plain form (one launch per stream and frame) and one
    launch per stream.  Returns the figures as a dict."""
    import ctypes
    import torch
    from paper_1412_1945_amd import obg
    from synth import frames as S
    from synth.fast import make_frames_gpu
    L = obg.load()
    wl = S.cfg3(n_streams=a.streams)
    streams = []
    print(f"# batched: generating {len(wl.streams)} streams on the GPU", file=sys.stderr, flush=True)
    for spec, d, thr in zip(wl.streams, wl.depth, wl.thr):
        g = obg.FrameGeom(spec.width, spec.height, d)
        fr = torch.empty((spec.n_frames, spec.height, spec.row_pitch), dtype=torch.uint8, device="cuda")
        make_frames_gpu(spec, range(spec.n_frames), fr)
        T, N = spec.n_train, spec.n_test
        streams.append({"geom": g, "train": fr[:T], "n_train": T, "thr": thr, "test": fr[T:], "n_test": N,
                        "occ": obg.empty_occ(g, T), "leafset": obg.empty_leafset(g),
                        "mask": obg.empty_mask(g, N), "frames": fr,
                        "p_occ": obg.empty_occ(g, T), "p_leaf": obg.empty_leafset(g), "p_mask": obg.empty_mask(g, N)})
    torch.cuda.synchronize()
    px_train = sum(s["n_train"] * s["geom"].width * s["geom"].height for s in streams)
    px_test = sum(s["n_test"] * s["geom"].width * s["geom"].height for s in streams)
    px = px_train + px_test
    ev = lambda: torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    hs = ctypes.c_void_p(stream.cuda_stream)

    print("# batched: plan create and tune", file=sys.stderr, flush=True)
    plan = obg.obg_plan_create([{"geom": s["geom"], "thr": s["thr"], "max_train": s["n_train"],
                                 "max_test": s["n_test"]} for s in streams])
    items = obg.work_items([dict(s, stream=i) for i, s in enumerate(streams)])
    plan.tune(items)
    info = plan.info()
    for _ in range(warmup):
        plan.run(items)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record(stream)
    for _ in range(steps):
        plan.run(items)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_batched = e0.elapsed_time(e1) / steps
    status_ok = obg.item_status(items) == [obg.ITEM_OK] * len(streams)

    # plain: one call per stream and frame, raw C calls with prepared arguments
    calls = []
    for s in streams:
        g = s["geom"]
        gc = g.c()
        fp = g.frame_pitch
        tr, te = s["train"].data_ptr(), s["test"].data_ptr()
        ow = g.words * 4
        mw = g.height * g.mask_row_words * 8
        calls.append((gc, tr, te, fp, s["p_occ"].data_ptr(), ow, s["p_leaf"].data_ptr(), s["p_mask"].data_ptr(),
                      mw, s["n_train"], s["n_test"], s["thr"]))

    def plain_per_frame(hs=hs):
        for gc, tr, te, fp, occ, ow, leaf, mask, mw, T, N, (num, den) in calls:
            gr = ctypes.byref(gc)
            for f in range(T):
                L.obg_train_frame(gr, tr + f * fp, 1, occ + f * ow, None, hs)
            L.obg_merge(gr, occ, T, 0, T, num, den, leaf, hs)
            for f in range(N):
                L.obg_classify(gr, te + f * fp, 1, leaf, mask + f * mw, None, hs)

    def plain_per_stream():
        for gc, tr, te, fp, occ, ow, leaf, mask, mw, T, N, (num, den) in calls:
            gr = ctypes.byref(gc)
            L.obg_train_frame(gr, tr, T, occ, None, hs)
            L.obg_merge(gr, occ, T, 0, T, num, den, leaf, hs)
            L.obg_classify(gr, te, N, leaf, mask, None, hs)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, (time.perf_counter() - t0) * 1e3 / reps

    print("# batched: plain per frame", file=sys.stderr, flush=True)
    ms_plain, host_plain = timed(plain_per_frame, 2)
    same = all(torch.equal(s["occ"], s["p_occ"]) and torch.equal(s["leafset"], s["p_leaf"])
               and torch.equal(s["mask"], s["p_mask"]) for s in streams)
    def timed_median(fn, reps):
        # each repetition bracketed by its own events: a host stall between
        # launches (the per-stream form issues 3 calls per stream from
        # Python) shows in one repetition, not in the median
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[len(ts) // 2], ts

    print("# batched: plain per stream", file=sys.stderr, flush=True)
    ms_stream, stream_reps = timed_median(plain_per_stream, 5)
    same2 = all(torch.equal(s["mask"], s["p_mask"]) and torch.equal(s["leafset"], s["p_leaf"]) for s in streams)
    bytes_step = 3 * px + px_test // 8 + sum(s["n_train"] * s["geom"].words * 4 for s in streams)
    out = {
        "workload": wl.name, "streams": len(streams),
        "train_gpx": round(px_train / 1e9, 3), "test_gpx": round(px_test / 1e9, 3),
        "ms": round(ms_batched, 3), "gpixel_s": round(px / (ms_batched * 1e-3) / 1e9, 1),
        "plan": info,
        "plain_per_frame": {"ms": round(ms_plain, 3), "host_ms": round(host_plain, 3),
                            "gpixel_s": round(px / (ms_plain * 1e-3) / 1e9, 1),
                            "launches": sum(c[9] + c[10] + 1 for c in calls)},
        "plain_per_stream": {"ms": round(ms_stream, 3), "gpixel_s": round(px / (ms_stream * 1e-3) / 1e9, 1),
                             "ms_reps": [round(t, 3) for t in stream_reps], "statistic": "median of 5"},
        "batched_vs_plain": round(ms_plain / ms_batched, 2),
        "batched_vs_per_stream": round(ms_stream / ms_batched, 2),
        "bit_exact_vs_plain": bool(same and same2 and status_ok),
        "roofline": {"bound": "hbm", "achieved": round(bytes_step / (ms_batched * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(bytes_step / (ms_batched * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "whole batched run (prepare + train + merge + classify)",
                     "bytes": bytes_step},
    }
    if verify_oracle:
        out["cpu_baseline"] = batched_cpu_baseline(streams)
    plan.close()
    del streams, calls
    torch.cuda.empty_cache()
    return out


def batched_cpu_baseline(streams, budget_s=10.0):
    """The oracle on the batched workload, single-threaded, smallest streams
    first until the time budget is spent: each stream's trees and merge, then
    two of its test frames.  Its leaf sets and masks are compared with the
    batched run's outputs (outside the timed calls)."""
    import numpy as np
    from oracle import octree
    t_all = t_run = 0.0
    px = 0
    order = sorted(range(len(streams)), key=lambda i: (streams[i]["geom"].width * streams[i]["geom"].height, i))
    checked, ok, fg = 0, True, 0
    for i in order:
        if t_all > budget_s:
            break
        t0 = time.perf_counter()
        s = streams[i]
        g, T, N = s["geom"], s["n_train"], s["n_test"]
        train = list(s["train"].cpu().numpy())
        tests = [s["test"][t].cpu().numpy() for t in (0, N - 1)]
        t1 = time.perf_counter()
        f = octree.Forest(g.width, g.height, g.depth)
        model = f.merge(f.add_frames(train), *s["thr"])
        masks = [model.classify(x) for x in tests]
        t_run += time.perf_counter() - t1
        px += (T + len(tests)) * g.width * g.height
        ok = ok and bool(np.array_equal(model.leafset(), s["leafset"].cpu().numpy().view(np.uint32)))
        for t, want in zip((0, N - 1), masks):
            ok = ok and bool(np.array_equal(want, s["mask"][t].cpu().numpy().view(np.uint64)))
            fg += int(np.unpackbits(want.view(np.uint8)).sum())
        checked += 1
        t_all += time.perf_counter() - t0
    return {"value": px / t_run / 1e9, "unit": "Gpixel/s", "cores": 1, "kind": "oracle",
            "sample": f"the {checked} smallest streams of the batched workload: trees of all training frames, "
                      f"the merge, and test frames 0 and 199, single-threaded, {t_run:.1f} s",
            "verified": {"streams": checked, "leaf_sets_and_masks_equal": ok, "foreground_bits_compared": fg}}


def run_batched(a):
    out = {"metric": "train+classify Gpixel/s (batched)", "unit": "Gpixel/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u8", "data": "synthetic"}
    b = batched_leg(a, a.steps, a.warmup, verify_oracle=not a.no_cpu_baseline)
    out.update({"value": b["gpixel_s"], "ms_per_step": b["ms"],
                "config": {"workload": b["workload"], "streams": b["streams"], "train_gpx": b["train_gpx"],
                           "test_gpx": b["test_gpx"]},
                "batched": b, "roofline": b["roofline"]})
    print(json.dumps(out), flush=True)


def oracle_served_replay(spec, depth, T, num, den, n_frames, period, window, budget_s, region=(0, 0)):
    """The oracle on one served stream: model from frames 0..T-1, then each
    test frame is classified and kept as a tree; every `period` test frames the
    model is re-merged from the trees of the last `window` frames.  Stops
    after the first test frame that ends past `budget_s` seconds."""
    from oracle import octree
    from synth.frames import make_frames
    t0 = time.perf_counter()
    f = octree.Forest(spec.width, spec.height, depth, region[0], region[1])
    train = make_frames(spec, range(T), device="cpu").numpy()
    model = f.merge(f.add_frames(list(train)), num, den)
    trees, masks = {}, []
    for k in range(T, n_frames):
        fr = make_frames(spec, [k], device="cpu").numpy()[0]
        masks.append(model.classify(fr))
        trees[k] = f.add_frame(fr)
        t = k - T
        if (t + 1) % period == 0:
            model = f.merge([trees[k - window + 1 + j] for j in range(window)], num, den)
        for j in [i for i in trees if i <= k - window]:
            f.drop(trees.pop(j))
        if time.perf_counter() - t0 > budget_s:
            break
    return masks, time.perf_counter() - t0


def served_leg(a):
    """Serving: 256 streams of the mixed workload, Poisson arrivals at 5-30 fps
    each, frames written into HBM by the synthetic source when admitted,
    continuous batching under a 32 GiB budget, re-merge every 100 test frames
    over the last 50.  Two runs: real time (latency at the offered load) and
    every frame offered at once (capacity).  Returns the figures as a dict
    (a full bench line)."""
    import numpy as np
    import torch
    from paper_1412_1945_amd import obg
    from synth import frames as S
    from synth.fast import IngestContext, poisson_arrivals
    obg.load()
    if a.serve_regions:
        import random as _random
        rng = _random.Random("rates/regions")
        specs = [S.StreamSpec(3840, 2160, 30, 0, seed=5, stream=i, bimodal_frac=0.2, drift_amp=0.1,
                              fg="ellipses", fg_coverage=0.10) for i in range(a.serve_regions)]
        depths, thrs = [4] * len(specs), [(1, 2)] * len(specs)
        rates = [rng.uniform(5.0, 30.0) for _ in specs]
        region = (32, 32)
    else:
        specs, depths, thrs, rates = S.cfg4()
        region = (0, 0)
    period, window = 100, 50
    horizon = max(a.serve_seconds, a.serve_capacity_seconds)
    arrivals_all = poisson_arrivals(rates, horizon, seed=4)
    arrivals = [x[x < a.serve_seconds] for x in arrivals_all]
    streams = [{"width": sp.width, "height": sp.height, "depth": d, "n_train": sp.n_train, "thr": thr,
                "region_w": region[0], "region_h": region[1]} for sp, d, thr in zip(specs, depths, thrs)]
    n_frames = [len(x) for x in arrivals]
    n_source = [len(x) for x in arrivals_all]
    # watched stream: the first smallest one, its masks kept for the oracle sample
    small = min(range(len(specs)), key=lambda i: (specs[i].width * specs[i].height, i))
    wmax = max(n_frames[small] - specs[small].n_train, 0)
    print(f"# served: {len(specs)} streams, {sum(n_frames)} frames over {a.serve_seconds} s; "
          f"building the frame source", file=sys.stderr, flush=True)
    ctx = IngestContext(specs, n_source, slots=8)
    budget = int(a.serve_budget_gib * (1 << 30))
    stride = max(n_source)

    def serve(arr, speed, watch, inflight):
        watch = watch and wmax > 0
        sums = np.zeros((len(specs), stride), dtype=np.uint64)
        masks = ([np.zeros((wmax, specs[small].height, (specs[small].width + 63) // 64), dtype=np.uint64)]
                 if watch else [])
        st = obg.obg_serve_run(streams, arr, ctx.fn, ctx.ctx, speed=speed, budget_bytes=budget,
                               max_inflight=inflight, max_batch_frames=a.serve_batch, remerge_period=period,
                               remerge_window=window, checksums=sums,
                               watch=[small] if watch else None, watch_masks=masks,
                               watch_max_frames=wmax if watch else 0)
        return st, sums, masks

    # warm-up: one second of arrivals, offered at once
    serve([x[x < 1.0] for x in arrivals_all], 1e9, False, a.serve_capacity_inflight)
    print("# served capacity run", file=sys.stderr, flush=True)
    cap_arr = [x[x < a.serve_capacity_seconds] for x in arrivals_all]
    cap, cap_sums, _ = serve(cap_arr, 1e9, False, a.serve_capacity_inflight)
    print(f"# served real-time run ({a.serve_seconds} s)", file=sys.stderr, flush=True)
    rt, rt_sums, wmasks = serve(arrivals, 1.0, True, a.serve_inflight)
    ctx.close()
    # frames served in both runs give the same masks
    same = all(np.array_equal(cap_sums[s, :n], rt_sums[s, :n])
               for s in range(len(specs)) for n in [min(len(cap_arr[s]), len(arrivals[s]))])

    def path_bytes(arr):
        b = 0
        for sp, d, x in zip(specs, depths, arr):
            n, T = len(x), sp.n_train
            n_reg = (-(-sp.width // region[0]) * -(-sp.height // region[1])) if region[0] else 1
            words_b = max(4, (1 << (3 * d)) // 8) * n_reg
            px = sp.width * sp.height
            n_test = max(n - T, 0)
            b += n * (3 * px + words_b) + n_test * (sp.height * ((sp.width + 63) // 64) * 8 + words_b)
            merges = (1 if n >= T else 0) + n_test // period
            b += merges * words_b * (window + 1)
        return b

    cap_px = cap["train_pixels"] + cap["test_pixels"]
    rt_px = rt["train_pixels"] + rt["test_pixels"]
    cap_bytes = path_bytes(cap_arr)
    achieved = cap_bytes / cap["path_busy_s"] / 1e9
    out = {
        "metric": "train+classify Gpixel/s (served), p50/p99 frame latency",
        "value": round(cap_px / cap["wall_s"] / 1e9, 3),
        "unit": "Gpixel/s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(cap["wall_s"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": (f"served-{len(specs)}-streams-3840x2160-regions32-d4" if region[0]
                                else f"served-{len(specs)}-streams-mixed"), "streams": len(specs),
                   "fps_range": [5, 30], "offered_gpixel_s": round(sum(r * sp.width * sp.height for r, sp in
                                                                       zip(rates, specs)) / 1e9, 3),
                   "budget_gib": a.serve_budget_gib, "remerge_period": period, "remerge_window": window,
                   "max_inflight_batches": {"realtime": a.serve_inflight, "capacity": a.serve_capacity_inflight},
                   "max_batch_frames": a.serve_batch},
        "capacity": {"simulated_s": a.serve_capacity_seconds, "frames": cap["frames_served"],
                     "gpixel": round(cap_px / 1e9, 2), "wall_s": round(cap["wall_s"], 3),
                     "gpixel_s": round(cap_px / cap["wall_s"] / 1e9, 2),
                     "device_busy_s": round(cap["busy_s"], 3), "path_busy_s": round(cap["path_busy_s"], 3),
                     "path_gpixel_s": round(cap_px / cap["path_busy_s"] / 1e9, 2),
                     "batches": cap["batches"], "merges": cap["merges"],
                     "peak_gib": round(cap["peak_bytes"] / 2 ** 30, 2),
                     "admission_waits": cap["admission_waits"]},
        "realtime": {"simulated_s": a.serve_seconds, "frames": rt["frames_served"],
                     "gpixel": round(rt_px / 1e9, 2), "wall_s": round(rt["wall_s"], 3),
                     "gpixel_s": round(rt_px / rt["wall_s"] / 1e9, 3),
                     "lat_p50_ms": round(rt["lat_p50_ms"], 3), "lat_p99_ms": round(rt["lat_p99_ms"], 3),
                     "lat_max_ms": round(rt["lat_max_ms"], 3), "lat_mean_ms": round(rt["lat_mean_ms"], 3),
                     "batches": rt["batches"], "merges": rt["merges"],
                     "device_busy_frac": round(rt["busy_s"] / rt["wall_s"], 4),
                     "peak_gib": round(rt["peak_bytes"] / 2 ** 30, 2),
                     "admission_waits": rt["admission_waits"]},
        "capacity_vs_realtime_identical": bool(same),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": ("served path in the capacity run: the region passes (trees of training "
                                "frames, classify + trees of test frames) and the merges" if region[0] else
                                "served path in the capacity run: serve_kernel (occupancy of training "
                                "frames, fused classify+occupancy of test frames) and the merges") +
                               ", timed with HIP events on the batch streams",
                     "bytes": cap_bytes},
    }
    if not a.no_cpu_baseline:
        print("# cpu baseline (oracle replay of the watched stream)", file=sys.stderr, flush=True)
        sp = specs[small]
        got, dt = oracle_served_replay(sp, depths[small], sp.n_train, *thrs[small], n_frames[small],
                                       period, window, budget_s=15.0, region=region)
        ok = bool(wmasks) and all(np.array_equal(wmasks[0][i], got[i]) for i in range(len(got)))
        fg = sum(int(np.unpackbits(m.view(np.uint8)).sum()) for m in got)
        px = (sp.n_train + len(got)) * sp.width * sp.height
        out["cpu_baseline"] = {"value": px / dt / 1e9, "unit": "Gpixel/s", "cores": 1, "kind": "oracle",
                               "cpu_model": host_cpu()[1],
                               "sample": f"stream {small} ({sp.width}x{sp.height}, d={depths[small]}): "
                                         f"{sp.n_train} training frames and the first {len(got)} served test "
                                         f"frames with re-merges, {dt:.1f} s single-threaded",
                               "masks_equal_served": bool(ok), "test_frames_compared": len(got),
                               "foreground_bits_compared": fg}
    del ctx
    torch.cuda.empty_cache()
    return out


def run_served(a):
    print(json.dumps(served_leg(a)), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    if a.workload == "batched":
        return run_batched(a)
    if a.workload == "served":
        return run_served(a)
    if a.probe_sweep:
        return probe_sweep()
    if a.knob_sweep:
        return knob_sweep()
    import torch
    from paper_1412_1945_amd import obg
    from synth.frames import make_frames

    obg.load()
    dev = torch.device("cuda:0")
    wl = workload(a.workload, a.n_test, a.depth)
    spec = wl.streams[0]
    depth = wl.depth[0]
    num, den = wl.thr[0]
    rw, rh = wl.region
    g = obg.FrameGeom(spec.width, spec.height, depth, region_w=rw, region_h=rh)
    T, N = spec.n_train, spec.n_test
    print(f"# generating {T}+{N} frames {spec.width}x{spec.height} on the GPU", file=sys.stderr, flush=True)
    frames = torch.empty((T + N, spec.height, spec.row_pitch), dtype=torch.uint8, device=dev)
    if a.probe:
        flat = frames.view(-1)
        nbytes = (N * spec.height * spec.row_pitch // (48 * 512)) * (48 * 512)
        flat.fill_(7)
        print(json.dumps({"probe": run_probes(obg, torch, flat, nbytes), "bytes": nbytes}), flush=True)
        return
    # ground truth of the test frames (the generator's foreground), packed in
    # the mask layout, for Section 5's agreement figures
    truth = torch.zeros((N, spec.height, g.mask_row_words), dtype=torch.int64, device=dev)
    shifts = torch.arange(64, device=dev, dtype=torch.int64)
    chunk = 50
    for i in range(0, T + N, chunk):
        ids = list(range(i, min(T + N, i + chunk)))
        _, tr = make_frames(spec, ids, device=dev, out=frames[ids[0]: ids[-1] + 1], with_truth=True)
        lo = max(ids[0], T)
        if lo <= ids[-1]:
            tb = torch.zeros((len(ids), spec.height, g.mask_row_words * 64), dtype=torch.int64, device=dev)
            tb[:, :, : spec.width] = tr.to(torch.int64)
            packed = (tb.view(len(ids), spec.height, g.mask_row_words, 64) << shifts).sum(-1)
            truth[lo - T: ids[-1] + 1 - T] = packed[lo - ids[0]:]
        del tr
    torch.cuda.synchronize()
    train, test = frames[:T], frames[T:]
    occ = obg.empty_occ(g, T)
    leaf = obg.empty_leafset(g)
    mask = obg.empty_mask(g, N)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        obg.obg_train_frame(g, train, T, occ)
        obg.obg_merge(g, occ, T, 0, T, num, den, leaf)
        if ev is not None:
            ev[0].record(stream)
        obg.obg_classify(g, test, N, leaf, mask)
        if ev is not None:
            ev[1].record(stream)

    print(f"# warmup {a.warmup}", file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()

    # whole steps
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for _ in range(a.steps):
        step()
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_step = t_start.elapsed_time(t_end) / a.steps

    # classify kernel alone, same launches, events on the launching stream
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(a.steps)]
    for ev in evs:
        step(ev)
    torch.cuda.synchronize()
    cls_ms = sorted(e[0].elapsed_time(e[1]) for e in evs)
    cls_avg = sum(cls_ms) / len(cls_ms)

    # agreement with the ground truth (Section 5's background-class figures)
    counts = torch.zeros(3, dtype=torch.int64, device=dev)
    obg.obg_score(g, mask, truth, N, counts)
    tp, fp, fn = (int(v) for v in counts.cpu().tolist())
    tn = N * spec.pixels - tp - fp - fn
    p0 = tn / (tn + fn) if tn + fn else 0.0
    r0 = tn / (tn + fp) if tn + fp else 0.0
    accuracy = {"f0": round(2 * p0 * r0 / (p0 + r0), 6) if p0 + r0 else 0.0, "p0": round(p0, 6),
                "r0": round(r0, 6), "foreground_recall": round(tp / (tp + fn), 4) if tp + fn else None,
                "foreground_precision": round(tp / (tp + fp), 4) if tp + fp else None,
                "truth": "synthetic foreground objects of the generator"}
    del truth

    # the merge alone, and over trees of groups of 5 frames (Section 3)
    def time_merge(group, reps=20):
        leaf_g = obg.empty_leafset(g)
        ts = []
        for r in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            obg.obg_merge_groups(g, occ, T, 0, T, group, num, den, leaf_g)
            e1.record(stream)
            torch.cuda.synchronize()
            if r:
                ts.append(e0.elapsed_time(e1))
        return sorted(ts)[len(ts) // 2]
    merge_ms, merge_g5_ms = time_merge(1), time_merge(5)

    # the fused pass of the serving path: mask and the frame's occupancy in one read
    occ_t = obg.empty_occ(g, N)
    mask_f = obg.empty_mask(g, N)
    fused = []
    for r in range(min(a.steps, 10) + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        obg.obg_classify(g, test, N, leaf, mask_f, occ_t)
        e1.record(stream)
        torch.cuda.synchronize()
        if r:
            fused.append(e0.elapsed_time(e1))
    fused_ms = sum(fused) / len(fused)
    # redraw of the test frames with their own pruned trees (Section 2)
    qout = torch.empty_like(test)
    qts = []
    for r in range(min(a.steps, 10) + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        obg.obg_quantize(g, test, N, qout)
        e1.record(stream)
        torch.cuda.synchronize()
        if r:
            qts.append(e0.elapsed_time(e1))
    q_ms = sorted(qts)[len(qts) // 2]
    del qout
    fused_same = bool(torch.equal(mask_f, mask))
    occ_bytes = N * g.n_regions * g.words * 4

    px_step = (T + N) * spec.pixels
    value = px_step / (ms_step * 1e-3) / 1e9
    cls_bytes = N * (3 * spec.pixels + spec.height * g.mask_row_words * 8)
    achieved = cls_bytes / (cls_avg * 1e-3) / 1e9
    traffic = None
    if os.path.exists(a.traffic_json):
        try:
            tj = json.load(open(a.traffic_json))
            if (tj.get("workload") == wl.name and tj.get("n_test") == N
                    and tj.get("source_hash") == kernel_source_hash()):
                traffic = tj.get("bytes_per_launch")
        except (OSError, ValueError):
            traffic = None
    probes = run_probes(obg, torch, test.reshape(-1), (N * spec.height * spec.row_pitch // (48 * 512)) * (48 * 512))

    out = {
        "metric": "train+classify Gpixel/s",
        "value": round(value, 3),
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": wl.name, "width": spec.width, "height": spec.height,
                   "depth": depth, "train_frames": T, "test_frames": N,
                   "threshold": f"{num}/{den}", "regions": f"{rw}x{rh}" if rw else "none"},
        "classify": {"ms_avg": round(cls_avg, 4), "ms_p50": round(cls_ms[len(cls_ms) // 2], 4),
                     "gpixel_s": round(N * spec.pixels / (cls_avg * 1e-3) / 1e9, 3)},
        "train_merge_ms": round(ms_step - cls_avg, 4),
        "merge": {"ms_p50": round(merge_ms, 4), "groups_of_5_ms_p50": round(merge_g5_ms, 4),
                  "bitset_bytes_read": T * g.n_regions * g.words * 4},
        "accuracy": accuracy,
        "redraw": {"ms_p50": round(q_ms, 4), "gpixel_s": round(N * spec.pixels / (q_ms * 1e-3) / 1e9, 3),
                   "tb_s": round(6 * N * spec.pixels / (q_ms * 1e-3) / 1e12, 3)},
        "classify_occ": {"ms_avg": round(fused_ms, 4),
                         "gpixel_s": round(N * spec.pixels / (fused_ms * 1e-3) / 1e9, 3),
                         "tb_s": round((cls_bytes + occ_bytes) / (fused_ms * 1e-3) / 1e12, 3),
                         "mask_equal_unfused": fused_same},
        "probe": probes,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "strip_kernel (classify)",
                     "bytes_per_launch": cls_bytes,
                     "frac_of_read_write_probe": round(achieved / 1000 / probes["read_write"]["tb_s"], 4)},
    }
    if not a.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        host_train = list(train.cpu().numpy())

        def classify_with(leaf_host):
            leaf_dev = torch.from_numpy(np.ascontiguousarray(leaf_host).view(np.int32)).to(dev)
            mask_f.fill_(-1)
            obg.obg_classify(g, test, N, leaf_dev, mask_f)
            torch.cuda.synchronize()
            return lambda i: mask_f[i].cpu().numpy().view(np.uint64)

        out["cpu_baseline"] = cpu_baseline(host_train, lambda i: test[i].cpu().numpy(), N, spec, depth,
                                           num, den, (rw, rh), a.cpu_seconds,
                                           gpu_leaf=leaf.cpu().numpy().view(np.uint32),
                                           gpu_mask=lambda i: mask[i].cpu().numpy().view(np.uint64),
                                           gpu_classify=classify_with)
    if a.workload == "plain1080" and not a.no_extra_legs:
        # the rest of the metric: batched vs plain (64 streams) and served
        # latency (256 streams), each with its own roofline and oracle check
        del frames, train, test, occ, leaf, mask, occ_t, mask_f
        torch.cuda.empty_cache()
        out["batched"] = batched_leg(a, steps=min(a.steps, 10), warmup=min(a.warmup, 2),
                                     verify_oracle=not a.no_cpu_baseline)
        sv = served_leg(a)
        for k in ("metric", "unit", "n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline",
                  "dtype", "data", "value", "ms_per_step"):
            sv.pop(k, None)
        out["served"] = sv
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
