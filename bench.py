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

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="plain1080",
                   choices=["plain1080", "region4k", "small"])
    p.add_argument("--n-test", type=int, default=None, help="override the number of test frames")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-test", type=int, default=900,
                   help="test frames in the oracle's timed sample")
    p.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "classify_traffic.json"),
                   help="HBM traffic of the classify kernel measured with rocprofv3 counters")
    p.add_argument("--probe", action="store_true",
                   help="only run the streaming probes (read, read+write, 1 GiB copy) and print them")
    return p.parse_args()


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "device.h", "internal.h", "api.hip"):
        with open(os.path.join(ROOT, "paper_1412_1945_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def run_probes(obg, torch, src, nbytes, reps=5):
    """Achievable streaming rates for the classify access pattern (TB/s)."""
    dst = torch.empty(max(nbytes // 24, 1 << 30) + 4096, dtype=torch.uint8, device=src.device)
    sink = torch.empty(512 * 512, dtype=torch.int32, device=src.device)
    out = {}
    for name, kind, n in [("read", obg.PROBE_READ, nbytes), ("read_write", obg.PROBE_READ_WRITE, nbytes),
                          ("copy_1gib", obg.PROBE_COPY, 1 << 30)]:
        times = []
        for r in range(reps + 1):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            obg.obg_probe(kind, src, dst, n, sink, 512)
            b.record()
            torch.cuda.synchronize()
            if r:
                times.append(a.elapsed_time(b))
        ms = min(times)
        moved = n * (2 if kind == obg.PROBE_COPY else 1) + (n // 24 if kind == obg.PROBE_READ_WRITE else 0)
        out[name] = {"ms": round(ms, 4), "tb_s": round(moved / (ms * 1e-3) / 1e12, 3)}
    return out


def workload(name, n_test):
    from synth import frames as S
    if name == "plain1080":
        return S.cfg1(n_test=n_test or 1000)
    if name == "region4k":
        return S.cfg2(n_test=n_test or 500)
    return S.cfg0()


def cpu_baseline(host_train, host_test, spec, depth, num, den, region):
    """The oracle as it is, single-threaded, on every training frame and a
    sample of test frames of the same workload."""
    from oracle import octree
    t0 = time.perf_counter()
    f = octree.Forest(spec.width, spec.height, depth, region[0], region[1])
    idx = f.add_frames(host_train)
    model = f.merge(idx, num, den)
    for fr in host_test:
        model.classify(fr)
    dt = time.perf_counter() - t0
    px = (len(host_train) + len(host_test)) * spec.pixels
    return {"value": px / dt / 1e9, "unit": "Gpixel/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(host_train)} training frames (trees + merge) and {len(host_test)} test "
                      f"frames (classify) of the same stream, {spec.width}x{spec.height}, "
                      f"{dt:.1f} s single-threaded"}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    from paper_1412_1945_amd import obg
    from synth.frames import make_frames

    obg.load()
    dev = torch.device("cuda:0")
    wl = workload(a.workload, a.n_test)
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
    chunk = 50
    for i in range(0, T + N, chunk):
        ids = list(range(i, min(T + N, i + chunk)))
        make_frames(spec, ids, device=dev, out=frames[ids[0]: ids[-1] + 1])
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
        "probe": probes,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "strip_kernel (classify)",
                     "bytes_per_launch": cls_bytes,
                     "frac_of_read_write_probe": round(achieved / 1000 / probes["read_write"]["tb_s"], 4)},
    }
    if not a.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        ns = min(a.cpu_sample_test, N)
        host_train = list(train.cpu().numpy())
        host_test = list(test[:ns].cpu().numpy())
        out["cpu_baseline"] = cpu_baseline(host_train, host_test, spec, depth, num, den, (rw, rh))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
