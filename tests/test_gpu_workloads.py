"""The batched and served workloads at their real scale.

Batched: 64 streams of mixed resolution (320x240 .. 3840x2160), depth, T and
threshold, 200 test frames each, in one plan.  Every stream's trees, leaf set
and masks equal one-stream calls; the oracle checks every stream's trees and
leaf set in full, and the masks of one stream per (resolution, depth) pair
(whole frames and sampled pixels of every test frame).  A second run of the
same plan classifies one stream per pair (all 20 pairs: a 4K stream at depth
4, which the mix lacks, is a plan stream that only this run names) against
another stream's merged tree, so that the compared masks hold both classes.

Served: 256 such streams with Poisson arrivals; ten seconds of arrivals are
offered at once and served under the 32 GiB budget.  The oracle replays one
stream of each resolution up to 1920x1080 in full (re-merges included), and
a 3840x2160 stream on sampled pixels of every test frame; three streams
served alone give the same masks as in the mix.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

FG_MIN, FG_MAX = 0.001, 0.999


def _threads():
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


@pytest.fixture(scope="module")
def env(oracle_lib):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_1945_amd import obg
    obg.load()
    return obg, oracle_lib


def _oracle_trees(O, frame_chunks, width, height, depth):
    """Trees of every frame (the oracle's Store Color and pruning), built on
    all host threads, each thread with a forest of its own.  frame_chunks
    yields (first frame index, uint8 numpy [n, H, row_pitch]).  Returns the
    occupancy bitset of every frame."""
    occs = {}

    def build(job):
        k0, arr = job
        f = O.Forest(width, height, depth)
        out = {}
        for j in range(arr.shape[0]):
            i = f.add_frame(arr[j])
            out[k0 + j] = f.export(i)
            f.drop(i)
        return out

    with ThreadPoolExecutor(_threads()) as ex:
        for k0, chunk in frame_chunks:
            step = max(1, -(-chunk.shape[0] // _threads()))
            jobs = [(k0 + j, chunk[j: j + step]) for j in range(0, chunk.shape[0], step)]
            for part in ex.map(build, jobs):
                occs.update(part)
    return occs


def _merge_from_trees(O, occs, ids, width, height, depth, thr):
    """Algorithm 2 over the trees of frames `ids` (trees rebuilt from their
    occupancy, which the pins show equal to trees built from the frames)."""
    f = O.Forest(width, height, depth)
    return f.merge([f.add_occupancy(occs[k]) for k in ids], *thr)


def _gpu_chunks(spec, ids, chunk=24):
    from synth.fast import make_frames_gpu
    ids = list(ids)
    buf = torch.empty((min(chunk, len(ids)), spec.height, spec.row_pitch), dtype=torch.uint8, device="cuda")
    for i in range(0, len(ids), chunk):
        part = ids[i: i + chunk]
        make_frames_gpu(spec, part, buf[: len(part)])
        yield part[0], buf[: len(part)].cpu().numpy()


def _sample_check(model, frame_host, g_mask_frame, n, rng, label):
    """n sampled pixels of one frame: the GPU mask bit against Check Color."""
    H, W = model.height, model.width
    ys, xs = rng.integers(0, H, n), rng.integers(0, W, n)
    fg = 0
    for y, x in zip(ys.tolist(), xs.tolist()):
        r, g, b = (int(v) for v in frame_host[y, 3 * x: 3 * x + 3])
        want = not model.check_pixel(x, y, r, g, b)
        assert ((int(g_mask_frame[y, x >> 6]) >> (x & 63)) & 1) == int(want), f"{label}: pixel ({x},{y})"
        fg += int(want)
    return fg


def _check_stream_masks(model, frames_dev, mask_dev, n_test, label, rng, mixed, samples=64):
    """Whole first and last test frames, and `samples` pixels of every test
    frame.  Returns (foreground bits, pixels) of what was compared."""
    g_mask = mask_dev.cpu().numpy().view(np.uint64)
    fg, px = 0, 0
    for t in sorted({0, n_test - 1}):
        host = frames_dev[t].cpu().numpy()
        want = model.classify(host)
        assert np.array_equal(g_mask[t], want), f"{label}: test frame {t}"
        fg += int(np.unpackbits(want.view(np.uint8)).sum())
        px += model.width * model.height
    whole = fg / px
    for t0 in range(0, n_test, 32):
        host = frames_dev[t0: t0 + 32].cpu().numpy()
        for j in range(host.shape[0]):
            fg += _sample_check(model, host[j], g_mask[t0 + j], samples, rng, f"{label} frame {t0 + j}")
            px += samples
    if mixed:
        assert FG_MIN < whole < FG_MAX, f"{label}: whole frames hold one class only ({whole})"
    return fg, px


def test_batched_64_streams_full_size(env):
    obg, O = env
    from oracle import models
    from synth import frames as S
    from synth.fast import make_frames_gpu
    wl = S.cfg3()
    streams = []
    print(f"[case] batched workload: {len(wl.streams)} streams, generating frames", flush=True)
    for spec, d, thr in zip(wl.streams, wl.depth, wl.thr):
        g = obg.FrameGeom(spec.width, spec.height, d)
        fr = torch.empty((spec.n_frames, spec.height, spec.row_pitch), dtype=torch.uint8, device="cuda")
        make_frames_gpu(spec, range(spec.n_frames), fr)
        T, N = spec.n_train, spec.n_test
        streams.append({"geom": g, "train": fr[:T], "n_train": T, "thr": thr, "test": fr[T:], "n_test": N,
                        "occ": obg.empty_occ(g, T), "leafset": obg.empty_leafset(g), "mask": obg.empty_mask(g, N),
                        "frames": fr, "spec": spec})
    pairs = {}
    for i, s in enumerate(streams):
        pairs.setdefault((s["geom"].width, s["geom"].height, s["geom"].depth), i)
    # plan streams for the pairs the mix lacks: classify-only, named by the second run alone
    extra = []
    for (W, H) in S.MIX_RES:
        for d in (3, 4, 5, 6):
            if (W, H, d) not in pairs:
                spec = S.StreamSpec(W, H, 0, 20, seed=3, stream=1000 + len(extra), bimodal_frac=0.2, drift_amp=0.1,
                                    fg="ellipses", fg_coverage=0.05)
                g = obg.FrameGeom(W, H, d)
                fr = torch.empty((20, H, spec.row_pitch), dtype=torch.uint8, device="cuda")
                make_frames_gpu(spec, range(20), fr)
                extra.append({"geom": g, "n_train": 0, "thr": (1, 2), "test": fr, "n_test": 20,
                              "leafset": obg.empty_leafset(g), "mask": obg.empty_mask(g, 20), "frames": fr})
                pairs[(W, H, d)] = len(streams) + len(extra) - 1
    assert len(pairs) == 20
    every = streams + extra
    torch.cuda.synchronize()
    plan = obg.obg_plan_create([{"geom": s["geom"], "thr": s["thr"], "max_train": s["n_train"],
                                 "max_test": s["n_test"]} for s in every])
    items = obg.work_items([dict(s, stream=i) for i, s in enumerate(streams)])
    print("[case] batched workload: plan tune and run", flush=True)
    plan.tune(items)
    plan.run(items)
    torch.cuda.synchronize()
    assert obg.item_status(items) == [obg.ITEM_OK] * len(streams)
    print("[case] batched workload: one-stream calls", flush=True)
    for i, s in enumerate(streams):
        g, T, N = s["geom"], s["n_train"], s["n_test"]
        occ, leaf, mask = obg.empty_occ(g, T), obg.empty_leafset(g), obg.empty_mask(g, N)
        obg.obg_train_frame(g, s["train"], T, occ)
        obg.obg_merge(g, occ, T, 0, T, s["thr"][0], s["thr"][1], leaf)
        obg.obg_classify(g, s["test"], N, leaf, mask)
        torch.cuda.synchronize()
        assert torch.equal(s["occ"], occ), f"stream {i} trees"
        assert torch.equal(s["leafset"], leaf), f"stream {i} leaf set"
        assert torch.equal(s["mask"], mask), f"stream {i} masks"
        del occ, mask
    print("[case] batched workload: oracle trees and leaf sets of every stream", flush=True)
    models_own = {}
    for i, s in enumerate(streams):
        g, T = s["geom"], s["n_train"]
        chunks = ((k, s["frames"][k: k + 32].cpu().numpy()) for k in range(0, T, 32))
        occs = _oracle_trees(O, chunks, g.width, g.height, g.depth)
        g_occ = s["occ"].cpu().numpy().view(np.uint32)
        for k in range(T):
            assert np.array_equal(g_occ[k], occs[k]), f"stream {i}: tree of training frame {k}"
        model = _merge_from_trees(O, occs, range(T), g.width, g.height, g.depth, s["thr"])
        assert np.array_equal(s["leafset"].cpu().numpy().view(np.uint32), model.leafset()), f"stream {i} leaf set"
        if pairs.get((g.width, g.height, g.depth)) == i:
            models_own[i] = model
    rng = np.random.default_rng(33)
    for i, model in models_own.items():
        s = streams[i]
        print(f"[case] batched workload: masks of stream {i} ({s['geom'].width}x{s['geom'].height}, "
              f"d={s['geom'].depth}) against its own merged tree", flush=True)
        _check_stream_masks(model, s["test"], s["mask"], s["n_test"], f"stream {i}", rng, mixed=False)
    # the second run of the same plan: one classify-only item per pair, with
    # another stream's merged tree as the model
    chosen = sorted(pairs.values())
    entries = []
    for i in chosen:
        s = every[i]
        leaf = torch.from_numpy(models.foreign_leafset(s["geom"].depth).view(np.int32)).cuda()
        entries.append({"stream": i, "geom": s["geom"], "n_train": 0, "n_test": s["n_test"], "test": s["test"],
                        "leafset": leaf, "mask": s["mask"]})
    items2 = obg.work_items(entries)
    print(f"[case] batched workload: second run, {len(entries)} classify-only items", flush=True)
    plan.run(items2)
    torch.cuda.synchronize()
    assert obg.item_status(items2) == [obg.ITEM_OK] * len(entries)
    fg_total = px_total = 0
    for e in entries:
        g = e["geom"]
        model = models.foreign_model(g.width, g.height, g.depth)
        fg, px = _check_stream_masks(model, e["test"], e["mask"], e["n_test"],
                                     f"stream {e['stream']} ({g.width}x{g.height}, d={g.depth}) foreign model",
                                     rng, mixed=True)
        fg_total += fg
        px_total += px
    print(f"[case] batched workload: {fg_total} foreground bits of {px_total} compared", flush=True)
    plan.close()


def _replay_served(O, spec, depth, thr, n, period, window, masks, full, rng, label):
    """The oracle's run of one served stream: trees of all n frames, the model
    from the training frames, then every test frame checked with the model in
    force and the model re-merged after every `period` test frames from the
    trees of the last `window` frames.  full: whole masks of every test
    frame; else 256 sampled pixels of each."""
    T = spec.n_train
    occs = _oracle_trees(O, _gpu_chunks(spec, range(n)), spec.width, spec.height, depth)
    model = _merge_from_trees(O, occs, range(T), spec.width, spec.height, depth, thr)
    fg = px = 0
    t = 0
    with ThreadPoolExecutor(_threads()) as ex:
        while T + t < n:
            block = list(range(T + t, min(n, T + t - t % period + period)))
            for k0, chunk in _gpu_chunks(spec, block):
                ks = list(range(k0, k0 + chunk.shape[0]))
                if full:
                    got = list(ex.map(model.classify, [chunk[j] for j in range(len(ks))]))
                    for k, want in zip(ks, got):
                        assert np.array_equal(masks[k - T], want), f"{label}: test frame {k - T}"
                        fg += int(np.unpackbits(want.view(np.uint8)).sum())
                        px += spec.width * spec.height
                else:
                    for j, k in enumerate(ks):
                        fg += _sample_check(model, chunk[j], masks[k - T], 256, rng, f"{label} test frame {k - T}")
                        px += 256
            t += len(block)
            if t % period == 0:
                k = T + t - 1
                model = _merge_from_trees(O, occs, range(k - window + 1, k + 1), spec.width, spec.height, depth, thr)
    return fg, px


def test_served_256_streams(env):
    obg, O = env
    from synth import frames as S
    from synth.fast import IngestContext, poisson_arrivals
    specs, depths, thrs, rates = S.cfg4()
    period, window = 100, 50
    arrivals = poisson_arrivals(rates, 10.0, seed=4)
    streams = [{"width": sp.width, "height": sp.height, "depth": d, "n_train": sp.n_train, "thr": thr}
               for sp, d, thr in zip(specs, depths, thrs)]
    # streams that reach at least one re-merge within the ten seconds
    live = [i for i in range(len(specs)) if len(arrivals[i]) > specs[i].n_train + period]
    order = sorted(live, key=lambda i: (specs[i].width * specs[i].height, i))
    assert len(order) >= 20
    # one watched stream per resolution
    watch = []
    for (W, H) in S.MIX_RES:
        cand = [i for i in order if (specs[i].width, specs[i].height) == (W, H)]
        assert cand, (W, H)
        watch.append(cand[0])
    alone = [order[0], order[len(order) // 2], order[-1]]

    def serve(which, watch_list):
        sp = [specs[i] for i in which]
        st = [streams[i] for i in which]
        ar = [arrivals[i] for i in which]
        ctx = IngestContext(sp, [len(a) for a in ar], slots=8)
        sums = np.zeros((len(which), max(len(a) for a in ar)), dtype=np.uint64)
        wl = [which.index(w) for w in watch_list]
        masks = [np.zeros((max(len(ar[j]) - st[j]["n_train"], 0), st[j]["height"], (st[j]["width"] + 63) // 64),
                          dtype=np.uint64) for j in wl]
        stats = obg.obg_serve_run(st, ar, ctx.fn, ctx.ctx, speed=1e9, budget_bytes=32 << 30, max_inflight=3,
                                  max_batch_frames=256, remerge_period=period, remerge_window=window,
                                  checksums=sums, watch=wl, watch_masks=masks,
                                  watch_max_frames=max((m.shape[0] for m in masks), default=0))
        ctx.close()
        return stats, sums, masks

    every = list(range(len(specs)))
    print(f"[case] served workload: {len(specs)} streams, {sum(len(a) for a in arrivals)} frames at once", flush=True)
    stats, sums, masks = serve(every, watch)
    assert stats["frames_served"] == stats["frames_arrived"] == sum(len(a) for a in arrivals)
    assert stats["merges"] >= len(specs)
    rng = np.random.default_rng(44)
    for w, m in zip(watch, masks):
        spec = specs[w]
        n = len(arrivals[w])
        full = spec.width * spec.height <= 1920 * 1080
        print(f"[case] served workload: oracle replay of stream {w} ({spec.width}x{spec.height}, d={depths[w]}, "
              f"{n} frames, {'whole masks' if full else 'sampled pixels'})", flush=True)
        fg, px = _replay_served(O, spec, depths[w], thrs[w], n, period, window, m, full, rng, f"stream {w}")
        print(f"[case] served workload: stream {w}: {fg} foreground bits of {px} compared", flush=True)
    for w in alone:
        print(f"[case] served workload: stream {w} ({specs[w].width}x{specs[w].height}) alone", flush=True)
        _, s1, _ = serve([w], [])
        n, T = len(arrivals[w]), specs[w].n_train
        assert np.array_equal(s1[0, T:n], sums[w, T:n]), f"stream {w}: alone differs from the mix"
        assert np.count_nonzero(sums[w, T:n]) == n - T
