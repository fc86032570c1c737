"""Batched form: a plan over many streams, run on device work items, against
the one-stream calls (bit for bit) and against the oracle."""
import numpy as np
import pytest
import torch

import brute

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env(oracle_lib):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_1945_amd import obg
    obg.load()
    return obg, oracle_lib


def _stream(obg, rng, W, H, d, T, n_test, thr, ncol):
    rp = ((3 * W + 15) // 16) * 16
    frames = brute.tiny_frames(rng, T + n_test, W, H, n_colours=ncol, row_pitch=rp)
    g = obg.FrameGeom(W, H, d)
    dev = torch.from_numpy(np.stack(frames)).cuda()
    return {
        "geom": g, "train": dev[:T].contiguous(), "n_train": T, "thr": thr,
        "test": dev[T:].contiguous() if n_test else None, "n_test": n_test,
        "occ": obg.empty_occ(g, T), "leafset": obg.empty_leafset(g),
        "mask": obg.empty_mask(g, n_test) if n_test else None,
        "host": frames,
    }


def _mixed(obg, seed):
    rng = np.random.default_rng(seed)
    shapes = [(64, 8, 1), (17, 5, 2), (160, 12, 3), (333, 7, 4), (96, 31, 5), (130, 9, 6),
              (48, 48, 5), (200, 3, 4), (1, 1, 3), (640, 4, 6)]
    out = []
    for i, (W, H, d) in enumerate(shapes):
        T = int(rng.integers(2, 9))
        n_test = 0 if i == 3 else int(rng.integers(1, 4))
        thr = [(3, 10), (1, 2), (7, 10), (1, 1)][i % 4]
        out.append(_stream(obg, rng, W, H, d, T, n_test, thr, ncol=int(rng.integers(3, 40))))
    return out


def _plan(obg, streams, max_train=None, max_test=None):
    return obg.obg_plan_create([{"geom": s["geom"], "thr": s["thr"],
                                 "max_train": s["n_train"] if max_train is None else max_train,
                                 "max_test": s["n_test"] if max_test is None else max_test} for s in streams])


def _items(obg, streams, which=None):
    which = range(len(streams)) if which is None else which
    return obg.work_items([dict(s, stream=i) for i, s in ((i, streams[i]) for i in which)])


def _one_stream_reference(obg, s, leaf_in=None):
    """One launch per frame, as a plain caller would."""
    g, T, N = s["geom"], s["n_train"], s["n_test"]
    occ = obg.empty_occ(g, T) if T else None
    leaf = obg.empty_leafset(g) if leaf_in is None else leaf_in
    for f in range(T):
        obg.obg_train_frame(g, s["train"][f], 1, occ[f])
    if T:
        obg.obg_merge(g, occ, T, 0, T, s["thr"][0], s["thr"][1], leaf)
    mask = obg.empty_mask(g, N) if N else None
    for f in range(N):
        obg.obg_classify(g, s["test"][f], 1, leaf, mask[f])
    return occ, leaf, mask


def _oracle_check(O, s, leaf_in=None):
    g = s["geom"]
    if leaf_in is None:
        f = O.Forest(g.width, g.height, g.depth)
        model = f.merge(f.add_frames(s["host"][: s["n_train"]]), *s["thr"])
        assert np.array_equal(s["leafset"].cpu().numpy().view(np.uint32).reshape(1, -1), model.leafset())
    else:
        model = O.Model.from_leafset(leaf_in, g.width, g.height, g.depth)
    for t in range(s["n_test"]):
        want = model.classify(s["host"][s["n_train"] + t])
        assert np.array_equal(s["mask"][t].cpu().numpy().view(np.uint64), want), f"frame {t}"


@pytest.mark.parametrize("tune,per_depth,graph", [(False, 1, 1), (False, 1, 2), (True, 1, 1), (False, 2, 1),
                                                   (False, 2, 2)],
                         ids=["graph", "no_graph", "tuned", "per_depth_graph", "per_depth_no_graph"])
def test_plan_equals_one_stream_calls_and_oracle(env, tune, per_depth, graph):
    obg, O = env
    streams = _mixed(obg, 11 + (1 if tune else 0) + 10 * (per_depth - 1) + 3 * (graph - 1))
    print(f"[case] plan tune={tune} per_depth={per_depth} graph={graph} streams={len(streams)}", flush=True)
    obg.obg_tune_set("batch_per_depth", per_depth)
    obg.obg_tune_set("batch_graph", graph)
    try:
        plan = _plan(obg, streams)
    finally:
        obg.obg_tune_set("batch_per_depth", 0)
        obg.obg_tune_set("batch_graph", 0)
    items = _items(obg, streams)
    if tune:
        plan.tune(items)
    info = plan.info()
    assert info["graph"] == (1 if graph == 1 else 0)
    if not tune:
        assert info["per_depth_launches"] == per_depth - 1
    for rep in range(2):                   # outputs are rewritten completely on every run
        for s in streams:
            s["occ"].fill_(-1)
            s["leafset"].fill_(-1)
            if s["mask"] is not None:
                s["mask"].fill_(-1)
        plan.run(items)
        torch.cuda.synchronize()
        assert obg.item_status(items) == [obg.ITEM_OK] * len(streams)
        for i, s in enumerate(streams):
            occ, leaf, mask = _one_stream_reference(obg, s)
            torch.cuda.synchronize()
            assert torch.equal(s["occ"], occ), f"stream {i} occupancy"
            assert torch.equal(s["leafset"], leaf), f"stream {i} leaf set"
            if mask is not None:
                assert torch.equal(s["mask"], mask), f"stream {i} masks"
    for i, s in enumerate(streams):
        _oracle_check(O, s)
    plan.close()


def test_plan_serves_changing_work(env):
    """One plan (and its one captured graph) runs two different item arrays:
    other frames and buffers, fewer frames than the plan's maxima, a subset of
    the streams, and streams that only classify against a given leaf set.
    Each run equals the one-stream calls and the oracle; streams no item
    names keep their buffers."""
    obg, O = env
    rng = np.random.default_rng(101)
    shapes = [(64, 8, 3, 6, 3), (130, 9, 6, 5, 2), (96, 31, 5, 7, 3), (333, 7, 4, 4, 2), (48, 48, 2, 5, 3)]
    thr = [(1, 2), (3, 10), (7, 10), (1, 1), (1, 2)]
    first = [_stream(obg, rng, W, H, d, T, N, thr[i], ncol=int(rng.integers(3, 30)))
             for i, (W, H, d, T, N) in enumerate(shapes)]
    plan = _plan(obg, first, max_train=8, max_test=4)
    info0 = plan.info()
    print("[case] plan run 1: all streams", flush=True)
    items1 = _items(obg, first)
    plan.run(items1)
    torch.cuda.synchronize()
    assert obg.item_status(items1) == [0] * len(first)
    for i, s in enumerate(first):
        occ, leaf, mask = _one_stream_reference(obg, s)
        torch.cuda.synchronize()
        assert torch.equal(s["occ"], occ) and torch.equal(s["leafset"], leaf) and torch.equal(s["mask"], mask), i
        _oracle_check(O, s)
    # run 2: new frames and buffers; stream 1 classifies only (against the
    # leaf set of another stream of its depth), stream 3 is not named, stream
    # 4 trains only, counts below and at the maxima
    second = {}
    for i, (W, H, d, T, N) in enumerate(shapes):
        T2 = [8, 0, 2, None, 3][i]
        N2 = [4, 3, 1, None, 0][i]
        if T2 is None:
            continue
        s = _stream(obg, rng, W, H, d, max(T2, 1), N2, thr[i], ncol=int(rng.integers(3, 30)))
        s["n_train"] = T2
        if T2 == 0:
            s["train"], s["occ"] = None, None
            s["host"] = [None] + s["host"][1:]
        second[i] = s
    foreign = first[1]["leafset"].clone()
    second[1]["leafset"].copy_(foreign)
    sentinel = {k: first[3][k].clone() for k in ("occ", "leafset", "mask")}
    print("[case] plan run 2: a subset, classify-only and train-only items", flush=True)
    items2 = obg.work_items([dict(s, stream=i) for i, s in second.items()])
    plan.run(items2)
    torch.cuda.synchronize()
    assert obg.item_status(items2) == [0] * len(second)
    assert plan.info() == info0
    for i, s in second.items():
        if s["n_train"] == 0:
            s["host"] = s["host"][1:]
            leaf_in = foreign.clone()
            _, _, mask = _one_stream_reference(obg, s, leaf_in=leaf_in)
            torch.cuda.synchronize()
            assert torch.equal(s["leafset"], foreign), "a classify-only item's leaf set is input"
            assert torch.equal(s["mask"], mask)
            _oracle_check(O, s, leaf_in=foreign.cpu().numpy().view(np.uint32).reshape(1, -1))
            continue
        occ, leaf, mask = _one_stream_reference(obg, s)
        torch.cuda.synchronize()
        assert torch.equal(s["occ"], occ) and torch.equal(s["leafset"], leaf), i
        if s["n_test"]:
            assert torch.equal(s["mask"], mask), i
        _oracle_check(O, s)
    for k, v in sentinel.items():
        assert torch.equal(first[3][k], v), f"stream 3 not named in run 2, but its {k} changed"
    plan.close()


def test_plan_item_status(env):
    """Items the run cannot take are skipped with their reason; nothing of
    them is written, and the valid items of the same run are exact."""
    obg, O = env
    rng = np.random.default_rng(202)
    streams = [_stream(obg, rng, 64, 8, 4, 3, 2, (1, 2), ncol=9), _stream(obg, rng, 80, 6, 5, 4, 2, (1, 2), ncol=9)]
    # three more plan streams that no item names (a run holds at most as many
    # items as the plan has streams): their buffers must stay as they are
    idle = [_stream(obg, rng, 32, 4, 3, 2, 1, (1, 2), ncol=5) for _ in range(3)]
    for s in idle:
        s["occ"].fill_(5), s["leafset"].fill_(5), s["mask"].fill_(5)
    plan = _plan(obg, streams + idle)
    good = [dict(streams[0], stream=0)]
    bad_mask = obg.empty_mask(streams[1]["geom"], 2).fill_(7)
    # buffers that hold five training frames, so that only the plan's maximum refuses them
    g1 = streams[1]["geom"]
    five = torch.zeros((5, g1.height, g1.row_pitch), dtype=torch.uint8, device="cuda")
    five_occ = obg.empty_occ(g1, 5).fill_(9)
    bad = [dict(streams[1], stream=5),                          # no such stream
           dict(streams[1], stream=1, n_train=5, train=five, occ=five_occ),   # above max_train
           dict(streams[1], stream=1, mask=bad_mask),            # fine: taken
           dict(streams[1], stream=1, mask=bad_mask)]            # the stream again
    items = obg.work_items(good + bad)
    plan.run(items)
    torch.cuda.synchronize()
    assert obg.item_status(items) == [0, obg.ITEM_BAD_STREAM, obg.ITEM_BAD_COUNT, 0, obg.ITEM_DUPLICATE]
    assert bool((five_occ == 9).all()), "a skipped item wrote its trees"
    for s in idle:
        assert bool((s["occ"] == 5).all()) and bool((s["leafset"] == 5).all()) and bool((s["mask"] == 5).all())
    for s in streams:
        if s is streams[1]:
            s = dict(s, mask=bad_mask)
        occ, leaf, mask = _one_stream_reference(obg, s)
        torch.cuda.synchronize()
        assert torch.equal(s["occ"], occ) and torch.equal(s["leafset"], leaf) and torch.equal(s["mask"], mask)
    # NULL and misaligned buffers: fields patched in the packed items
    import ctypes
    W = ctypes.sizeof(obg.WorkItem)
    items = obg.work_items([dict(streams[0], stream=0), dict(streams[1], stream=1)])
    host = items.cpu().numpy().copy()
    host[W + obg.WorkItem.mask.offset: W + obg.WorkItem.mask.offset + 8] = 0
    host[obg.WorkItem.train_rgb.offset] += 8
    items = torch.from_numpy(host).cuda()
    streams[1]["mask"].fill_(3)
    before = streams[1]["mask"].clone()
    plan.run(items)
    torch.cuda.synchronize()
    assert obg.item_status(items) == [obg.ITEM_ALIGN, obg.ITEM_NULL]
    assert torch.equal(streams[1]["mask"], before)
    plan.close()


def test_batch_mixed_resolutions(env):
    """The uneven resolution / depth / T / threshold mix, few frames per stream."""
    from synth.frames import mixed_streams, make_frames, scaled
    obg, O = env
    specs, depths, thrs = mixed_streams(10, seed=5, n_test=3)
    streams = []
    for spec, d, thr in zip(specs, depths, thrs):
        spec = scaled(spec, n_train=min(spec.n_train, 6), n_test=3)
        fr = make_frames(spec, range(spec.n_frames), device="cuda")
        g = obg.FrameGeom(spec.width, spec.height, d)
        T = spec.n_train
        streams.append({"geom": g, "train": fr[:T], "n_train": T, "thr": thr, "test": fr[T:],
                        "n_test": 3, "occ": obg.empty_occ(g, T), "leafset": obg.empty_leafset(g),
                        "mask": obg.empty_mask(g, 3), "spec": spec, "frames": fr})
    print(f"[case] mixed batch of {len(streams)} streams", flush=True)
    plan = _plan(obg, streams)
    items = _items(obg, streams)
    plan.run(items)
    torch.cuda.synchronize()
    for i, s in enumerate(streams):
        occ, leaf, mask = _one_stream_reference(obg, s)
        torch.cuda.synchronize()
        assert torch.equal(s["occ"], occ) and torch.equal(s["leafset"], leaf) and torch.equal(s["mask"], mask), i
    # oracle on the first three streams
    for s in streams[:3]:
        g = s["geom"]
        host = s["frames"].cpu().numpy()
        f = O.Forest(g.width, g.height, g.depth)
        idx = f.add_frames(list(host[: s["n_train"]]))
        model = f.merge(idx, *s["thr"])
        assert np.array_equal(s["leafset"].cpu().numpy().view(np.uint32).reshape(1, -1), model.leafset())
        want = model.classify(host[s["n_train"] + 2])
        assert np.array_equal(s["mask"][2].cpu().numpy().view(np.uint64), want)
    plan.close()
