"""Batched form: many streams in one persistent launch per step, against the
one-stream calls (bit for bit) and against the oracle."""
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


def _one_stream_reference(obg, s):
    g, T, N = s["geom"], s["n_train"], s["n_test"]
    occ = obg.empty_occ(g, T)
    leaf = obg.empty_leafset(g)
    for f in range(T):                     # one launch per frame, as a plain caller would
        obg.obg_train_frame(g, s["train"][f], 1, occ[f])
    obg.obg_merge(g, occ, T, 0, T, s["thr"][0], s["thr"][1], leaf)
    mask = obg.empty_mask(g, N) if N else None
    for f in range(N):
        obg.obg_classify(g, s["test"][f], 1, leaf, mask[f])
    return occ, leaf, mask


@pytest.mark.parametrize("flags,per_depth", [(0, 1), (2, 1), (1, 1), (0, 2), (2, 2)],
                         ids=["graph", "no_graph", "autotune", "per_depth_graph", "per_depth_no_graph"])
def test_batch_equals_one_stream_calls_and_oracle(env, flags, per_depth):
    obg, O = env
    streams = _mixed(obg, 11 + flags + 10 * (per_depth - 1))
    print(f"[case] batch flags={flags} per_depth={per_depth} streams={len(streams)}", flush=True)
    obg.obg_tune_set("batch_per_depth", per_depth)
    try:
        batch = obg.obg_batch_create(streams, flags=flags)
    finally:
        obg.obg_tune_set("batch_per_depth", 0)
    info = batch.info()
    assert info["graph"] == (0 if flags & 2 else 1)
    if not flags & 1:
        assert info["per_depth_launches"] == per_depth - 1
    for rep in range(2):                   # outputs are rewritten completely on every run
        for s in streams:
            s["occ"].fill_(-1)
            s["leafset"].fill_(-1)
            if s["mask"] is not None:
                s["mask"].fill_(-1)
        batch.run()
        torch.cuda.synchronize()
        for i, s in enumerate(streams):
            occ, leaf, mask = _one_stream_reference(obg, s)
            torch.cuda.synchronize()
            assert torch.equal(s["occ"], occ), f"stream {i} occupancy"
            assert torch.equal(s["leafset"], leaf), f"stream {i} leaf set"
            if mask is not None:
                assert torch.equal(s["mask"], mask), f"stream {i} masks"
    for i, s in enumerate(streams):
        g = s["geom"]
        f = O.Forest(g.width, g.height, g.depth)
        idx = f.add_frames(s["host"][: s["n_train"]])
        model = f.merge(idx, *s["thr"])
        assert np.array_equal(s["leafset"].cpu().numpy().view(np.uint32).reshape(1, -1), model.leafset())
        for t in range(s["n_test"]):
            want = model.classify(s["host"][s["n_train"] + t])
            assert np.array_equal(s["mask"][t].cpu().numpy().view(np.uint64), want), f"stream {i} frame {t}"
    batch.close()


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
    batch = obg.obg_batch_create(streams)
    batch.run()
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
    batch.close()
