"""GPU parity: libobg.so (through the C ABI) against the CPU oracle, bit for bit.

Inputs are seeded: random tiny frames (numpy) and the synthetic streams of
synth.frames; the oracle sees the same bytes as the GPU.  Every comparison is
exact -- occupancy bitsets, pixel counts, merged leaf sets and masks are
integers with one correct value each.
"""
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


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def upload(frames, frame_pitch=None):
    """Stack host frames [H, row_pitch] into one device buffer with frame_pitch."""
    h, rp = frames[0].shape
    fp = frame_pitch or h * rp
    buf = np.zeros((len(frames), fp), dtype=np.uint8)
    for i, f in enumerate(frames):
        buf[i, : h * rp] = f.reshape(-1)
    return torch.from_numpy(buf).cuda()


def run_pipeline(obg, g, dev_train, T, dev_test, n_test, num, den, counts=False):
    occ = obg.empty_occ(g, T)
    cnt = torch.empty((T, g.n_regions, 1 << (3 * g.depth)), dtype=torch.int32, device="cuda") if counts else None
    leaf = obg.empty_leafset(g)
    mask = obg.empty_mask(g, n_test)
    obg.obg_train_frame(g, dev_train, T, occ, cnt)
    obg.obg_merge(g, occ, T, 0, T, num, den, leaf)
    obg.obg_classify(g, dev_test, n_test, leaf, mask)
    torch.cuda.synchronize()
    return occ, cnt, leaf, mask


def check_against_oracle(env, W, H, d, frames, T, num, den, rw=0, rh=0, row_pitch=None,
                         frame_pitch=None, counts=True, label=""):
    obg, O = env
    rp = row_pitch or frames[0].shape[1]
    g = obg.FrameGeom(W, H, d, row_pitch=rp, frame_pitch=frame_pitch or 0, region_w=rw, region_h=rh)
    print(f"[case] {label} W={W} H={H} d={d} T={T} thr={num}/{den} region={rw}x{rh} pitch={rp}", flush=True)
    dtrain = upload(frames[:T], g.frame_pitch)
    dtest = upload(frames[T:], g.frame_pitch)
    n_test = len(frames) - T
    occ, cnt, leaf, mask = run_pipeline(obg, g, dtrain, T, dtest, n_test, num, den, counts)
    f = O.Forest(W, H, d, rw, rh)
    idx = f.add_frames(frames[:T], store_levels=8 if W * H <= 4096 else None)
    for i in idx:
        o, c = f.export(i, with_counts=True)
        assert np.array_equal(u32(occ[i]).reshape(o.shape), o), f"{label} occupancy frame {i}"
        if counts:
            assert np.array_equal(u32(cnt[i]).reshape(c.shape), c), f"{label} counts frame {i}"
    model = f.merge(idx, num, den)
    assert np.array_equal(u32(leaf).reshape(model.n_regions, -1), model.leafset()), f"{label} leaf set"
    for i in range(n_test):
        want = model.classify(frames[T + i])
        assert np.array_equal(u64(mask[i]).reshape(want.shape), want), f"{label} mask frame {i}"
    return occ, leaf, mask


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d", range(1, 9))
def test_all_depths_ragged_widths(env, d):
    rng = np.random.default_rng(d)
    for W, H in [(1, 1), (17, 3), (64, 2), (100, 5), (130, 4)]:
        rp = ((3 * W + 15) // 16) * 16
        frames = brute.tiny_frames(rng, 6, W, H, n_colours=7, row_pitch=rp)
        check_against_oracle(env, W, H, d, frames, 4, 1, 2, label=f"depth{d}", counts=(d <= 6))


@pytest.mark.parametrize("W", [15, 16, 33, 48, 63, 65, 127, 160, 193])
def test_widths_and_padding(env, W):
    rng = np.random.default_rng(W)
    H = 9
    rp = ((3 * W + 15) // 16) * 16 + 32          # extra row padding
    frames = brute.tiny_frames(rng, 7, W, H, n_colours=10, row_pitch=rp)
    for f in frames:
        f[:, 3 * W:] = 0xAB                     # padding bytes must not matter
    check_against_oracle(env, W, H, 5, frames, 5, 2, 5, row_pitch=rp,
                         frame_pitch=H * rp + 48, label="pad")


@pytest.mark.parametrize("num,den", [(1, 10), (3, 10), (1, 2), (7, 10), (1, 1), (3, 2)])
def test_thresholds(env, num, den):
    rng = np.random.default_rng(num * 100 + den)
    W, H = 96, 12
    frames = brute.tiny_frames(rng, 14, W, H, n_colours=24, row_pitch=288)
    check_against_oracle(env, W, H, 3, frames, 10, num, den, label="thr")


@pytest.mark.parametrize("rw,rh,d", [(32, 32, 4), (16, 8, 3), (48, 20, 5), (24, 20, 4), (32, 16, 6), (7, 5, 2), (16, 4, 7)])
def test_regions(env, rw, rh, d):
    rng = np.random.default_rng(rw * rh + d)
    W, H = 200, 70
    frames = brute.tiny_frames(rng, 6, W, H, n_colours=12, row_pitch=608)
    check_against_oracle(env, W, H, d, frames, 4, 1, 2, rw=rw, rh=rh, label="region",
                         counts=(d <= 6))


def test_cfg0_full(env):
    """The small plain workload end to end; frames made on the GPU."""
    from synth.frames import cfg0, make_frames
    obg, O = env
    wl = cfg0()
    s = wl.streams[0]
    dev = make_frames(s, range(s.n_frames), device="cuda")
    host = make_frames(s, [0, s.n_train, s.n_frames - 1], device="cpu")
    assert torch.equal(dev[[0, s.n_train, s.n_frames - 1]].cpu(), host), "generator differs between devices"
    frames = list(dev.cpu().numpy())
    num, den = wl.thr[0]
    check_against_oracle(env, s.width, s.height, wl.depth[0], frames, s.n_train, num, den, label="cfg0")


def test_merge_ring_windows(env):
    """Merge over windows of a ring of synthetic bitsets, including wrap-around."""
    obg, O = env
    rng = np.random.default_rng(77)
    for d, nreg, ring, dens in [(2, 3, 9, 0.5), (4, 2, 60, 0.3), (5, 1, 120, 0.6), (6, 1, 40, 0.05), (1, 5, 7, 0.5)]:
        W = 8
        g = obg.FrameGeom(W * nreg, 8, d, region_w=(W if nreg > 1 else 0), region_h=(8 if nreg > 1 else 0))
        words = g.words
        lc = 1 << (3 * d)
        bits = rng.random((ring, nreg, max(lc, 32))) < dens
        bits[:, :, lc:] = False
        occ = np.packbits(bits, axis=-1, bitorder="little").view(np.uint32).reshape(ring, nreg, words)
        docc = torch.from_numpy(occ.view(np.int32).copy()).cuda()
        for first, n, num, den in [(0, ring, 1, 2), (ring - 3, min(ring, 5), 3, 10), (1, ring - 1, 7, 10),
                                   (ring // 2, ring, 1, 1), (0, 1, 1, 2), (ring - 1, ring, 2, 3)]:
            print(f"[case] merge d={d} nreg={nreg} ring={ring} first={first} n={n} thr={num}/{den}", flush=True)
            leaf = obg.empty_leafset(g)
            obg.obg_merge(g, docc, ring, first, n, num, den, leaf)
            torch.cuda.synchronize()
            f = O.Forest(g.width, g.height, d, g.region_w, g.region_h)
            idx = [f.add_occupancy(occ[(first + t) % ring]) for t in range(n)]
            want = f.merge(idx, num, den).leafset()
            assert np.array_equal(u32(leaf).reshape(want.shape), want)


def test_merge_large_one_thread_per_word(env):
    """Merges of at least 512 K words (a 4K frame with 32x32 regions: 8160
    trees of 128 words) count each word's window in one thread instead of
    four waves; against the oracle on synthetic bitsets, with windows that
    wrap the ring and groups of two slots (a group's tree holds what any of
    its slots holds)."""
    obg, O = env
    rng = np.random.default_rng(4242)
    g = obg.FrameGeom(3840, 2160, 4, region_w=32, region_h=32)
    assert g.n_regions * g.words >= 1 << 19
    ring = 6
    bits = rng.random((ring, g.n_regions, 4096)) < 0.05
    occ = np.packbits(bits, axis=-1, bitorder="little").view(np.uint32).reshape(ring, g.n_regions, g.words)
    del bits
    docc = torch.from_numpy(occ.view(np.int32).copy()).cuda()
    for first, n, grp, num, den in [(4, 5, 1, 1, 2), (0, 6, 1, 1, 3), (3, 5, 2, 1, 2), (5, 6, 2, 2, 3)]:
        print(f"[case] large merge regions=8160 first={first} n={n} group={grp} thr={num}/{den}", flush=True)
        leaf = obg.empty_leafset(g)
        if grp == 1:
            obg.obg_merge(g, docc, ring, first, n, num, den, leaf)
        else:
            obg.obg_merge_groups(g, docc, ring, first, n, grp, num, den, leaf)
        torch.cuda.synchronize()
        slots = [occ[(first + t) % ring] for t in range(n)]
        trees = [np.bitwise_or.reduce(np.stack(slots[i: i + grp]), axis=0) for i in range(0, n, grp)]
        f = O.Forest(g.width, g.height, 4, 32, 32)
        want = f.merge([f.add_occupancy(t) for t in trees], num, den).leafset()
        assert np.array_equal(u32(leaf).reshape(want.shape), want)


def test_merge_groups_of_frames(env):
    """Trees of groups of consecutive frames (Section 3): the GPU merge of
    grouped ring windows against the oracle's group trees built from the
    frames, including a short last group and a window that wraps the ring."""
    obg, O = env
    rng = np.random.default_rng(91)
    for W, H, d, rw, rh, T, grp, ring, first, num, den in [
            (40, 12, 4, 0, 0, 9, 2, 9, 0, 1, 2), (40, 12, 4, 0, 0, 9, 4, 12, 7, 2, 3),
            (33, 20, 5, 16, 8, 7, 3, 10, 5, 1, 2), (64, 8, 3, 0, 0, 6, 6, 6, 0, 1, 1),
            (25, 9, 6, 0, 0, 8, 1, 8, 3, 1, 2), (48, 16, 2, 16, 16, 10, 3, 13, 11, 7, 10)]:
        rp = ((3 * W + 15) // 16) * 16
        frames = brute.tiny_frames(rng, T + 1, W, H, n_colours=int(rng.integers(4, 20)), row_pitch=rp)
        g = obg.FrameGeom(W, H, d, region_w=rw, region_h=rh)
        print(f"[case] grouped merge W={W} H={H} d={d} region={rw}x{rh} T={T} group={grp} ring={ring} "
              f"first={first} thr={num}/{den}", flush=True)
        dev = upload(frames, g.frame_pitch)
        occ = obg.empty_occ(g, ring)
        occ.zero_()
        for t in range(T):                    # frame t's tree into ring slot first + t
            obg.obg_train_frame(g, dev[t], 1, occ[(first + t) % ring])
        leaf = obg.empty_leafset(g)
        obg.obg_merge_groups(g, occ, ring, first, T, grp, num, den, leaf)
        torch.cuda.synchronize()
        f = O.Forest(W, H, d, rw, rh)
        idx = [f.add_group(frames[i: min(i + grp, T)]) for i in range(0, T, grp)]
        model = f.merge(idx, num, den)
        assert np.array_equal(u32(leaf).reshape(model.leafset().shape), model.leafset())
        if grp == 1:
            plain = obg.empty_leafset(g)
            obg.obg_merge(g, occ, ring, first, T, num, den, plain)
            torch.cuda.synchronize()
            assert torch.equal(plain, leaf)
        mask = obg.empty_mask(g, 1)
        obg.obg_classify(g, dev[T], 1, leaf, mask)
        torch.cuda.synchronize()
        assert np.array_equal(u64(mask[0]), model.classify(frames[T]))


@pytest.mark.parametrize("d", range(1, 9))
def test_redraw_against_oracle(env, d):
    """Redraw with each frame's own pruned tree (Section 2), ragged widths and
    regions, in place and out of place, against the oracle's tree walk."""
    obg, O = env
    rng = np.random.default_rng(60 + d)
    for W, H, rw, rh in [(1, 1, 0, 0), (15, 3, 0, 0), (16, 2, 0, 0), (33, 17, 0, 0), (100, 9, 32, 4), (257, 5, 0, 0)]:
        rp = ((3 * W + 15) // 16) * 16
        frames = brute.tiny_frames(rng, 3, W, H, n_colours=(None if W % 2 else 9), row_pitch=rp)
        g = obg.FrameGeom(W, H, d, region_w=rw, region_h=rh)
        print(f"[case] redraw W={W} H={H} d={d} region={rw}x{rh}", flush=True)
        dev = upload(frames, g.frame_pitch)
        out = torch.full_like(dev, 0xA5)
        obg.obg_quantize(g, dev, 3, out)
        inplace = dev.clone()
        obg.obg_quantize(g, inplace, 3, inplace)
        torch.cuda.synchronize()
        f = O.Forest(W, H, d, rw, rh)
        for t in range(3):
            want = f.redraw(f.add_frame(frames[t]), frames[t])
            got = out[t].cpu().numpy().reshape(H, rp)
            assert np.array_equal(got[:, : 3 * W], want), (W, H, t)
            assert (got[:, 3 * W:] == 0xA5).all()          # row padding untouched
            assert np.array_equal(inplace[t].cpu().numpy().reshape(H, rp)[:, : 3 * W], want)


def test_score_against_plain_counts(env):
    """Section 5's counts from masks and ground truth (bits past the width,
    set at random in both, are ignored) against counting pixel by pixel."""
    obg, O = env
    from oracle import metrics as M
    rng = np.random.default_rng(17)
    for W, H, n in [(1, 1, 1), (63, 5, 3), (64, 4, 2), (65, 7, 2), (200, 9, 4), (1000, 3, 1)]:
        g = obg.FrameGeom(W, H, 4)
        mw = g.mask_row_words
        m = rng.random((n, H, W)) < 0.3
        t = rng.random((n, H, W)) < 0.2
        def pack(b):
            words = np.zeros((n, H, mw), dtype=np.uint64)
            for x in range(W):
                words[:, :, x >> 6] |= b[:, :, x].astype(np.uint64) << np.uint64(x & 63)
            pad = rng.integers(0, 2 ** 63, (n, H), dtype=np.int64).astype(np.uint64) << np.uint64(1)
            if W & 63:
                words[:, :, -1] |= pad & ~np.uint64((1 << (W & 63)) - 1)
            return torch.from_numpy(words.view(np.int64)).cuda()
        print(f"[case] score W={W} H={H} n={n}", flush=True)
        counts = torch.full((3,), -1, dtype=torch.int64, device="cuda")
        obg.obg_score(g, pack(m), pack(t), n, counts)
        torch.cuda.synchronize()
        tp, fp, fn, tn = M.confusion(m, t)
        assert counts.cpu().tolist() == [tp, fp, fn]
        assert tn == n * W * H - tp - fp - fn


def test_fused_classify_occupancy(env):
    obg, O = env
    rng = np.random.default_rng(3)
    # the 2112-wide case has 66 region columns: its two d=4 tables take more
    # than 64 KiB of LDS per workgroup
    for W, H, d, rw, rh in [(160, 40, 4, 0, 0), (96, 33, 6, 0, 0), (128, 64, 3, 32, 32), (50, 10, 7, 0, 0),
                            (2112, 40, 4, 32, 32)]:
        rp = ((3 * W + 15) // 16) * 16
        frames = brute.tiny_frames(rng, 5, W, H, n_colours=9, row_pitch=rp)
        g = obg.FrameGeom(W, H, d, region_w=rw, region_h=rh)
        print(f"[case] fused W={W} H={H} d={d} region={rw}x{rh}", flush=True)
        dev = upload(frames, g.frame_pitch)
        occ_t = obg.empty_occ(g, 5)
        obg.obg_train_frame(g, dev, 5, occ_t)
        leaf = obg.empty_leafset(g)
        obg.obg_merge(g, occ_t, 5, 0, 3, 1, 2, leaf)
        mask_a = obg.empty_mask(g, 5)
        mask_b = obg.empty_mask(g, 5)
        occ_c = obg.empty_occ(g, 5)
        obg.obg_classify(g, dev, 5, leaf, mask_a)
        obg.obg_classify(g, dev, 5, leaf, mask_b, occ_c)
        torch.cuda.synchronize()
        assert torch.equal(mask_a, mask_b)
        assert torch.equal(occ_t, occ_c)


FUSED_KNOBS = [{}, {"fused_span": 4}, {"fused_span": 100}, {"fused_span": 8192}, {"fused_span": 4, "interleave": 1},
               {"mask_stage": 2}, {"layout": 2, "occ_wg_per_cu": 4}, {"occ_blind": 1}]


@pytest.mark.parametrize("knobs", FUSED_KNOBS,
                         ids=[",".join(f"{k}={v}" for k, v in kn.items()) or "default" for kn in FUSED_KNOBS])
def test_fused_knobs_against_oracle(env, knobs):
    """The fused pass (masks and each test frame's tree from one read, dual
    LDS tables, staged masks) under its launch knobs: items of 4 groups (many
    per frame, trees ORed into zeroed words), of a size that is not a multiple
    of 4, larger than the staging limit, dealt round-robin, and the compact
    table order.  Masks and trees equal the oracle's, frame by frame."""
    obg, O = env
    rng = np.random.default_rng(5150)
    try:
        for k, v in knobs.items():
            obg.obg_tune_set(k, v)
        for W, H, d in [(200, 30, 3), (333, 17, 5), (130, 26, 6), (64, 8, 4)]:
            rp = ((3 * W + 15) // 16) * 16
            T, N = 3, 4
            frames = brute.tiny_frames(rng, T + N, W, H, n_colours=13, row_pitch=rp)
            # the right half of every test frame from another palette: both classes
            other = brute.tiny_frames(rng, N, W, H, n_colours=13, row_pitch=rp)
            half = 3 * (W // 2)
            for i in range(N):
                frames[T + i][:, half:] = other[i][:, half:]
            g = obg.FrameGeom(W, H, d)
            print(f"[case] fused knobs {knobs} W={W} H={H} d={d}", flush=True)
            dtrain, dtest = upload(frames[:T], g.frame_pitch), upload(frames[T:], g.frame_pitch)
            occ_t, leaf = obg.empty_occ(g, T), obg.empty_leafset(g)
            obg.obg_train_frame(g, dtrain, T, occ_t)
            obg.obg_merge(g, occ_t, T, 0, T, 1, 2, leaf)
            mask = obg.empty_mask(g, N).fill_(-1)
            occ = obg.empty_occ(g, N).fill_(-1)
            obg.obg_classify(g, dtest, N, leaf, mask, occ)
            torch.cuda.synchronize()
            f = O.Forest(W, H, d)
            model = f.merge(f.add_frames(frames[:T]), 1, 2)
            tests = f.add_frames(frames[T:])
            fg = 0
            for i in range(N):
                want = model.classify(frames[T + i])
                assert np.array_equal(u64(mask[i]).reshape(want.shape), want), f"fused {knobs} mask {i} d={d}"
                fg += int(np.unpackbits(want.view(np.uint8)).sum())
                o = f.export(tests[i])
                assert np.array_equal(u32(occ[i]).reshape(o.shape), o), f"fused {knobs} tree {i} d={d}"
            assert 0 < fg < N * W * H, "masks hold both classes"
    finally:
        for k in obg.TUNE_KEYS:
            obg.obg_tune_set(k, 0)


@pytest.mark.parametrize("W,H,d,rw,rh", [(1280, 720, 4, 32, 32), (1000, 200, 5, 48, 40), (1010, 64, 3, 16, 16),
                                         (3840, 64, 4, 32, 32), (640, 96, 6, 32, 32), (1920, 128, 5, 64, 64)])
def test_region_chunks_one_frame_per_call(env, W, H, d, rw, rh):
    """Calls of one frame with regions cut each row of regions into chunks of
    whole region columns (the last one ragged, with the row's padding), and a
    call of a few frames too: trees, pixel counts, masks and fused trees equal
    the oracle's whatever the output buffers held before (stored trees must
    cover every word)."""
    obg, O = env
    rng = np.random.default_rng(W + H + d)
    rp = ((3 * W + 15) // 16) * 16
    T = 3
    frames = brute.tiny_frames(rng, T + 2, W, H, n_colours=20, row_pitch=rp)
    g = obg.FrameGeom(W, H, d, region_w=rw, region_h=rh)
    print(f"[case] region chunks W={W} H={H} d={d} region={rw}x{rh}", flush=True)
    dev = upload(frames, g.frame_pitch)
    f = O.Forest(W, H, d, rw, rh)
    idx = f.add_frames(frames)
    want = [f.export(i, with_counts=True) for i in idx]
    model = f.merge(idx[:T], 1, 2)
    # one frame per call, outputs full of ones beforehand
    occ = obg.empty_occ(g, T + 2).fill_(-1)
    for i in range(T):
        obg.obg_train_frame(g, dev[i:i + 1], 1, occ[i:i + 1])
    leaf = obg.empty_leafset(g).fill_(-1)
    obg.obg_merge(g, occ, T, 0, T, 1, 2, leaf)
    mask = obg.empty_mask(g, 2).fill_(-1)
    for i in range(2):
        obg.obg_classify(g, dev[T + i:T + i + 1], 1, leaf, mask[i:i + 1], occ[T + i:T + i + 1])
    torch.cuda.synchronize()
    for i in range(T + 2):
        assert np.array_equal(u32(occ[i]).reshape(want[i][0].shape), want[i][0]), f"trees of frame {i}"
    assert np.array_equal(u32(leaf).reshape(model.n_regions, -1), model.leafset()), "leaf set"
    for i in range(2):
        w = model.classify(frames[T + i])
        assert np.array_equal(u64(mask[i]).reshape(w.shape), w), f"mask of frame {i}"
    # all frames in one call, with pixel counts where they fit
    occ2 = obg.empty_occ(g, T + 2).fill_(-1)
    cnt = None
    if d <= 5:
        cnt = torch.full((T + 2, g.n_regions, 1 << (3 * d)), -1, dtype=torch.int32, device="cuda")
    obg.obg_train_frame(g, dev, T + 2, occ2, cnt)
    mask2 = obg.empty_mask(g, 2).fill_(-1)
    occ3 = obg.empty_occ(g, 2).fill_(-1)
    obg.obg_classify(g, dev[T:], 2, leaf, mask2, occ3)
    torch.cuda.synchronize()
    assert torch.equal(occ2, occ), "trees: one call differs from calls of one frame"
    assert torch.equal(occ3, occ[T:]), "fused trees of two frames"
    assert torch.equal(mask2, mask), "masks of two frames"
    if cnt is not None:
        for i in range(T + 2):
            assert np.array_equal(u32(cnt[i]).reshape(want[i][1].shape), want[i][1]), f"counts of frame {i}"


def test_repeat_runs_identical(env):
    """Results are exact integers; repeated launches must give identical bytes
    (a race in LDS or in the atomics would show here)."""
    obg, O = env
    rng = np.random.default_rng(99)
    W, H = 480, 270
    frames = brute.tiny_frames(rng, 8, W, H, n_colours=40, row_pitch=1440)
    for d, rw, rh in [(4, 0, 0), (5, 0, 0), (6, 0, 0), (4, 32, 32)]:
        g = obg.FrameGeom(W, H, d, region_w=rw, region_h=rh)
        dev = upload(frames, g.frame_pitch)
        outs = []
        for rep in range(3):
            occ, _, leaf, mask = run_pipeline(obg, g, dev, 6, dev[6:], 2, 1, 2)
            outs.append((occ.clone(), leaf.clone(), mask.clone()))
        for o in outs[1:]:
            assert all(torch.equal(a, b) for a, b in zip(outs[0], o))


def test_zero_frames_is_noop(env):
    obg, O = env
    g = obg.FrameGeom(64, 4, 4)
    occ = torch.full((1, 1, g.words), 7, dtype=torch.int32, device="cuda")
    dummy = torch.zeros(64 * 3 * 4, dtype=torch.uint8, device="cuda")
    obg.obg_train_frame(g, dummy, 0, occ)
    torch.cuda.synchronize()
    assert int(occ[0, 0, 0]) == 7


KNOBS = [
    {},
    {"layout": 2},
    {"mask_stage": 2},
    {"interleave": 2},
    {"classify_block": 256, "classify_span": 4096, "classify_wg_per_cu": 4},
    {"classify_span": 100, "mask_stage": 1},
    {"train_block": 256, "occ_wg_per_cu": 8},
    {"occ_wg_per_cu": 1},
    {"occ_blind": 1},
    {"occ_blind": 2},
    {"region_chunks": 2},
]


@pytest.mark.parametrize("knobs", KNOBS, ids=[",".join(f"{k}={v}" for k, v in kn.items()) or "default" for kn in KNOBS])
def test_launch_knobs_do_not_change_results(env, knobs):
    """Every launch shape gives the same bytes as the oracle (no LDS or atomic races)."""
    obg, O = env
    rng = np.random.default_rng(4242)
    cases = [(160, 24, 4, 0, 0), (333, 17, 5, 0, 0), (96, 40, 3, 32, 16), (200, 30, 6, 0, 0), (480, 64, 4, 32, 32)]
    try:
        for k, v in knobs.items():
            obg.obg_tune_set(k, v)
        for W, H, d, rw, rh in cases:
            rp = ((3 * W + 15) // 16) * 16
            frames = brute.tiny_frames(rng, 6, W, H, n_colours=11, row_pitch=rp)
            check_against_oracle(env, W, H, d, frames, 4, 1, 2, rw=rw, rh=rh, label=f"knobs{knobs}")
    finally:
        for k in obg.TUNE_KEYS:
            obg.obg_tune_set(k, 0)
