"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own code: hand-worked keys and
merge cases (golden files), brute-force sets of quantised colours, closed
forms and invariants.  The last test plants mistakes in the oracle (compile
time switches) and shows that each one is caught by at least one pin.
"""
import json
import os

import numpy as np
import pytest

import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_keys():
    rows = []
    with open(os.path.join(GOLDEN, "path_keys.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                d, r, g, b, k = (int(v) for v in line.split())
                rows.append((d, r, g, b, k))
    return rows


def _golden_merges():
    with open(os.path.join(GOLDEN, "merge_examples.json")) as f:
        return json.load(f)["cases"]


def _frame_from_rows(rows):
    a = np.asarray(rows, dtype=np.uint8)
    return a.reshape(a.shape[0], -1), a.shape[1], a.shape[0]


# ---------------------------------------------------------------------------
# reusable checks (each returns normally or raises AssertionError)

def check_golden_keys(O, mutant=0):
    for d, r, g, b, k in _golden_keys():
        fr = np.array([[r, g, b]], dtype=np.uint8)
        f = O.Forest(1, 1, d, mutant=mutant)
        f.add_frame(fr)
        assert brute.bitset_keys(f.export(0)) == [k], (d, r, g, b, k)


def check_golden_merges(O, mutant=0):
    for case in _golden_merges():
        d = case["depth"]
        frames = []
        for fr in case["train"]:
            a, w, h = _frame_from_rows(fr)
            frames.append(a)
        f = O.Forest(w, h, d, mutant=mutant)
        idx = f.add_frames(frames)
        m = f.merge(idx, case["num"], case["den"])
        leaf, dang = m.leafset(with_dangling=True)
        assert brute.bitset_keys(leaf) == case["leaves"], case["name"]
        assert dang == case["dangling"], case["name"]
        t, tw, th = _frame_from_rows(case["test"])
        m2 = O.Model.from_leafset(leaf, tw, th, d, mutant=mutant)
        got = [int(v) for v in m2.classify(t)[:, 0]]
        assert got == case["mask_rows"], case["name"]


def check_brute(O, seed, mutant=0, store_levels=8, regions=(0, 0)):
    rng = np.random.default_rng(seed)
    rw, rh = regions
    for trial in range(6):
        d = int(rng.integers(1, 9))
        W = int(rng.integers(1, 13))
        H = int(rng.integers(1, 9))
        if trial == 0 and rw:
            W, H = 4 * rw - 1, 3 * rh + 1     # several ragged region rows and columns
        T = int(rng.integers(1, 7))
        ncol = int(rng.integers(2, 10)) if trial % 2 == 0 else None
        frames = brute.tiny_frames(rng, T + 2, W, H, n_colours=ncol, row_pitch=3 * W + 5)
        train, test = frames[:T], frames[T:]
        k = int(rng.integers(1, T + 1))
        num, den = k, T          # threshold k/T: keep keys in >= k frames
        f = O.Forest(W, H, d, rw, rh, mutant=mutant)
        idx = f.add_frames(train, store_levels)
        for i, fr in zip(idx, train):
            occ, cnt = f.export(i, with_counts=True)
            sets = brute.frame_sets(fr, W, H, d, rw, rh)
            assert len(sets) == occ.shape[0]
            for r, s in enumerate(sets):
                assert brute.bitset_triples(occ[r], d) == set(s), (trial, r)
                got = {brute.triple_of_key(kk, d): int(cnt[r, kk]) for kk in np.nonzero(cnt[r])[0]}
                assert got == dict(s), (trial, r)
        model = f.merge(idx, num, den)
        kept = brute.merged_sets(train, W, H, d, num, den, rw, rh)
        leaf = model.leafset()
        for r in range(leaf.shape[0]):
            assert brute.bitset_triples(leaf[r], d) == kept[r], (trial, r)
        for fr in test + train:
            got, pad = brute.unpack_mask(model.classify(fr), W)
            assert not pad.any()
            assert np.array_equal(got, brute.mask_bits(fr, kept, W, H, d, rw, rh)), trial


def check_groups(O, seed, mutant=0):
    """Trees of groups of frames (Section 3): each group's tree holds the
    colours of all its frames; the merge counts groups."""
    rng = np.random.default_rng(seed)
    for trial in range(5):
        d = int(rng.integers(1, 7))
        W, H = int(rng.integers(1, 11)), int(rng.integers(1, 7))
        rw, rh = ((3, 2) if trial % 2 else (0, 0))
        T = int(rng.integers(1, 9))
        gsz = int(rng.integers(1, T + 1))
        frames = brute.tiny_frames(rng, T + 2, W, H, n_colours=int(rng.integers(2, 8)), row_pitch=3 * W + 3)
        train, test = frames[:T], frames[T:]
        G = (T + gsz - 1) // gsz
        k = int(rng.integers(1, G + 1))
        f = O.Forest(W, H, d, rw, rh, mutant=mutant)
        idx = [f.add_group(train[i: i + gsz]) for i in range(0, T, gsz)]
        assert len(idx) == G
        model = f.merge(idx, k, G)
        kept = brute.grouped_sets(train, gsz, W, H, d, k, G, rw, rh)
        leaf = model.leafset()
        for r in range(leaf.shape[0]):
            assert brute.bitset_triples(leaf[r], d) == kept[r], (trial, r)
        for fr in test:
            got, _ = brute.unpack_mask(model.classify(fr), W)
            assert np.array_equal(got, brute.mask_bits(fr, kept, W, H, d, rw, rh)), trial
    # one group of every frame at threshold 1: the union of the frames' colours
    frames = brute.tiny_frames(rng, 4, 6, 5, n_colours=12)
    f = O.Forest(6, 5, 3, mutant=mutant)
    union = set().union(*[brute.frame_sets(fr, 6, 5, 3)[0] for fr in frames])
    assert brute.bitset_triples(f.merge([f.add_group(frames)], 1, 1).leafset()[0], 3) == union


def check_redraw(O, seed, mutant=0):
    """Redraw with the frame's own pruned tree (Section 2): every pixel takes
    its leaf's zero-filled colour, i.e. each channel keeps its top d bits; the
    redrawn colours are exactly the tree's leaves."""
    rng = np.random.default_rng(seed)
    for trial in range(6):
        d = int(rng.integers(1, 9))
        W, H = int(rng.integers(1, 12)), int(rng.integers(1, 7))
        rw, rh = ((4, 3) if trial % 3 == 2 else (0, 0))
        fr = brute.tiny_frames(rng, 1, W, H, n_colours=(None if trial % 2 else 6), row_pitch=3 * W + 7)[0]
        f = O.Forest(W, H, d, rw, rh, mutant=mutant)
        i = f.add_frame(fr)
        out = f.redraw(i, fr)
        q = brute.quantised(fr, W, d)
        assert np.array_equal(out.reshape(H, W, 3), (q << (8 - d)).astype(np.uint8)), trial
        leaves = set().union(*[brute.bitset_triples(w, d) for w in f.export(i)])
        assert {tuple(int(v) >> (8 - d) for v in px) for px in out.reshape(-1, 3)} == leaves, trial
        if d == 8:
            assert np.array_equal(out, fr[:, : 3 * W])


def check_pixel_checks(O, seed, mutant=0):
    """Check Color of one pixel at a time (the checker of the sampled pixels of
    full-size runs) against brute-force membership of the pixel's quantised
    colour in its region's kept set.  Regions are not square, frames are not
    square, and the leaf sets are sparse (the intersection of the training
    frames' trees), so a mixed-up channel or region index changes answers.
    Every answer also equals the frame-wide labels of the same model."""
    rng = np.random.default_rng(seed)
    for trial, (rw, rh) in enumerate([(3, 2), (5, 1), (2, 4), (0, 0), (4, 3)]):
        d = int(rng.integers(1, 9)) if trial else 3
        s = 8 - d
        W, H = int(rng.integers(7, 14)), int(rng.integers(3, 7))
        T = int(rng.integers(2, 5))
        frames = brute.tiny_frames(rng, T + 2, W, H, n_colours=int(rng.integers(3, 9)), row_pitch=3 * W + 5)
        train, test = frames[:T], frames[T:]
        f = O.Forest(W, H, d, rw, rh, mutant=mutant)
        model = f.merge(f.add_frames(train), T, T)
        kept = brute.merged_sets(train, W, H, d, T, T, rw, rh)
        reg = brute.region_ids(W, H, rw, rh)
        for fr in test + train:
            px = np.asarray(fr[:, : 3 * W], dtype=np.int64).reshape(H, W, 3)
            labels, _ = brute.unpack_mask(model.classify(fr), W)
            for y in range(H):
                for x in range(W):
                    r, g, b = (int(v) for v in px[y, x])
                    bg = model.check_pixel(x, y, r, g, b)
                    assert bg == ((r >> s, g >> s, b >> s) in kept[reg[y, x]]), (trial, x, y)
                    assert bg == (not labels[y, x]), (trial, x, y)
        # a colour kept in one region only: background there, foreground elsewhere
        for r0 in range(len(kept)):
            only = kept[r0] - set().union(set(), *[kept[q] for q in range(len(kept)) if q != r0])
            for t in sorted(only)[:2]:
                c = [v << s for v in t]
                for y in range(H):
                    for x in range(W):
                        assert model.check_pixel(x, y, *c) == (reg[y, x] == r0), (trial, t, x, y)
        for x, y in [(-1, 0), (0, -1), (W, 0), (0, H)]:
            with pytest.raises(IndexError):
                model.check_pixel(x, y, 0, 0, 0)


def check_union_and_training_background(O, seed, mutant=0):
    """Threshold of one frame: every training pixel is background."""
    rng = np.random.default_rng(seed)
    W, H, d, T = 9, 7, 4, 5
    frames = brute.tiny_frames(rng, T, W, H)
    f = O.Forest(W, H, d, mutant=mutant)
    idx = f.add_frames(frames)
    m = f.merge(idx, 1, T)
    for fr in frames:
        got, _ = brute.unpack_mask(m.classify(fr), W)
        assert not got.any()


# ---------------------------------------------------------------------------
# tests

def test_golden_path_keys(oracle_lib):
    check_golden_keys(oracle_lib)


def test_golden_merge_cases(oracle_lib):
    check_golden_merges(oracle_lib)


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_plain(oracle_lib, seed):
    check_brute(oracle_lib, seed)


@pytest.mark.parametrize("seed", range(3))
def test_brute_force_regions(oracle_lib, seed):
    check_brute(oracle_lib, 100 + seed, regions=(3, 2))


@pytest.mark.parametrize("seed", range(3))
def test_brute_force_groups(oracle_lib, seed):
    check_groups(oracle_lib, 300 + seed)


@pytest.mark.parametrize("seed", range(2))
def test_redraw_keeps_top_bits(oracle_lib, seed):
    check_redraw(oracle_lib, 500 + seed)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_check_pixel_against_brute_force(oracle_lib, seed):
    check_pixel_checks(oracle_lib, 6000 + seed)


def test_brute_force_direct_depth(oracle_lib):
    """Storing at the kept depth directly gives the same trees as pruning."""
    check_brute(oracle_lib, 7, store_levels=None)


def test_prune_equals_direct_build(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(11)
    frames = brute.tiny_frames(rng, 3, 17, 5)
    for d in range(1, 9):
        for lv in range(d, 9):
            a = O.Forest(17, 5, d)
            b = O.Forest(17, 5, d)
            for fr in frames:
                a.add_frame(fr, lv)
                b.add_frame(fr, d)
            for i in range(3):
                oa, ca = a.export(i, True)
                ob, cb = b.export(i, True)
                assert np.array_equal(oa, ob) and np.array_equal(ca, cb)
                assert a.nodes(i) == b.nodes(i)


def test_union_threshold_all_training_background(oracle_lib):
    check_union_and_training_background(oracle_lib, 3)


def test_intersection_at_threshold_one(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(5)
    W, H, d, T = 6, 6, 3, 4
    frames = brute.tiny_frames(rng, T, W, H, n_colours=5)
    f = O.Forest(W, H, d)
    idx = f.add_frames(frames)
    inter = set.intersection(*[set(brute.frame_sets(fr, W, H, d)[0]) for fr in frames])
    assert brute.bitset_triples(f.merge(idx, 1, 1).leafset()[0], d) == inter
    # any threshold above one keeps nothing: every pixel is foreground
    m = f.merge(idx, 3, 2)
    assert not m.leafset().any()
    got, _ = brute.unpack_mask(m.classify(frames[0]), W)
    assert got.all()


def test_closed_form_frame_count(oracle_lib):
    """Merged leaf set == keys whose frame count C(k) satisfies C*den >= num*T."""
    O = oracle_lib
    rng = np.random.default_rng(21)
    W, H, d, T = 10, 8, 2, 7
    frames = brute.tiny_frames(rng, T, W, H, n_colours=12)
    f = O.Forest(W, H, d)
    idx = f.add_frames(frames)
    occ = np.stack([f.export(i)[0] for i in idx])
    bits = np.unpackbits(occ.view(np.uint8), axis=1, bitorder="little")[:, : 1 << (3 * d)]
    C = bits.sum(axis=0)
    for num, den in [(1, 10), (3, 10), (1, 2), (7, 10), (1, 1), (2, 7), (3, 7)]:
        want = [int(k) for k in np.nonzero(C * den >= num * T)[0]]
        assert brute.bitset_keys(f.merge(idx, num, den).leafset()) == want, (num, den)


def test_monotone_shrink(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(8)
    W, H, d, T = 12, 9, 3, 9
    frames = brute.tiny_frames(rng, T, W, H, n_colours=15)
    f = O.Forest(W, H, d)
    idx = f.add_frames(frames)
    prev = None
    for k in range(1, T + 2):
        cur = set(brute.bitset_keys(f.merge(idx, k, T).leafset()))
        if prev is not None:
            assert cur <= prev
        prev = cur
    assert prev == set()


def test_parent_closure_across_depths(oracle_lib):
    """Leaf set at depth d-1 contains the parent of every leaf at depth d."""
    O = oracle_lib
    rng = np.random.default_rng(9)
    W, H, T = 11, 6, 5
    frames = brute.tiny_frames(rng, T, W, H, n_colours=20)
    for d in range(2, 9):
        fa, fb = O.Forest(W, H, d), O.Forest(W, H, d - 1)
        ia, ib = fa.add_frames(frames), fb.add_frames(frames)
        la = brute.bitset_keys(fa.merge(ia, 1, 2).leafset())
        lb = set(brute.bitset_keys(fb.merge(ib, 1, 2).leafset()))
        assert {k >> 3 for k in la} <= lb


def test_low_bits_ignored(oracle_lib):
    """Flipping any of the 8-d low bits of any channel leaves masks unchanged."""
    O = oracle_lib
    rng = np.random.default_rng(10)
    W, H, T = 13, 5, 4
    frames = brute.tiny_frames(rng, T + 1, W, H, n_colours=6)
    for d in range(1, 8):
        f = O.Forest(W, H, d)
        m = f.merge(f.add_frames(frames[:T]), 1, 2)
        base = m.classify(frames[T])
        noise = rng.integers(0, 1 << (8 - d), size=frames[T].shape).astype(np.uint8)
        flipped = frames[T] ^ noise
        assert np.array_equal(m.classify(flipped), base), d


def test_depth8_is_exact_colour_membership(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(12)
    W, H = 7, 4
    frames = brute.tiny_frames(rng, 3, W, H, n_colours=9)
    f = O.Forest(W, H, 8)
    m = f.merge(f.add_frames(frames[:2]), 1, 2)
    seen = set()
    for fr in frames[:2]:
        seen |= {tuple(p) for p in fr[:, : 3 * W].reshape(-1, 3).tolist()}
    got, _ = brute.unpack_mask(m.classify(frames[2]), W)
    want = np.array([tuple(p) not in seen for p in frames[2][:, : 3 * W].reshape(-1, 3).tolist()])
    assert np.array_equal(got.ravel(), want)


def test_one_region_covering_frame_equals_plain(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(13)
    W, H, d = 10, 6, 3
    frames = brute.tiny_frames(rng, 5, W, H, n_colours=8)
    a, b = O.Forest(W, H, d), O.Forest(W, H, d, W, H)
    ma = a.merge(a.add_frames(frames[:4]), 1, 2)
    mb = b.merge(b.add_frames(frames[:4]), 1, 2)
    assert np.array_equal(ma.leafset(), mb.leafset())
    assert np.array_equal(ma.classify(frames[4]), mb.classify(frames[4]))


def test_counts_sum_to_region_pixels(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(14)
    W, H, d = 23, 9, 4
    fr = brute.tiny_frames(rng, 1, W, H)[0]
    f = O.Forest(W, H, d, 8, 4)
    f.add_frame(fr, 8)
    _, cnt = f.export(0, True)
    reg = brute.region_ids(W, H, 8, 4)
    assert list(cnt.sum(axis=1)) == [int((reg == r).sum()) for r in range(cnt.shape[0])]


def test_trees_from_occupancy_equal_trees_from_frames(oracle_lib):
    """The zero-fill colour of every leaf (Section 2) rebuilds the same tree."""
    O = oracle_lib
    rng = np.random.default_rng(15)
    W, H, d = 9, 9, 3
    frames = brute.tiny_frames(rng, 4, W, H, n_colours=10)
    a, b = O.Forest(W, H, d, 4, 4), O.Forest(W, H, d, 4, 4)
    ia = a.add_frames(frames)
    ib = [b.add_occupancy(a.export(i)) for i in ia]
    for i, j in zip(ia, ib):
        assert np.array_equal(a.export(i), b.export(j))
    ma, mb = a.merge(ia, 1, 2), b.merge(ib, 1, 2)
    assert np.array_equal(ma.leafset(), mb.leafset())
    mc = O.Model.from_leafset(ma.leafset(), W, H, d, 4, 4)
    for fr in frames:
        assert np.array_equal(ma.classify(fr), mc.classify(fr))


# ---------------------------------------------------------------------------
# planted mistakes

MUTANTS = {
    1: "red/green swapped in the child index",
    2: "colour bits read least significant first",
    3: "strict > in the merge threshold",
    4: "merge counts trees without the child test",
    5: "Check Color skips the last level",
    6: "region grid transposed",
    7: "pruning removes one level too many",
    8: "mask polarity inverted",
    9: "numberOfTrees off by one in the merge test",
    10: "a group's tree built from its first frame only",
    11: "one pixel's check takes red and blue exchanged",
    12: "one pixel's check looks its region up in the transposed grid",
}


def _pin_battery(O, mutant):
    check_golden_keys(O, mutant)
    check_golden_merges(O, mutant)
    for s in range(3):
        check_brute(O, 1000 + s, mutant)
    check_brute(O, 2000, mutant, regions=(3, 2))
    check_union_and_training_background(O, 3000, mutant)
    check_groups(O, 4000, mutant)
    check_redraw(O, 5000, mutant)
    check_pixel_checks(O, 6000, mutant)


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_reject_planted_mistake(oracle_lib, mutant):
    oracle_lib.build(mutant)
    with pytest.raises(AssertionError):
        _pin_battery(oracle_lib, mutant)


def test_pin_battery_passes_unmutated(oracle_lib):
    _pin_battery(oracle_lib, 0)
