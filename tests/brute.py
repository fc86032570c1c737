"""Brute-force statements of what the method computes, for tiny inputs.

Independent of the oracle: no trees, no keys in the inner logic -- just sets
of quantised colour triples (r >> s, g >> s, b >> s) with s = 8 - depth, which
is what a depth-d pruned octree holds (Section 2: a level-N node keeps the N
most significant bits of each channel).
"""
from collections import Counter

import numpy as np


def quantised(frame, width, depth):
    """[H, W, 3] array of colour triples reduced to their top `depth` bits."""
    h = frame.shape[0]
    px = np.asarray(frame[:, : 3 * width], dtype=np.int64).reshape(h, width, 3)
    return px >> (8 - depth)


def region_ids(width, height, rw, rh):
    if rw == 0:
        return np.zeros((height, width), dtype=np.int64)
    cols = (width + rw - 1) // rw
    y = np.arange(height).reshape(-1, 1)
    x = np.arange(width).reshape(1, -1)
    return (y // rh) * cols + x // rw


def frame_sets(frame, width, height, depth, rw=0, rh=0):
    """Per region: the set of quantised triples present, and their pixel counts."""
    q = quantised(frame, width, depth)
    reg = region_ids(width, height, rw, rh)
    nreg = int(reg.max()) + 1
    sets = [Counter() for _ in range(nreg)]
    for y in range(height):
        for x in range(width):
            sets[reg[y, x]][tuple(int(v) for v in q[y, x])] += 1
    return sets


def merged_sets(frames, width, height, depth, num, den, rw=0, rh=0):
    """Per region: triples present in at least num/den of the frames."""
    per = [frame_sets(f, width, height, depth, rw, rh) for f in frames]
    T = len(frames)
    out = []
    for r in range(len(per[0])):
        c = Counter()
        for p in per:
            for t in p[r]:
                c[t] += 1
        out.append({t for t, n in c.items() if n * den >= num * T})
    return out


def grouped_sets(frames, group, width, height, depth, num, den, rw=0, rh=0):
    """Per region: triples present in at least num/den of the groups of
    `group` consecutive frames (the last group may be shorter); a group holds
    a triple when any of its frames does."""
    groups = [frames[i: i + group] for i in range(0, len(frames), group)]
    per = []
    for grp in groups:
        sets = [frame_sets(f, width, height, depth, rw, rh) for f in grp]
        per.append([set().union(*[s[r] for s in sets]) for r in range(len(sets[0]))])
    G = len(groups)
    out = []
    for r in range(len(per[0])):
        c = Counter()
        for p in per:
            for t in p[r]:
                c[t] += 1
        out.append({t for t, n in c.items() if n * den >= num * G})
    return out


def mask_bits(frame, kept, width, height, depth, rw=0, rh=0):
    """bool [H, W]: True where the pixel's triple is not in its region's set."""
    q = quantised(frame, width, depth)
    reg = region_ids(width, height, rw, rh)
    out = np.zeros((height, width), dtype=bool)
    for y in range(height):
        for x in range(width):
            out[y, x] = tuple(int(v) for v in q[y, x]) not in kept[reg[y, x]]
    return out


def triple_of_key(key, depth):
    """Read a path key back as the triple it stands for (digit i = 4r+2g+b of level i)."""
    r = g = b = 0
    for i in range(depth):
        digit = (key >> (3 * (depth - 1 - i))) & 7
        r = (r << 1) | (digit >> 2)
        g = (g << 1) | ((digit >> 1) & 1)
        b = (b << 1) | (digit & 1)
    return (r, g, b)


def bitset_keys(words):
    w = np.asarray(words, dtype=np.uint32).ravel()
    bits = np.unpackbits(w.view(np.uint8), bitorder="little")
    return [int(k) for k in np.nonzero(bits)[0]]


def bitset_triples(words, depth):
    return {triple_of_key(k, depth) for k in bitset_keys(words)}


def unpack_mask(mask, width):
    m = np.asarray(mask, dtype=np.uint64)
    bits = np.unpackbits(m.view(np.uint8), axis=-1, bitorder="little")
    return bits[:, :width].astype(bool), bits[:, width:]


def tiny_frames(rng, n, width, height, n_colours=None, row_pitch=None):
    """Random frames; with n_colours, pixels come from a small shared palette."""
    rp = row_pitch or 3 * width
    out = []
    pal = rng.integers(0, 256, size=(n_colours, 3)) if n_colours else None
    for _ in range(n):
        f = np.zeros((height, rp), dtype=np.uint8)
        if pal is not None:
            px = pal[rng.integers(0, n_colours, size=(height, width))]
        else:
            px = rng.integers(0, 256, size=(height, width, 3))
        f[:, : 3 * width] = px.reshape(height, 3 * width)
        out.append(f)
    return out
