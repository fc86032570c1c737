"""Section 5's agreement figures, written out plainly (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.

Section 5 scores a foreground detector by its background class: with Tn, Tp,
Fn and Fp the numbers of true negatives, true positives, false negatives and
false positives (positive = foreground),

    P0 = Tn / (Tn + Fn),   R0 = Tn / (Tn + Fp),   F0 = 2 P0 R0 / (P0 + R0).

Reading: when a denominator is zero the ratio is taken as 0 (no background
pixel predicted, or none present), and F0 = 0 when P0 + R0 = 0.
"""
import numpy as np


def confusion(mask, truth):
    """mask, truth: bool arrays of the same shape, True = foreground.
    Returns (tp, fp, fn, tn) as Python ints, counted pixel by pixel."""
    mask = np.asarray(mask, dtype=bool)
    truth = np.asarray(truth, dtype=bool)
    assert mask.shape == truth.shape
    tp = fp = fn = tn = 0
    for m, t in zip(mask.reshape(-1).tolist(), truth.reshape(-1).tolist()):
        if m and t:
            tp += 1
        elif m and not t:
            fp += 1
        elif t:
            fn += 1
        else:
            tn += 1
    return tp, fp, fn, tn


def background_scores(tp, fp, fn, tn):
    """(P0, R0, F0) of the background class, as defined in Section 5."""
    p0 = tn / (tn + fn) if tn + fn else 0.0
    r0 = tn / (tn + fp) if tn + fp else 0.0
    f0 = 2.0 * p0 * r0 / (p0 + r0) if p0 + r0 else 0.0
    return p0, r0, f0
