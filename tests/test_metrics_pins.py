"""Pins of the Section 5 agreement figures (oracle/metrics.py)."""
import numpy as np

from oracle import metrics as M


def test_hand_worked_example():
    # 2 x 5 frame; 1 = foreground
    truth = np.array([[0, 0, 1, 1, 0],
                      [0, 0, 0, 1, 0]], dtype=bool)
    mask = np.array([[0, 1, 1, 0, 0],
                     [1, 0, 0, 1, 0]], dtype=bool)
    # tp: (0,2), (1,3) -> 2; fp: (0,1), (1,0) -> 2; fn: (0,3) -> 1; tn: 10 - 5 = 5
    assert M.confusion(mask, truth) == (2, 2, 1, 5)
    p0, r0, f0 = M.background_scores(2, 2, 1, 5)
    assert abs(p0 - 5 / 6) < 1e-15
    assert abs(r0 - 5 / 7) < 1e-15
    assert abs(f0 - 2 * (5 / 6) * (5 / 7) / (5 / 6 + 5 / 7)) < 1e-15
    assert abs(f0 - 10 / 13) < 1e-12            # 2 Tn / (2 Tn + Fn + Fp) = 10 / 13


def test_perfect_and_inverted():
    rng = np.random.default_rng(0)
    truth = rng.random((7, 9)) < 0.3
    tp, fp, fn, tn = M.confusion(truth, truth)
    assert fp == fn == 0 and tp == truth.sum() and tn == (~truth).sum()
    assert M.background_scores(tp, fp, fn, tn)[2] == 1.0
    tp, fp, fn, tn = M.confusion(~truth, truth)
    assert tp == tn == 0
    assert M.background_scores(tp, fp, fn, tn) == (0.0, 0.0, 0.0)


def test_f0_closed_form():
    rng = np.random.default_rng(1)
    for _ in range(200):
        tp, fp, fn, tn = (int(v) for v in rng.integers(0, 1000, 4))
        if tn == 0:
            continue
        f0 = M.background_scores(tp, fp, fn, tn)[2]
        assert abs(f0 - 2 * tn / (2 * tn + fn + fp)) < 1e-12


def test_counts_sum_to_pixels():
    rng = np.random.default_rng(2)
    m, t = rng.random((3, 11, 13)) < 0.5, rng.random((3, 11, 13)) < 0.2
    c = M.confusion(m, t)
    assert sum(c) == m.size
    assert c[0] + c[2] == t.sum() and c[0] + c[1] == m.sum()
