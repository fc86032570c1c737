"""Leaf sets of other streams, built by the oracle.

TEST INFRASTRUCTURE ONLY (imported by the test suite and by the CPU-baseline
leg of the benchmark).

A stream's own merged tree can hold nearly every depth-d cell (a 1920x1080
frame of the synthetic recipe covers all 32768 depth-5 cells), and then every
mask bit is 0 and a mask comparison shows nothing.  Classifying the same
frames against the merged tree of a smaller stream drawn with another seed
leaves both classes in the masks: the model's side length per depth is
chosen so that about a third to a half of a frame's pixels fall outside it.
Check Color (Algorithm 3) then has real work on both branches.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from oracle import octree

# side of the square training stream per depth, and its training frames
MODEL_SIDE = {1: 8, 2: 16, 3: 64, 4: 128, 5: 256, 6: 512, 7: 512, 8: 512}
MODEL_FRAMES = 20


@lru_cache(maxsize=None)
def _leafset(depth: int, seed: int) -> bytes:
    from synth.frames import StreamSpec, make_frames
    side = MODEL_SIDE[depth]
    spec = StreamSpec(side, side, MODEL_FRAMES, 0, seed=seed, stream=depth, bimodal_frac=0.2, drift_amp=0.1)
    frames = make_frames(spec, range(MODEL_FRAMES), device="cpu").numpy()
    forest = octree.Forest(side, side, depth)
    model = forest.merge(forest.add_frames(list(frames)), 1, 2)
    return model.leafset().tobytes()


def foreign_leafset(depth: int, n_regions: int = 1, seed: int = 909) -> np.ndarray:
    """[n_regions, ceil(8^d/32)] uint32: the merged tree (threshold 1/2) of a
    square stream of another seed, the same for every region."""
    one = np.frombuffer(_leafset(depth, seed), dtype=np.uint32)
    return np.ascontiguousarray(np.broadcast_to(one, (n_regions, one.size)))


def foreign_model(width: int, height: int, depth: int, region_w: int = 0, region_h: int = 0,
                  seed: int = 909) -> octree.Model:
    """The oracle's model of foreign_leafset for a frame geometry."""
    n_reg = octree.num_regions(width, height, region_w, region_h)
    return octree.Model.from_leafset(foreign_leafset(depth, n_reg, seed), width, height, depth, region_w, region_h)
