"""ctypes wrapper of the C oracle (octree_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and by
the CPU-baseline leg of the benchmark.  The GPU library never imports it.

Arrays in and out are numpy; layouts are the ones documented at the top of
octree_oracle.c (frames uint8 [H, row_pitch]; bitsets uint32
[n_regions, ceil(8^d/32)]; counts uint32 [n_regions, 8^d]; masks uint64
[H, ceil(W/64)]).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Iterable, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "octree_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(mutant: int = 0, out: Optional[str] = None) -> str:
    """Compile the oracle with gcc (a planted-mistake variant when mutant > 0)."""
    out = out or (LIB if mutant == 0 else os.path.join(HERE, f"liboracle_m{mutant}.so"))
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread",
           f"-DORC_MUTANT={mutant}", "-o", out + ".tmp", SRC]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_U32 = ctypes.c_uint32


def _bind(lib: ctypes.CDLL) -> ctypes.CDLL:
    sig = {
        "orc_forest_new": (_P, [_I, _I, _I, _I, _I]),
        "orc_forest_regions": (_I, [_P]),
        "orc_forest_add_frame": (_I, [_P, _P, _I64, _I]),
        "orc_forest_add_group": (_I, [_P, _P, _I, _I64, _I]),
        "orc_redraw": (_I, [_P, _I, _P, _I64, _P, _I64]),
        "orc_forest_add_occupancy": (_I, [_P, _P]),
        "orc_forest_frame_export": (_I, [_P, _I, _P, _P]),
        "orc_forest_frame_nodes": (_I64, [_P, _I]),
        "orc_forest_drop_frame": (None, [_P, _I]),
        "orc_forest_free": (None, [_P]),
        "orc_merge": (_P, [_P, _P, _I, _U32, _U32]),
        "orc_model_from_leafset": (_P, [_I, _I, _I, _I, _I, _P]),
        "orc_model_leafset": (_I, [_P, _P, _P]),
        "orc_classify": (_I, [_P, _P, _I64, _P]),
        "orc_check_pixel": (_I, [_P, _I, _I, ctypes.c_uint8, ctypes.c_uint8, ctypes.c_uint8]),
        "orc_model_free": (None, [_P]),
        "orc_release_pool": (None, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIBS = {}


def load(mutant: int = 0) -> ctypes.CDLL:
    if mutant not in _LIBS:
        path = LIB if mutant == 0 else os.path.join(HERE, f"liboracle_m{mutant}.so")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
            build(mutant, path)
        _LIBS[mutant] = _bind(ctypes.CDLL(path))
    return _LIBS[mutant]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def leaf_words(depth: int) -> int:
    return ((1 << (3 * depth)) + 31) // 32


def num_regions(width: int, height: int, region_w: int = 0, region_h: int = 0) -> int:
    if region_w == 0:
        return 1
    return ((width + region_w - 1) // region_w) * ((height + region_h - 1) // region_h)


class Forest:
    """The pruned per-frame (per-region) octrees of a sequence of frames."""

    def __init__(self, width, height, depth, region_w=0, region_h=0, mutant=0):
        self.lib = load(mutant)
        self.width, self.height, self.depth = width, height, depth
        self.region_w, self.region_h = region_w, region_h
        self.h = self.lib.orc_forest_new(width, height, depth, region_w, region_h)
        if not self.h:
            raise ValueError("oracle: bad geometry")
        self.n_regions = self.lib.orc_forest_regions(self.h)
        self.n = 0

    def add_frame(self, rgb: np.ndarray, store_levels: Optional[int] = None) -> int:
        rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
        assert rgb.ndim == 2 and rgb.shape[0] == self.height and rgb.shape[1] >= 3 * self.width
        lv = self.depth if store_levels is None else store_levels
        i = self.lib.orc_forest_add_frame(self.h, _ptr(rgb), rgb.shape[1], lv)
        if i < 0:
            raise ValueError("oracle: bad store_levels")
        self.n += 1
        return i

    def add_frames(self, frames: Iterable[np.ndarray], store_levels=None):
        return [self.add_frame(f, store_levels) for f in frames]

    def add_group(self, frames: Sequence[np.ndarray], store_levels: Optional[int] = None) -> int:
        """One tree (per region) holding the colours of every frame of the group."""
        fs = [np.ascontiguousarray(f, dtype=np.uint8) for f in frames]
        assert fs and all(f.shape == fs[0].shape for f in fs)
        assert fs[0].ndim == 2 and fs[0].shape[0] == self.height and fs[0].shape[1] >= 3 * self.width
        lv = self.depth if store_levels is None else store_levels
        ptrs = (ctypes.c_void_p * len(fs))(*[f.ctypes.data for f in fs])
        i = self.lib.orc_forest_add_group(self.h, ptrs, len(fs), fs[0].shape[1], lv)
        if i < 0:
            raise ValueError("oracle: bad group")
        self.n += 1
        return i

    def add_occupancy(self, occ: np.ndarray) -> int:
        occ = np.ascontiguousarray(occ, dtype=np.uint32).reshape(self.n_regions, leaf_words(self.depth))
        i = self.lib.orc_forest_add_occupancy(self.h, _ptr(occ))
        self.n += 1
        return i

    def export(self, frame: int, with_counts: bool = False):
        occ = np.zeros((self.n_regions, leaf_words(self.depth)), dtype=np.uint32)
        cnt = np.zeros((self.n_regions, 1 << (3 * self.depth)), dtype=np.uint32) if with_counts else None
        rc = self.lib.orc_forest_frame_export(self.h, frame, _ptr(occ), _ptr(cnt) if with_counts else None)
        if rc != 0:
            raise IndexError(frame)
        return (occ, cnt) if with_counts else occ

    def nodes(self, frame: int) -> int:
        return self.lib.orc_forest_frame_nodes(self.h, frame)

    def drop(self, frame: int):
        self.lib.orc_forest_drop_frame(self.h, frame)

    def redraw(self, frame: int, rgb: np.ndarray) -> np.ndarray:
        """The frame (which built tree `frame`) redrawn with that tree's leaf
        colours: [height, 3 * width] uint8."""
        rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
        out = np.zeros((self.height, 3 * self.width), dtype=np.uint8)
        rc = self.lib.orc_redraw(self.h, frame, _ptr(rgb), rgb.shape[1], _ptr(out), out.shape[1])
        if rc != 0:
            raise ValueError("oracle: a pixel's path is missing from the frame's tree")
        return out

    def merge(self, frames: Sequence[int], num: int, den: int) -> "Model":
        idx = np.ascontiguousarray(frames, dtype=np.int32)
        h = self.lib.orc_merge(self.h, _ptr(idx), len(idx), num, den)
        if not h:
            raise ValueError("oracle: bad merge arguments")
        return Model(self.lib, h, self.width, self.height, self.depth, self.region_w, self.region_h)

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.orc_forest_free(self.h)
            self.h = None


class Model:
    """Merged (background) octree of every region."""

    def __init__(self, lib, h, width, height, depth, region_w, region_h):
        self.lib, self.h = lib, h
        self.width, self.height, self.depth = width, height, depth
        self.region_w, self.region_h = region_w, region_h
        self.n_regions = num_regions(width, height, region_w, region_h)

    @classmethod
    def from_leafset(cls, leaf: np.ndarray, width, height, depth, region_w=0, region_h=0, mutant=0):
        lib = load(mutant)
        leaf = np.ascontiguousarray(leaf, dtype=np.uint32)
        h = lib.orc_model_from_leafset(width, height, depth, region_w, region_h, _ptr(leaf))
        if not h:
            raise ValueError("oracle: bad geometry")
        return cls(lib, h, width, height, depth, region_w, region_h)

    def leafset(self, with_dangling: bool = False):
        leaf = np.zeros((self.n_regions, leaf_words(self.depth)), dtype=np.uint32)
        dang = ctypes.c_int64(0)
        self.lib.orc_model_leafset(self.h, _ptr(leaf), ctypes.byref(dang))
        return (leaf, dang.value) if with_dangling else leaf

    def classify(self, rgb: np.ndarray) -> np.ndarray:
        rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
        assert rgb.ndim == 2 and rgb.shape[0] == self.height and rgb.shape[1] >= 3 * self.width
        mask = np.zeros((self.height, (self.width + 63) // 64), dtype=np.uint64)
        self.lib.orc_classify(self.h, _ptr(rgb), rgb.shape[1], _ptr(mask))
        return mask

    def check_pixel(self, x: int, y: int, r: int, g: int, b: int) -> bool:
        """Check Color (Algorithm 3) of one pixel at (x, y) with colour (r, g, b)
        against its region's merged tree: True = background."""
        rc = self.lib.orc_check_pixel(self.h, x, y, r, g, b)
        if rc < 0:
            raise IndexError((x, y))
        return bool(rc)

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.orc_model_free(self.h)
            self.h = None


def train(frames: Sequence[np.ndarray], width, height, depth, num, den,
          region_w=0, region_h=0, store_levels=None, with_counts=False, mutant=0):
    """Per-frame trees of all frames, then one merge over all of them.

    Returns (per-frame occupancy [T, n_reg, words], per-frame counts or None,
    merged Model)."""
    f = Forest(width, height, depth, region_w, region_h, mutant=mutant)
    idx = f.add_frames(frames, store_levels)
    occs, cnts = [], []
    for i in idx:
        if with_counts:
            o, c = f.export(i, True)
            cnts.append(c)
        else:
            o = f.export(i)
        occs.append(o)
    model = f.merge(idx, num, den)
    return np.stack(occs), (np.stack(cnts) if with_counts else None), model
