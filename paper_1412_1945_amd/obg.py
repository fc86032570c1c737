"""Python binding of libobg.so (ctypes; argument marshalling only).

Every function has the name of the C entry point it calls.  Tensors are torch
tensors on the GPU; the library receives their device pointers and the current
HIP stream, and all the work runs in the library's kernels.  A missing or
unloadable library raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libobg.so")

OBG_OK, OBG_EINVAL, OBG_EALIGN, OBG_EHIP, OBG_ENOMEM = 0, -1, -2, -3, -4


class ObgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"obg error {code}: {msg}")
        self.code = code


class Geom(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("row_pitch", ctypes.c_int64), ("frame_pitch", ctypes.c_int64),
        ("depth", ctypes.c_int32),
        ("region_w", ctypes.c_int32), ("region_h", ctypes.c_int32),
    ]


class PlanStream(ctypes.Structure):
    _fields_ = [("geom", Geom), ("thr_num", ctypes.c_uint32), ("thr_den", ctypes.c_uint32),
                ("max_train", ctypes.c_int32), ("max_test", ctypes.c_int32)]


class WorkItem(ctypes.Structure):
    _fields_ = [
        ("stream", ctypes.c_int32), ("n_train", ctypes.c_int32), ("n_test", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("train_rgb", ctypes.c_void_p), ("test_rgb", ctypes.c_void_p),
        ("occ", ctypes.c_void_p), ("leafset", ctypes.c_void_p), ("mask", ctypes.c_void_p),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n_streams", ctypes.c_int32),
        ("max_train_items", ctypes.c_int64), ("max_classify_items", ctypes.c_int64),
        ("train_block", ctypes.c_int32), ("train_wg_per_cu", ctypes.c_int32),
        ("train_items_per_wg", ctypes.c_int32),
        ("classify_block", ctypes.c_int32), ("classify_wg_per_cu", ctypes.c_int32),
        ("classify_span", ctypes.c_int32),
        ("classify_round_robin", ctypes.c_int32), ("per_depth_launches", ctypes.c_int32),
        ("graph", ctypes.c_int32), ("tune_candidates", ctypes.c_int32),
        ("tune_default_ms", ctypes.c_double), ("tune_best_ms", ctypes.c_double),
    ]


ITEM_OK, ITEM_BAD_STREAM, ITEM_BAD_COUNT, ITEM_NULL, ITEM_ALIGN, ITEM_DUPLICATE = 0, 1, 2, 3, 4, 5


class ServeStream(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("n_train", ctypes.c_int32), ("thr_num", ctypes.c_uint32), ("thr_den", ctypes.c_uint32),
                ("region_w", ctypes.c_int32), ("region_h", ctypes.c_int32)]


class ServeConfig(ctypes.Structure):
    _fields_ = [
        ("streams", ctypes.POINTER(ServeStream)), ("n_streams", ctypes.c_int32),
        ("arrivals", ctypes.POINTER(ctypes.POINTER(ctypes.c_double))),
        ("n_arrivals", ctypes.POINTER(ctypes.c_int32)),
        ("speed", ctypes.c_double), ("budget_bytes", ctypes.c_uint64),
        ("max_inflight", ctypes.c_int32), ("max_batch_frames", ctypes.c_int32),
        ("remerge_period", ctypes.c_int32), ("remerge_window", ctypes.c_int32),
        ("ingest", ctypes.c_void_p), ("ingest_ctx", ctypes.c_void_p),
        ("checksums", ctypes.POINTER(ctypes.c_uint64)), ("checksum_stride", ctypes.c_int32),
        ("watch_streams", ctypes.POINTER(ctypes.c_int32)), ("n_watch", ctypes.c_int32),
        ("watch_masks", ctypes.POINTER(ctypes.POINTER(ctypes.c_uint64))), ("watch_max_frames", ctypes.c_int32),
        ("state_in", ctypes.c_void_p), ("state_out", ctypes.c_void_p),
    ]


class ServeStats(ctypes.Structure):
    _fields_ = [
        ("frames_arrived", ctypes.c_int64), ("frames_served", ctypes.c_int64),
        ("train_frames", ctypes.c_int64), ("test_frames", ctypes.c_int64), ("pixels", ctypes.c_int64),
        ("batches", ctypes.c_int64), ("merges", ctypes.c_int64), ("admission_waits", ctypes.c_int64),
        ("wall_s", ctypes.c_double),
        ("lat_p50_ms", ctypes.c_double), ("lat_p99_ms", ctypes.c_double), ("lat_max_ms", ctypes.c_double),
        ("lat_mean_ms", ctypes.c_double), ("peak_bytes", ctypes.c_double),
        ("train_pixels", ctypes.c_int64), ("test_pixels", ctypes.c_int64),
        ("busy_s", ctypes.c_double), ("path_busy_s", ctypes.c_double),
    ]


_lib: Optional[ctypes.CDLL] = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "or python paper_1412_1945_amd/build.py")
        lib = ctypes.CDLL(LIB_PATH)
        P, I32, I64, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        G = ctypes.POINTER(Geom)
        sigs = {
            "obg_num_regions": (I64, [G]),
            "obg_occ_words": (I64, [G]),
            "obg_mask_words": (I64, [G]),
            "obg_train_frame": (ctypes.c_int, [G, P, I32, P, P, P]),
            "obg_merge": (ctypes.c_int, [G, P, I32, I32, I32, U32, U32, P, P]),
            "obg_merge_groups": (ctypes.c_int, [G, P, I32, I32, I32, I32, U32, U32, P, P]),
            "obg_quantize": (ctypes.c_int, [G, P, I32, P, P]),
            "obg_score": (ctypes.c_int, [G, P, P, I32, P, P]),
            "obg_classify": (ctypes.c_int, [G, P, I32, P, P, P, P]),
            "obg_tune_set": (ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
            "obg_tune_get": (ctypes.c_int, [ctypes.c_int]),
            "obg_probe": (ctypes.c_int, [ctypes.c_int, P, P, I64, P, I32, P]),
            "obg_probe_shaped": (ctypes.c_int, [ctypes.POINTER(ProbeShape), P, P, I64, P, P]),
            "obg_plan_create": (ctypes.c_int, [ctypes.POINTER(PlanStream), I32, ctypes.POINTER(ctypes.c_void_p)]),
            "obg_plan_tune": (ctypes.c_int, [P, P, I32, P]),
            "obg_batch_run": (ctypes.c_int, [P, P, I32, P]),
            "obg_plan_info_get": (ctypes.c_int, [P, ctypes.POINTER(PlanInfo)]),
            "obg_plan_destroy": (None, [P]),
            "obg_batch_run_noalloc": (ctypes.c_int, [ctypes.POINTER(PlanStream), I32, P, I32, P]),
            "obg_serve_run": (ctypes.c_int, [ctypes.POINTER(ServeConfig), ctypes.POINTER(ServeStats)]),
            "obg_serve_state_bytes": (I64, [ctypes.POINTER(ServeStream), I32, I32]),
            "obg_last_error": (ctypes.c_char_p, []),
            "obg_version": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    return ["obg_num_regions", "obg_occ_words", "obg_mask_words", "obg_train_frame",
            "obg_merge", "obg_merge_groups", "obg_classify", "obg_quantize", "obg_score", "obg_tune_set", "obg_tune_get", "obg_probe", "obg_probe_shaped",
            "obg_plan_create", "obg_plan_tune", "obg_batch_run", "obg_plan_info_get", "obg_plan_destroy",
            "obg_batch_run_noalloc",
            "obg_serve_run", "obg_serve_state_bytes", "obg_last_error", "obg_version"]


@dataclass
class FrameGeom:
    width: int
    height: int
    depth: int
    row_pitch: int = 0
    frame_pitch: int = 0
    region_w: int = 0
    region_h: int = 0

    def __post_init__(self):
        if self.row_pitch == 0:
            self.row_pitch = ((3 * self.width + 15) // 16) * 16
        if self.frame_pitch == 0:
            self.frame_pitch = self.height * self.row_pitch

    def c(self) -> Geom:
        return Geom(self.width, self.height, self.row_pitch, self.frame_pitch, self.depth,
                    self.region_w, self.region_h)

    @property
    def n_regions(self) -> int:
        if self.region_w == 0:
            return 1
        return (-(-self.width // self.region_w)) * (-(-self.height // self.region_h))

    @property
    def words(self) -> int:
        return max(1, (1 << (3 * self.depth)) // 32)

    @property
    def mask_row_words(self) -> int:
        return (self.width + 63) // 64


def _check(rc: int):
    if rc != OBG_OK:
        raise ObgError(rc, load().obg_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _need(t: torch.Tensor, dtype, numel: int, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")


def _frames_ok(g: FrameGeom, rgb: torch.Tensor, n_frames: int):
    _need(rgb, torch.uint8, 0, "rgb")
    need = n_frames * g.frame_pitch
    if rgb.numel() < need:
        raise ValueError(f"rgb holds {rgb.numel()} bytes, {n_frames} frames need {need}")


def obg_num_regions(g: FrameGeom) -> int:
    return load().obg_num_regions(ctypes.byref(g.c()))


def obg_occ_words(g: FrameGeom) -> int:
    return load().obg_occ_words(ctypes.byref(g.c()))


def obg_mask_words(g: FrameGeom) -> int:
    return load().obg_mask_words(ctypes.byref(g.c()))


def obg_train_frame(g: FrameGeom, rgb: torch.Tensor, n_frames: int, occ: torch.Tensor,
                    counts: Optional[torch.Tensor] = None, stream=None):
    _frames_ok(g, rgb, n_frames)
    _need(occ, torch.int32, n_frames * g.n_regions * g.words, "occ")
    if counts is not None:
        _need(counts, torch.int32, n_frames * g.n_regions * (1 << (3 * g.depth)), "counts")
    _check(load().obg_train_frame(ctypes.byref(g.c()), _ptr(rgb), n_frames, _ptr(occ),
                                  _ptr(counts), _stream(stream)))


def obg_merge(g: FrameGeom, occ_ring: torch.Tensor, ring_len: int, first: int, n_trees: int,
              thr_num: int, thr_den: int, leafset: torch.Tensor, stream=None):
    _need(occ_ring, torch.int32, ring_len * g.n_regions * g.words, "occ_ring")
    _need(leafset, torch.int32, g.n_regions * g.words, "leafset")
    _check(load().obg_merge(ctypes.byref(g.c()), _ptr(occ_ring), ring_len, first, n_trees,
                            thr_num, thr_den, _ptr(leafset), _stream(stream)))


def obg_merge_groups(g: FrameGeom, occ_ring: torch.Tensor, ring_len: int, first: int, n_trees: int, group: int,
                     thr_num: int, thr_den: int, leafset: torch.Tensor, stream=None):
    _need(occ_ring, torch.int32, ring_len * g.n_regions * g.words, "occ_ring")
    _need(leafset, torch.int32, g.n_regions * g.words, "leafset")
    _check(load().obg_merge_groups(ctypes.byref(g.c()), _ptr(occ_ring), ring_len, first, n_trees, group,
                                   thr_num, thr_den, _ptr(leafset), _stream(stream)))


def obg_classify(g: FrameGeom, rgb: torch.Tensor, n_frames: int, leafset: torch.Tensor,
                 mask: torch.Tensor, occ_out: Optional[torch.Tensor] = None, stream=None):
    _frames_ok(g, rgb, n_frames)
    _need(leafset, torch.int32, g.n_regions * g.words, "leafset")
    _need(mask, torch.int64, n_frames * g.height * g.mask_row_words, "mask")
    if occ_out is not None:
        _need(occ_out, torch.int32, n_frames * g.n_regions * g.words, "occ_out")
    _check(load().obg_classify(ctypes.byref(g.c()), _ptr(rgb), n_frames, _ptr(leafset),
                               _ptr(mask), _ptr(occ_out), _stream(stream)))


def obg_quantize(g: FrameGeom, rgb: torch.Tensor, n_frames: int, out: torch.Tensor, stream=None):
    _frames_ok(g, rgb, n_frames)
    _frames_ok(g, out, n_frames)
    _check(load().obg_quantize(ctypes.byref(g.c()), _ptr(rgb), n_frames, _ptr(out), _stream(stream)))


def obg_score(g: FrameGeom, mask: torch.Tensor, truth: torch.Tensor, n_frames: int, counts: torch.Tensor,
              stream=None):
    """counts: int64 GPU tensor of 3 (true positives, false positives, false negatives)."""
    _need(mask, torch.int64, n_frames * g.height * g.mask_row_words, "mask")
    _need(truth, torch.int64, n_frames * g.height * g.mask_row_words, "truth")
    _need(counts, torch.int64, 3, "counts")
    _check(load().obg_score(ctypes.byref(g.c()), _ptr(mask), _ptr(truth), n_frames, _ptr(counts), _stream(stream)))


TUNE_KEYS = {"train_block": 0, "occ_blind": 1, "occ_wg_per_cu": 2,
             "classify_wg_per_cu": 3, "classify_span": 4, "classify_block": 5, "layout": 6, "interleave": 7, "mask_stage": 8,
             "region_chunks": 9, "batch_per_depth": 10, "batch_graph": 11, "fused_span": 12}


def obg_tune_set(key, value: int):
    k = TUNE_KEYS[key] if isinstance(key, str) else key
    _check(load().obg_tune_set(k, value))


def obg_tune_get(key) -> int:
    k = TUNE_KEYS[key] if isinstance(key, str) else key
    return load().obg_tune_get(k)


PROBE_READ, PROBE_READ_WRITE, PROBE_COPY = 1, 2, 3


def obg_probe(kind: int, src: torch.Tensor, dst: Optional[torch.Tensor], nbytes: int,
              sink: Optional[torch.Tensor], grid: int = 512, stream=None):
    _need(src, torch.uint8, nbytes, "src")
    if dst is not None:
        _need(dst, torch.uint8, 0, "dst")
        need = nbytes if kind == PROBE_COPY else nbytes // 24
        if dst.numel() < need:
            raise ValueError(f"dst holds {dst.numel()} bytes, needs {need}")
    if sink is not None:
        _need(sink, torch.int32, grid * 512, "sink")
    rc = load().obg_probe(kind, _ptr(src), _ptr(dst), nbytes, _ptr(sink), grid, _stream(stream))
    if rc != OBG_OK:
        raise ObgError(rc, "probe arguments rejected")


class ProbeShape(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("grid", ctypes.c_int32), ("block", ctypes.c_int32),
                ("inflight", ctypes.c_int32), ("span", ctypes.c_int32), ("phase_items", ctypes.c_int32)]


def obg_probe_shaped(kind: int, src: torch.Tensor, dst: Optional[torch.Tensor], nbytes: int,
                     sink: torch.Tensor, grid: int, block: int, inflight: int, span: int,
                     phase_items: int = 0, stream=None):
    """The READ / READ_WRITE probe with its launch shape given (see obg.h)."""
    _need(src, torch.uint8, nbytes, "src")
    if dst is not None:
        _need(dst, torch.uint8, nbytes // 24, "dst")
    _need(sink, torch.int32, grid * block + 1, "sink")
    sh = ProbeShape(kind, grid, block, inflight, span, phase_items)
    _check(load().obg_probe_shaped(ctypes.byref(sh), _ptr(src), _ptr(dst), nbytes, _ptr(sink), _stream(stream)))


class Plan:
    """Owner of an obg_plan handle."""

    def __init__(self, handle, n_streams):
        self.h = handle
        self.n_streams = n_streams

    def run(self, items: torch.Tensor, n_items: Optional[int] = None, stream=None):
        """obg_batch_run on a device array of work items (see work_items)."""
        n = _n_items(items, n_items)
        _check(load().obg_batch_run(self.h, _ptr(items), n, _stream(stream)))

    def tune(self, items: torch.Tensor, n_items: Optional[int] = None, stream=None):
        """obg_plan_tune: time the launch shapes on this work and keep the fastest."""
        n = _n_items(items, n_items)
        _check(load().obg_plan_tune(self.h, _ptr(items), n, _stream(stream)))

    def info(self) -> dict:
        pi = PlanInfo()
        _check(load().obg_plan_info_get(self.h, ctypes.byref(pi)))
        return {name: getattr(pi, name) for name, _ in PlanInfo._fields_}

    def close(self):
        if self.h:
            load().obg_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _n_items(items: torch.Tensor, n_items: Optional[int]) -> int:
    _need(items, torch.uint8, 0, "items")
    have = items.numel() // ctypes.sizeof(WorkItem)
    n = have if n_items is None else n_items
    if n > have:
        raise ValueError(f"items hold {have} work items, {n} requested")
    return n


def _plan_streams(streams):
    arr = (PlanStream * max(1, len(streams)))()
    for i, sd in enumerate(streams):
        num, den = sd["thr"]
        arr[i] = PlanStream(sd["geom"].c(), num, den, sd["max_train"], sd["max_test"])
    return arr


def obg_plan_create(streams) -> Plan:
    """streams: list of dicts with keys geom (FrameGeom), thr (num, den),
    max_train, max_test."""
    h = ctypes.c_void_p()
    _check(load().obg_plan_create(_plan_streams(streams), len(streams), ctypes.byref(h)))
    return Plan(h, len(streams))


NOALLOC_MAX_STREAMS = 256


def obg_batch_run_noalloc(streams, items: torch.Tensor, n_items: Optional[int] = None, stream=None):
    """obg_batch_run_noalloc: the batched run of these stream descriptions
    (as for obg_plan_create) on a device array of work items, with no device
    memory allocated by the library."""
    n = _n_items(items, n_items)
    _check(load().obg_batch_run_noalloc(_plan_streams(streams), len(streams), _ptr(items), n, _stream(stream)))


def work_items(entries, device="cuda") -> torch.Tensor:
    """Pack work items into a device array (uint8 tensor of obg_work_item).
    entries: list of dicts with keys stream, geom (FrameGeom), n_train, n_test
    and the tensors train, test, occ, leafset, mask (None where a count is 0;
    leafset is read when n_train is 0 and n_test > 0).  Sizes are checked
    here; the run checks the rest and writes each item's status."""
    arr = (WorkItem * max(1, len(entries)))()
    for i, e in enumerate(entries):
        g, T, N = e["geom"], e.get("n_train", 0), e.get("n_test", 0)
        if T > 0:
            _frames_ok(g, e["train"], T)
            _need(e["occ"], torch.int32, T * g.words, "occ")
        if T > 0 or N > 0:
            _need(e["leafset"], torch.int32, g.words, "leafset")
        if N > 0:
            _frames_ok(g, e["test"], N)
            _need(e["mask"], torch.int64, N * g.height * g.mask_row_words, "mask")
        arr[i] = WorkItem(e["stream"], T, N, -1,
                          e["train"].data_ptr() if T > 0 else None, e["test"].data_ptr() if N > 0 else None,
                          e["occ"].data_ptr() if T > 0 else None,
                          e["leafset"].data_ptr() if (T > 0 or N > 0) else None,
                          e["mask"].data_ptr() if N > 0 else None)
    raw = bytes(memoryview(arr).cast("B"))[: len(entries) * ctypes.sizeof(WorkItem)]
    return torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device) if raw else \
        torch.zeros(0, dtype=torch.uint8, device=device)


def item_status(items: torch.Tensor) -> list:
    """Status of every work item of a finished run (OBG_ITEM_*)."""
    host = items.cpu().numpy().tobytes()
    n = len(host) // ctypes.sizeof(WorkItem)
    arr = (WorkItem * max(1, n)).from_buffer_copy(host + bytes(ctypes.sizeof(WorkItem) * (1 - min(1, n))))
    return [arr[i].status for i in range(n)]


def _serve_streams(streams):
    n = len(streams)
    arr = (ServeStream * n)()
    for i, s in enumerate(streams):
        arr[i] = ServeStream(s["width"], s["height"], s["depth"], s["n_train"], s["thr"][0], s["thr"][1],
                             s.get("region_w", 0), s.get("region_h", 0))
    return arr


def obg_serve_state_bytes(streams, remerge_window: int = 50) -> int:
    """Bytes of a serving checkpoint of these streams (-1: invalid)."""
    return load().obg_serve_state_bytes(_serve_streams(streams), len(streams), remerge_window)


def obg_serve_run(streams, arrivals, ingest_fn: int, ingest_ctx: int, speed: float = 1.0,
                  budget_bytes: int = 32 << 30, max_inflight: int = 3, max_batch_frames: int = 256,
                  remerge_period: int = 100, remerge_window: int = 50, checksums=None,
                  watch=None, watch_masks=None, watch_max_frames: int = 0,
                  state_in=None, state_out=None) -> dict:
    """streams: list of dicts (width, height, depth, n_train, thr=(num, den));
    arrivals: list of float64 numpy arrays (seconds); checksums: optional uint64
    numpy array [n_streams, stride]; watch: stream indices whose masks are
    copied into watch_masks (uint64 numpy arrays [frames, H, ceil(W/64)]);
    state_in / state_out: optional uint8 numpy arrays of obg_serve_state_bytes
    bytes (restore a checkpoint before the run / write one after it)."""
    import numpy as np
    n = len(streams)
    arr = _serve_streams(streams)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in arrivals]
    ptrs = (ctypes.POINTER(ctypes.c_double) * n)(*[a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrs])
    counts = (ctypes.c_int32 * n)(*[len(a) for a in arrs])
    cfg = ServeConfig()
    cfg.streams = arr
    cfg.n_streams = n
    cfg.arrivals = ptrs
    cfg.n_arrivals = counts
    cfg.speed = speed
    cfg.budget_bytes = budget_bytes
    cfg.max_inflight = max_inflight
    cfg.max_batch_frames = max_batch_frames
    cfg.remerge_period = remerge_period
    cfg.remerge_window = remerge_window
    cfg.ingest = ingest_fn
    cfg.ingest_ctx = ingest_ctx
    if checksums is not None:
        assert checksums.dtype == np.uint64 and checksums.flags.c_contiguous and checksums.shape[0] == n
        cfg.checksums = checksums.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        cfg.checksum_stride = checksums.shape[1]
    keep = []
    if watch:
        ws = (ctypes.c_int32 * len(watch))(*watch)
        wm = (ctypes.POINTER(ctypes.c_uint64) * len(watch))(
            *[m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)) for m in watch_masks])
        keep += [ws, wm]
        cfg.watch_streams = ws
        cfg.n_watch = len(watch)
        cfg.watch_masks = wm
        cfg.watch_max_frames = watch_max_frames
    need = None
    for name, buf in (("state_in", state_in), ("state_out", state_out)):
        if buf is None:
            continue
        need = need if need is not None else obg_serve_state_bytes(streams, remerge_window)
        assert buf.dtype == np.uint8 and buf.flags.c_contiguous and buf.size >= need > 0, name
        setattr(cfg, name, buf.ctypes.data)
    st = ServeStats()
    _check(load().obg_serve_run(ctypes.byref(cfg), ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in ServeStats._fields_}


def obg_version() -> str:
    return load().obg_version().decode()


# -- convenience allocation helpers (torch owns the memory) ------------------

def empty_occ(g: FrameGeom, n_frames: int, device="cuda") -> torch.Tensor:
    return torch.empty((n_frames, g.n_regions, g.words), dtype=torch.int32, device=device)


def empty_mask(g: FrameGeom, n_frames: int, device="cuda") -> torch.Tensor:
    return torch.empty((n_frames, g.height, g.mask_row_words), dtype=torch.int64, device=device)


def empty_leafset(g: FrameGeom, device="cuda") -> torch.Tensor:
    return torch.empty((g.n_regions, g.words), dtype=torch.int32, device=device)
