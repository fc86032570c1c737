"""The C-ABI library loads, exports what include/obg.h declares, and rejects
bad arguments before touching the GPU (no kernel is launched here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "obg.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1412_1945_amd import obg
    if not os.path.exists(obg.LIB_PATH):
        from paper_1412_1945_amd import build
        build.build()
    return obg


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(obg_[a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ["obg_train_frame", "obg_merge", "obg_classify", "obg_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    L = ctypes.CDLL(lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) == set(lib.exported_symbols())


def test_sizes(lib):
    g = lib.FrameGeom(160, 120, 4)
    assert lib.obg_num_regions(g) == 1
    assert lib.obg_occ_words(g) == 128
    assert lib.obg_mask_words(g) == 120 * 3
    g = lib.FrameGeom(3840, 2160, 4, region_w=32, region_h=32)
    assert lib.obg_num_regions(g) == 120 * 68
    assert lib.obg_occ_words(g) == 120 * 68 * 128
    g = lib.FrameGeom(10, 10, 1)
    assert lib.obg_occ_words(g) == 1
    g = lib.FrameGeom(10, 10, 8)
    assert lib.obg_occ_words(g) == (1 << 24) // 32
    bad = lib.FrameGeom(10, 10, 9)
    assert lib.obg_num_regions(bad) == -1


def _raw(lib):
    return lib.load()


def _geom(lib, **kw):
    base = dict(width=64, height=8, row_pitch=192, frame_pitch=192 * 8, depth=4, region_w=0, region_h=0)
    base.update(kw)
    return lib.Geom(**base)


FAKE = ctypes.c_void_p(0x100000)   # never dereferenced: every case fails validation first
# the serving loop's ingest callback: int (*)(void *ctx, const obg_ingest_item *, int32_t, hipStream_t)
INGEST_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p)


@pytest.mark.parametrize("kw,code", [
    (dict(depth=0), -1), (dict(depth=9), -1), (dict(width=0), -1), (dict(height=0), -1),
    (dict(row_pitch=176), -1), (dict(frame_pitch=100), -1),
    (dict(row_pitch=200, frame_pitch=1600), -2), (dict(frame_pitch=192 * 8 + 8), -2),
    (dict(region_w=16, region_h=0), -1), (dict(region_w=-1, region_h=4), -1),
])
def test_train_rejects_bad_geometry(lib, kw, code):
    L = _raw(lib)
    g = _geom(lib, **kw)
    rc = L.obg_train_frame(ctypes.byref(g), FAKE, 1, FAKE, None, None)
    assert rc == code, L.obg_last_error()
    assert L.obg_last_error()


def test_train_rejects_null_and_unaligned(lib):
    L = _raw(lib)
    g = _geom(lib)
    assert L.obg_train_frame(ctypes.byref(g), None, 1, FAKE, None, None) == -1
    assert L.obg_train_frame(ctypes.byref(g), FAKE, 1, None, None, None) == -1
    assert L.obg_train_frame(ctypes.byref(g), ctypes.c_void_p(0x100004), 1, FAKE, None, None) == -2
    assert L.obg_train_frame(ctypes.byref(g), FAKE, -1, FAKE, None, None) == -1
    assert L.obg_train_frame(None, FAKE, 1, FAKE, None, None) == -1
    # zero frames: nothing to do, nothing enqueued
    assert L.obg_train_frame(ctypes.byref(g), None, 0, None, None, None) == 0


@pytest.mark.parametrize("args,code", [
    ((4, 0, 0, 1, 2), -1),       # n_trees < 1
    ((4, 0, 5, 1, 2), -1),       # n_trees > ring_len
    ((4, 4, 2, 1, 2), -1),       # first outside the ring
    ((4, -1, 2, 1, 2), -1),
    ((4, 0, 2, 0, 2), -1),       # zero threshold
    ((4, 0, 2, 1, 0), -1),       # zero denominator
    ((70000, 0, 70000, 1, 2), -1),  # too many trees for the counters
])
def test_merge_rejects_bad_window(lib, args, code):
    L = _raw(lib)
    g = _geom(lib)
    ring, first, n, num, den = args
    rc = L.obg_merge(ctypes.byref(g), FAKE, ring, first, n, num, den, FAKE, None)
    assert rc == code, L.obg_last_error()


def test_merge_groups_rejects_bad_group(lib):
    L = _raw(lib)
    g = _geom(lib)
    assert L.obg_merge_groups(ctypes.byref(g), FAKE, 4, 0, 4, 0, 1, 2, FAKE, None) == -1
    assert L.obg_merge_groups(ctypes.byref(g), FAKE, 4, 0, 4, -2, 1, 2, FAKE, None) == -1
    assert L.obg_merge_groups(ctypes.byref(g), FAKE, 4, 0, 5, 2, 1, 2, FAKE, None) == -1   # window > ring
    assert L.obg_merge_groups(ctypes.byref(g), FAKE, 4, 0, 4, 2, 0, 2, FAKE, None) == -1


def test_quantize_rejects_bad_buffers(lib):
    L = _raw(lib)
    g = _geom(lib)
    assert L.obg_quantize(ctypes.byref(g), None, 1, FAKE, None) == -1
    assert L.obg_quantize(ctypes.byref(g), FAKE, 1, None, None) == -1
    assert L.obg_quantize(ctypes.byref(g), FAKE, 1, ctypes.c_void_p(0x100008), None) == -2
    # overlapping but not identical
    assert L.obg_quantize(ctypes.byref(g), FAKE, 2, ctypes.c_void_p(0x100000 + 1536), None) == -1
    assert L.obg_quantize(ctypes.byref(g), None, 0, None, None) == 0


def test_score_rejects_bad_buffers(lib):
    L = _raw(lib)
    g = _geom(lib)
    assert L.obg_score(ctypes.byref(g), FAKE, FAKE, 1, None, None) == -1
    assert L.obg_score(ctypes.byref(g), None, FAKE, 1, FAKE, None) == -1
    assert L.obg_score(ctypes.byref(g), FAKE, ctypes.c_void_p(0x100004), 1, FAKE, None) == -2
    assert L.obg_score(ctypes.byref(g), FAKE, FAKE, -1, FAKE, None) == -1


def test_classify_rejects_null(lib):
    L = _raw(lib)
    g = _geom(lib)
    assert L.obg_classify(ctypes.byref(g), FAKE, 1, None, FAKE, None, None) == -1
    assert L.obg_classify(ctypes.byref(g), FAKE, 1, FAKE, None, None, None) == -1
    assert L.obg_classify(ctypes.byref(g), None, 0, None, None, None, None) == 0


def test_binding_refuses_cpu_tensors(lib):
    import torch
    g = lib.FrameGeom(16, 4, 3)
    with pytest.raises(ValueError):
        lib.obg_train_frame(g, torch.zeros(16 * 4 * 3, dtype=torch.uint8), 1,
                            torch.zeros(16, dtype=torch.int32))


def test_plan_rejects_bad_streams(lib):
    import ctypes as C
    L = _raw(lib)
    g = _geom(lib)
    good = dict(geom=g, thr_num=1, thr_den=2, max_train=4, max_test=2)
    out = C.c_void_p()
    for bad, code in [(dict(max_train=-1), -1), (dict(max_train=70000), -1), (dict(max_test=-1), -1),
                      (dict(thr_num=0), -1), (dict(thr_den=0), -1),
                      (dict(geom=_geom(lib, depth=7)), -1), (dict(geom=_geom(lib, region_w=16, region_h=16)), -1),
                      (dict(geom=_geom(lib, row_pitch=200, frame_pitch=1600)), -2)]:
        d = dict(good)
        d.update(bad)
        arr = (lib.PlanStream * 1)(lib.PlanStream(**d))
        assert L.obg_plan_create(arr, 1, C.byref(out)) == code, (bad, L.obg_last_error())
        assert not out.value
    assert L.obg_plan_create(None, 0, C.byref(out)) == -1
    arr = (lib.PlanStream * 1)(lib.PlanStream(**good))
    assert L.obg_plan_create(arr, 0, C.byref(out)) == -1
    assert L.obg_plan_create(arr, 8193, C.byref(out)) == -1
    assert L.obg_plan_create(arr, 1, None) == -1
    # a run on no plan, or with more items than the plan has streams
    assert L.obg_batch_run(None, FAKE, 1, None) == -1
    assert L.obg_plan_tune(None, FAKE, 1, None) == -1
    L.obg_plan_destroy(None)


def test_noalloc_run_rejects_before_touching_the_device(lib):
    """The no-allocation batched run validates like a plan and its run, and
    its stream limit is the header's."""
    import ctypes as C
    L = _raw(lib)
    src = open(HEADER).read()
    assert int(re.search(r"#define OBG_NOALLOC_MAX_STREAMS\s+(\d+)", src).group(1)) == lib.NOALLOC_MAX_STREAMS
    good = dict(geom=_geom(lib), thr_num=1, thr_den=2, max_train=4, max_test=2)
    for bad, code in [(dict(max_train=-1), -1), (dict(thr_num=0), -1), (dict(geom=_geom(lib, depth=7)), -1),
                      (dict(geom=_geom(lib, region_w=16, region_h=16)), -1),
                      (dict(geom=_geom(lib, row_pitch=200, frame_pitch=1600)), -2)]:
        d = dict(good)
        d.update(bad)
        arr = (lib.PlanStream * 1)(lib.PlanStream(**d))
        assert L.obg_batch_run_noalloc(arr, 1, FAKE, 1, None) == code, (bad, L.obg_last_error())
    n = lib.NOALLOC_MAX_STREAMS + 1
    arr = (lib.PlanStream * n)(*[lib.PlanStream(**good)] * n)
    assert L.obg_batch_run_noalloc(arr, n, FAKE, 1, None) == -1
    assert b"without allocation" in L.obg_last_error()
    assert L.obg_batch_run_noalloc(None, 1, FAKE, 1, None) == -1
    assert L.obg_batch_run_noalloc(arr, 0, FAKE, 1, None) == -1
    assert L.obg_batch_run_noalloc(arr, 2, FAKE, 3, None) == -1          # more items than streams
    assert L.obg_batch_run_noalloc(arr, 2, None, 1, None) == -1          # items NULL
    assert L.obg_batch_run_noalloc(arr, 2, C.c_void_p(0x100004), 1, None) == -2   # misaligned items
    assert L.obg_batch_run_noalloc(arr, 2, FAKE, 0, None) == 0           # nothing to do


def test_shaped_probe_rejects_bad_shapes(lib):
    """The shaped probe refuses shapes outside its documented ranges before it
    touches the device."""
    import ctypes as C
    L = _raw(lib)
    good = dict(kind=lib.PROBE_READ_WRITE, grid=512, block=512, inflight=2, span=832, phase_items=0)
    for bad in [dict(kind=3), dict(grid=0), dict(grid=65537), dict(block=128), dict(inflight=3), dict(span=2),
                dict(span=4098), dict(span=830), dict(phase_items=-1), dict(phase_items=40),
                dict(kind=lib.PROBE_READ, phase_items=4)]:
        d = dict(good)
        d.update(bad)
        sh = lib.ProbeShape(**d)
        assert L.obg_probe_shaped(C.byref(sh), FAKE, FAKE, 1 << 30, FAKE, None) == -1, bad
    sh = lib.ProbeShape(**good)
    assert L.obg_probe_shaped(C.byref(sh), FAKE, None, 1 << 30, FAKE, None) == -1     # no dst for writes
    assert L.obg_probe_shaped(C.byref(sh), FAKE, FAKE, 100, FAKE, None) == -1         # less than one item
    assert L.obg_probe_shaped(None, FAKE, FAKE, 1 << 30, FAKE, None) == -1


def test_abi_struct_layouts(lib, tmp_path):
    """Sizes and field offsets of the C structs of include/obg.h, as a C
    compiler lays them out, equal those of the ctypes binding."""
    import ctypes as C
    structs = {"obg_geom": lib.Geom, "obg_plan_stream": lib.PlanStream, "obg_work_item": lib.WorkItem,
               "obg_plan_info": lib.PlanInfo, "obg_serve_stream": lib.ServeStream,
               "obg_serve_config": lib.ServeConfig, "obg_serve_stats": lib.ServeStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "obg.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True, capture_output=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, f"{cname}.{f}"


def test_serve_checkpoint_size_and_refusal(lib):
    """The checkpoint size follows its stated layout, and a state that is not
    a checkpoint of the streams is refused before any device work."""
    import numpy as np
    streams = [dict(width=64, height=32, depth=3, n_train=5, thr=(1, 2)),
               dict(width=96, height=64, depth=4, n_train=6, thr=(1, 2), region_w=32, region_h=32)]
    pad8 = lambda b: (b + 7) // 8 * 8
    want = 16 + 2 * 48
    for tree, ring_len in [(64, 10), (512 * 6, 10)]:
        want += pad8(tree) + pad8(ring_len * tree)
    assert lib.obg_serve_state_bytes(streams, 10) == want
    assert lib.obg_serve_state_bytes([dict(streams[0], depth=7)], 10) == -1
    assert lib.obg_serve_state_bytes(streams, 0) == -1
    arrivals = [np.array([0.0, 0.1, 0.2]), np.array([0.0, 0.1])]
    bad = np.zeros(want, dtype=np.uint8)
    calls = []

    @INGEST_FN
    def ingest(ctx, items, n, stream):
        calls.append(n)
        return 0

    cb = ctypes.cast(ingest, ctypes.c_void_p).value
    with pytest.raises(lib.ObgError) as e:
        # the state is checked before any device work
        lib.obg_serve_run(streams, arrivals, cb, 0, remerge_period=10, remerge_window=10, state_in=bad)
    assert e.value.code == -1
    with pytest.raises(lib.ObgError) as e:
        lib.obg_serve_run(streams, [np.array([0.0, float("nan"), 0.2]), arrivals[1]], cb, 0,
                          remerge_period=10, remerge_window=10)
    assert e.value.code == -1 and "finite" in str(e.value)
    assert calls == []


def test_tune_keys_match_header_and_refuse_bad_values(lib):
    """Every launch knob the header defines has the same number in the
    binding; values round-trip; unknown keys and negative values are refused."""
    src = open(HEADER).read()
    defs = {m.group(1).lower(): int(m.group(2))
            for m in re.finditer(r"#define OBG_TUNE_([A-Z_]+)\s+(\d+)", src)}
    count = defs.pop("count")
    assert lib.TUNE_KEYS == defs
    assert sorted(defs.values()) == list(range(count))
    L = lib.load()
    for key, k in defs.items():
        assert L.obg_tune_get(k) == 0, key
        assert L.obg_tune_set(k, 2) == 0, key
        assert lib.obg_tune_get(key) == 2, key
        lib.obg_tune_set(key, 0)
        assert L.obg_tune_get(k) == 0, key
    assert L.obg_tune_set(count, 1) != 0
    assert L.obg_tune_set(-1, 1) != 0
    assert L.obg_tune_get(count) == -1
    assert L.obg_tune_set(0, -1) != 0
    assert L.obg_tune_get(0) == 0
