"""The GPU evaluation of the synthetic streams gives the same bytes as frames.py."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fast():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from synth import fast
    return fast


def test_fast_generator_matches_definition(fast):
    from synth import frames as F
    specs = [F.cfg0().streams[0], F.cfg1(n_test=3).streams[0]]
    specs += F.mixed_streams(6, seed=9, n_test=4)[0]
    specs.append(F.StreamSpec(100, 37, 2, 3, seed=4, fg="ellipses", fg_coverage=0.2, drift_amp=0.3, bimodal_frac=0.5))
    # widths that end in a partial 16-pixel group, and narrower than one group
    for W, H in [(33, 17), (7, 5), (16, 3), (47, 2), (1, 1)]:
        specs.append(F.StreamSpec(W, H, 2, 3, seed=6, fg="ellipses", fg_coverage=0.3, drift_amp=0.2,
                                  bimodal_frac=0.3, block=5))
    specs.append(F.StreamSpec(70, 20, 2, 3, seed=7, fg="rect", rect_size=9))
    for spec in specs:
        ids = [0, 1, spec.n_train, spec.n_frames - 1]
        print(f"[case] {spec.width}x{spec.height} frames {ids}", flush=True)
        want = F.make_frames(spec, ids, device="cuda")
        got = torch.zeros_like(want)
        fast.make_frames_gpu(spec, ids, got)
        torch.cuda.synchronize()
        W = spec.width
        assert torch.equal(got[:, :, : 3 * W], want[:, :, : 3 * W]), (spec.width, spec.height)


def test_ingest_matches_definition(fast):
    """The serving source (per-stream tables, many streams per launch) writes
    the same bytes as the definition."""
    import ctypes
    from synth import frames as F
    specs = F.mixed_streams(5, seed=12, n_test=4)[0]
    specs += [F.StreamSpec(33, 17, 3, 4, seed=8, stream=5, fg="ellipses", fg_coverage=0.3, drift_amp=0.2,
                           bimodal_frac=0.4, block=5),
              F.StreamSpec(70, 20, 2, 3, seed=8, stream=6, fg="rect", rect_size=9)]
    ctx = fast.IngestContext(specs, [s.n_frames for s in specs], slots=2)

    class Item(ctypes.Structure):
        _fields_ = [("stream", ctypes.c_int32), ("frame", ctypes.c_int32), ("dst", ctypes.c_void_p)]

    lib = fast._load()
    lib.synth_ingest.restype = ctypes.c_int
    lib.synth_ingest.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
    # a small batch (one job per workgroup row) and a large one (equal runs of
    # groups with the noise table in LDS) take different kernels
    for first, rounds in ((3, 1), (0, 3)):
        jobs, bufs = [], []
        for s, spec in enumerate(specs):
            if s < first:
                continue
            for k in range(rounds):
                for f in sorted({0, spec.n_train - 1, spec.n_train, spec.n_frames - 1}):
                    buf = torch.zeros((spec.height, spec.row_pitch), dtype=torch.uint8, device="cuda")
                    bufs.append((s, f, buf))
                    jobs.append(Item(s, f, buf.data_ptr()))
        arr = (Item * len(jobs))(*jobs)
        px = sum(specs[s].width * specs[s].height for s, _, _ in bufs)
        print(f"[case] ingest {len(jobs)} frames of {len(specs)} streams, {px / 1e6:.1f} Mpx", flush=True)
        rc = lib.synth_ingest(ctx.ctx, ctypes.cast(arr, ctypes.c_void_p), len(jobs),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == 0
        torch.cuda.synchronize()
        for s, f, buf in bufs:
            spec = specs[s]
            want = F.make_frames(spec, [f], device="cuda")[0]
            W = spec.width
            assert torch.equal(buf[:, : 3 * W], want[:, : 3 * W]), (rounds, s, f, spec.width, spec.height)
    ctx.close()
