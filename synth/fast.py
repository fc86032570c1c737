"""GPU evaluation of the synthetic streams of frames.py (same bytes, faster).

frames.py stays the definition; this module packs its per-frame numbers
(frame hash, drift scale, object positions) and hands them to the HIP kernel
in gen.hip, which evaluates the per-pixel formula on the GPU.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence

import torch

from . import frames as F

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gen.hip")
LIB = os.path.join(HERE, "libsynth.so")
FRAME_INTS = 4 + 8 * 6


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", tmp, SRC],
                   check=True, capture_output=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None
_ntab = {}


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is not built")
        lib = ctypes.CDLL(LIB)
        I32, I64, U32, P = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p
        lib.synth_generate.restype = ctypes.c_int
        lib.synth_generate.argtypes = [I32, I32, I64, I64, U32, U32, U32, I32, I32, I32, I32, U32, U32, U32,
                                       P, I32, P, P, P]
        _lib = lib
    return _lib


def frame_records(spec: F.StreamSpec, frames: Sequence[int]) -> torch.Tensor:
    sk = F._stream_key(spec)
    rows = []
    for f in frames:
        hf = F.fmix32(sk ^ F.fmix32((f + F._P_FRAME) & F.M32))
        row = [f, hf, F.drift_scale_q16(spec, f), 0]
        if f >= spec.n_train:
            for o, (px, py) in zip(spec.objects, F.object_positions(spec, f)):
                row += [0 if o.kind == "rect" else 1, px, py, o.a, o.b, *o.colour]
            row[3] = len(spec.objects)
        rows.append(row + [0] * (FRAME_INTS - len(row)))
    recs = torch.tensor(rows, dtype=torch.int64).reshape(len(rows), FRAME_INTS)
    # the frame hash is an unsigned 32-bit value: keep its bits in int32
    recs = torch.where(recs >= 2 ** 31, recs - 2 ** 32, recs)
    return recs.to(torch.int32)


def make_frames_gpu(spec: F.StreamSpec, frames: Sequence[int], out: torch.Tensor, stream=None) -> torch.Tensor:
    """Write the frames into `out` (uint8 [len(frames), H, row_pitch] on the GPU)."""
    frames = list(frames)
    assert out.is_cuda and out.dtype == torch.uint8 and out.is_contiguous()
    assert out.numel() >= len(frames) * spec.height * spec.row_pitch
    dev = out.device
    key = (float(spec.noise_sigma), dev)
    if key not in _ntab:
        _ntab[key] = torch.tensor(F.noise_table(spec.noise_sigma), dtype=torch.int16, device=dev)
    sk = F._stream_key(spec)
    kp = F.fmix32(sk ^ F._P_PALETTE)
    kb = F.fmix32(sk ^ F._P_BIMODAL)
    bthr = int(spec.bimodal_frac * 4294967296.0)
    t0, t1, t2 = F.PICK_THRESHOLDS
    s = torch.cuda.current_stream(dev) if stream is None else stream
    lib = _load()
    for c0 in range(0, len(frames), 1024):
        chunk = frames[c0: c0 + 1024]
        recs = frame_records(spec, chunk).to(dev)
        dst = out.view(-1)[c0 * spec.height * spec.row_pitch:]
        rc = lib.synth_generate(spec.width, spec.height, spec.row_pitch, spec.height * spec.row_pitch,
                                kp, kb, min(bthr, 0xFFFFFFFF), 1 if spec.bimodal_frac > 0 else 0,
                                spec.bimodal_period, spec.block, spec.n_palette, t0, t1, t2,
                                ctypes.c_void_p(recs.data_ptr()), len(chunk),
                                ctypes.c_void_p(_ntab[key].data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                ctypes.c_void_p(s.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"synth_generate failed ({rc})")
        # recs must outlive the kernel: wait before the next chunk reuses memory
        s.synchronize()
    return out


def poisson_arrivals(rates, duration_s: float, seed: int):
    """Per stream: increasing arrival times (seconds) of a Poisson process."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for lam in rates:
        n_max = int(lam * duration_s * 1.5 + 50)
        gaps = rng.exponential(1.0 / lam, size=n_max)
        t = np.cumsum(gaps)
        while t[-1] < duration_s:
            t = np.concatenate([t, t[-1] + np.cumsum(rng.exponential(1.0 / lam, size=n_max))])
        out.append(np.ascontiguousarray(t[t < duration_s], dtype=np.float64))
    return out


class IngestContext:
    """Frame source of a serving run: frame f of stream s is frame f of the
    stream's synthetic sequence, written on the GPU when the server asks."""

    def __init__(self, specs, n_frames, slots: int, device="cuda"):
        lib = _load()
        P = ctypes.c_void_p
        lib.synth_ingest_create.restype = ctypes.c_void_p
        lib.synth_ingest_create.argtypes = [ctypes.c_int32, P, P, P, P, P, ctypes.c_int32]
        lib.synth_ingest_destroy.restype = None
        lib.synth_ingest_destroy.argtypes = [P]
        self.lib = lib
        params, recs, base, counts = [], [], [], []
        total = 0
        for spec, n in zip(specs, n_frames):
            sk = F._stream_key(spec)
            params += [spec.width, spec.height, spec.row_pitch, F.fmix32(sk ^ F._P_PALETTE),
                       F.fmix32(sk ^ F._P_BIMODAL), min(int(spec.bimodal_frac * 4294967296.0), 0xFFFFFFFF),
                       1 if spec.bimodal_frac > 0 else 0, spec.bimodal_period, spec.block, spec.n_palette, 0, 0]
            recs.append(frame_records(spec, range(max(n, 1))))
            base.append(total)
            counts.append(n)
            total += max(n, 1)
        p64 = torch.tensor(params, dtype=torch.int64)
        self.params = torch.where(p64 >= 2 ** 31, p64 - 2 ** 32, p64).to(torch.int32).contiguous()
        self.recs = torch.cat(recs).to(device).contiguous()
        self.base = torch.tensor(base, dtype=torch.int64).contiguous()
        self.counts = torch.tensor(counts, dtype=torch.int32).contiguous()
        sigma = specs[0].noise_sigma
        assert all(s.noise_sigma == sigma for s in specs)
        self.ntab = torch.tensor(F.noise_table(sigma), dtype=torch.int16, device=device)
        self.ctx = lib.synth_ingest_create(len(specs), self.params.data_ptr(), self.recs.data_ptr(),
                                           self.base.data_ptr(), self.counts.data_ptr(), self.ntab.data_ptr(),
                                           slots)
        if not self.ctx:
            raise RuntimeError("synth_ingest_create failed")
        self.fn = ctypes.cast(lib.synth_ingest, ctypes.c_void_p).value

    def close(self):
        if self.ctx:
            self.lib.synth_ingest_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
