"""Seeded synthetic camera streams (inputs only; none of the method's arithmetic).

The paper evaluates on recorded surveillance sequences with swaying leaves and
lighting change (Sec. 1 and Sec. 5).  Those recordings are not available here,
so every input is drawn from this module instead.  The same Python code runs on
the CPU and on the GPU: every per-pixel step is an integer torch operation on
int64 values that never overflow, so a frame generated on either device is
byte-identical.  Everything that needs floating point (drift scale, object
positions, the noise table) is computed once per frame on the host in Python
and enters the per-pixel code as an integer.

Per-pixel randomness comes from a counter-based hash: the 32-bit finaliser of
MurmurHash3 (Appleby, "fmix32"), applied to (seed, stream, frame, pixel).
There is no sequential random state, so any frame or pixel can be produced on
its own.

Frame layout: uint8 tensor [n_frames, height, row_pitch], pixel x of row y at
bytes 3x..3x+2 (R, G, B); row_pitch = 3*width rounded up to 16 bytes, padding
bytes zero.
"""
from __future__ import annotations

import math
import random
import statistics
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import torch

M32 = 0xFFFFFFFF


def _mul32(x, c: int):
    """(x * c) mod 2^32 for 0 <= x < 2^32, without leaving int64 range."""
    lo = c & 0xFFFF
    hi = c >> 16
    return (x * lo + ((x * hi) & 0xFFFF) * 65536) & M32


def fmix32(h):
    """MurmurHash3 32-bit finaliser; works on Python ints and int64 tensors."""
    h = h ^ (h >> 16)
    h = _mul32(h, 0x85EBCA6B)
    h = h ^ (h >> 13)
    h = _mul32(h, 0xC2B2AE35)
    h = h ^ (h >> 16)
    return h


# purpose constants that separate the independent hash streams
_P_STREAM = 0x9E3779B9
_P_PALETTE = 0x1B56C4E9
_P_FRAME = 0x7F4A7C15
_P_BIMODAL = 0x2545F491
_P_NOISE_A = 0x68E31DA4
_P_NOISE_B = 0xB5297A4D

# palette pick thresholds on a 16-bit draw: P = 0.7 / 0.2 / 0.07 / 0.03
PICK_THRESHOLDS = (45875, 58982, 63570)


def row_pitch_for(width: int, align: int = 16) -> int:
    return ((3 * width + align - 1) // align) * align


_NOISE_CACHE = {}


def noise_table(sigma: float) -> List[int]:
    """Inverse-normal table: entry u = round(sigma * Phi^-1((u + 0.5) / 65536))."""
    key = float(sigma)
    if key not in _NOISE_CACHE:
        nd = statistics.NormalDist(0.0, 1.0)
        tab = [int(round(sigma * nd.inv_cdf((u + 0.5) / 65536.0))) for u in range(65536)]
        _NOISE_CACHE[key] = tab
    return _NOISE_CACHE[key]


@dataclass
class FgObject:
    kind: str              # "rect" or "ellipse"
    a: int                 # half-width (ellipse semi-axis x) or rect width
    b: int                 # half-height (ellipse semi-axis y) or rect height
    colour: tuple          # (R, G, B)
    x0: float
    y0: float
    vx: float
    vy: float


@dataclass
class StreamSpec:
    """One synthetic camera stream.

    Frames 0..n_train-1 are training frames (background only); frames
    n_train..n_train+n_test-1 are test frames and carry the foreground objects.
    """
    width: int
    height: int
    n_train: int
    n_test: int
    seed: int = 0
    stream: int = 0
    block: int = 8                    # palette block edge in pixels
    n_palette: int = 4
    noise_sigma: float = 4.0
    bimodal_frac: float = 0.0         # fraction of pixels alternating colours 0/1
    bimodal_period: int = 7           # frames; colour 0 on 4 of every 7
    drift_amp: float = 0.0            # relative brightness drift amplitude
    drift_period: int = 300           # frames
    fg: str = "none"                  # "none" | "rect" | "ellipses"
    fg_coverage: float = 0.0          # target fraction of pixels for "ellipses"
    rect_size: int = 20
    rect_speed: int = 3
    objects: List[FgObject] = field(default_factory=list, repr=False)

    @property
    def row_pitch(self) -> int:
        return row_pitch_for(self.width)

    @property
    def n_frames(self) -> int:
        return self.n_train + self.n_test

    @property
    def pixels(self) -> int:
        return self.width * self.height

    def __post_init__(self):
        if not self.objects:
            self.objects = _make_objects(self)


def _stream_key(spec: StreamSpec) -> int:
    return fmix32(fmix32((spec.seed ^ _P_STREAM) & M32) ^ (spec.stream & M32))


def _make_objects(spec: StreamSpec) -> List[FgObject]:
    rng = random.Random(f"fg/{spec.seed}/{spec.stream}")
    W, H = spec.width, spec.height
    objs: List[FgObject] = []
    if spec.fg == "rect":
        s = min(spec.rect_size, W, H)
        col = (rng.randrange(256), rng.randrange(256), rng.randrange(256))
        x0 = rng.uniform(0, max(W - s, 0))
        y0 = rng.uniform(0, max(H - s, 0))
        objs.append(FgObject("rect", s, s, col, x0, y0, float(spec.rect_speed), 0.0))
    elif spec.fg == "ellipses":
        n = rng.randint(1, 6)
        area = spec.fg_coverage * W * H / n
        for _ in range(n):
            ratio = rng.uniform(0.5, 2.0)
            a = max(1, int(round(math.sqrt(area / (math.pi * ratio)))))
            b = max(1, int(round(ratio * a)))
            a = min(a, max(1, W // 2))
            b = min(b, max(1, H // 2))
            col = (rng.randrange(256), rng.randrange(256), rng.randrange(256))
            speed = rng.uniform(1.0, 5.0)
            ang = rng.uniform(0.0, 2.0 * math.pi)
            x0 = rng.uniform(a, max(a, W - 1 - a))
            y0 = rng.uniform(b, max(b, H - 1 - b))
            objs.append(FgObject("ellipse", a, b, col, x0, y0,
                                 speed * math.cos(ang), speed * math.sin(ang)))
    return objs


def _reflect(p: float, lo: float, hi: float) -> float:
    if hi <= lo:
        return lo
    span = hi - lo
    q = (p - lo) % (2.0 * span)
    return lo + (q if q <= span else 2.0 * span - q)


def object_positions(spec: StreamSpec, frame: int):
    """Integer top-left (rect) or centre (ellipse) of every object in a frame.

    Objects move from the first test frame on and bounce off the borders.
    """
    t = frame - spec.n_train
    out = []
    for o in spec.objects:
        if o.kind == "rect":
            x = _reflect(o.x0 + o.vx * t, 0.0, float(spec.width - o.a))
            y = _reflect(o.y0 + o.vy * t, 0.0, float(spec.height - o.b))
        else:
            x = _reflect(o.x0 + o.vx * t, float(o.a), float(spec.width - 1 - o.a))
            y = _reflect(o.y0 + o.vy * t, float(o.b), float(spec.height - 1 - o.b))
        out.append((int(math.floor(x + 0.5)), int(math.floor(y + 0.5))))
    return out


def drift_scale_q16(spec: StreamSpec, frame: int) -> int:
    if spec.drift_amp == 0.0:
        return 65536
    return int(round(65536.0 * (1.0 + spec.drift_amp *
                                math.sin(2.0 * math.pi * frame / spec.drift_period))))


def palette(spec: StreamSpec, device="cpu") -> torch.Tensor:
    """[n_blocks_y, n_blocks_x, n_palette, 3] int64 colours, fixed per stream."""
    nby = (spec.height + spec.block - 1) // spec.block
    nbx = (spec.width + spec.block - 1) // spec.block
    kp = fmix32(_stream_key(spec) ^ _P_PALETTE)
    idx = torch.arange(nby * nbx * spec.n_palette, device=device, dtype=torch.int64)
    h = fmix32(idx ^ kp)
    h = fmix32((h + 0x632BE5AB) & M32)
    rgb = torch.stack([h & 255, (h >> 8) & 255, (h >> 16) & 255], dim=-1)
    return rgb.view(nby, nbx, spec.n_palette, 3)


def _foreground(spec: StreamSpec, frame: int, ys: torch.Tensor, xs: torch.Tensor):
    """(mask bool [H,W], colour int64 [H,W,3]) of the objects in one frame."""
    H, W = spec.height, spec.width
    dev = ys.device
    fgm = torch.zeros((H, W), dtype=torch.bool, device=dev)
    col = torch.zeros((H, W, 3), dtype=torch.int64, device=dev)
    if frame < spec.n_train:
        return fgm, col
    for o, (px, py) in zip(spec.objects, object_positions(spec, frame)):
        if o.kind == "rect":
            m = (xs >= px) & (xs < px + o.a) & (ys >= py) & (ys < py + o.b)
        else:
            dx = (xs - px) * o.b
            dy = (ys - py) * o.a
            m = dx * dx + dy * dy <= (o.a * o.b) ** 2
        fgm = fgm | m
        c = torch.tensor(o.colour, dtype=torch.int64, device=dev)
        col = torch.where(m.unsqueeze(-1), c, col)
    return fgm, col


def make_frames(spec: StreamSpec, frames: Sequence[int], device="cpu",
                with_truth: bool = False, out: Optional[torch.Tensor] = None):
    """Generate the given frame indices of a stream.

    Returns uint8 [len(frames), height, row_pitch] (and, with ``with_truth``,
    the bool ground-truth foreground [len(frames), height, width]).
    """
    H, W, P = spec.height, spec.width, spec.row_pitch
    frames = list(frames)
    dev = torch.device(device)
    if out is None:
        out = torch.zeros((len(frames), H, P), dtype=torch.uint8, device=dev)
    truth = torch.zeros((len(frames), H, W), dtype=torch.bool, device=dev) if with_truth else None
    pal = palette(spec, dev)
    ys = torch.arange(H, device=dev, dtype=torch.int64).view(H, 1)
    xs = torch.arange(W, device=dev, dtype=torch.int64).view(1, W)
    pix = (ys * W + xs)
    nbx = (W + spec.block - 1) // spec.block
    pal_flat = pal.reshape(-1, 3)
    pal_base = ((ys // spec.block) * nbx + xs // spec.block) * spec.n_palette
    sk = _stream_key(spec)
    hb = fmix32(pix ^ fmix32(sk ^ _P_BIMODAL))
    bimodal = hb < int(spec.bimodal_frac * 4294967296.0)
    phase = fmix32(hb ^ 0x5851F42D) % spec.bimodal_period
    ntab = torch.tensor(noise_table(spec.noise_sigma), dtype=torch.int64, device=dev)
    thr0, thr1, thr2 = PICK_THRESHOLDS
    for i, f in enumerate(frames):
        hf = fmix32(sk ^ fmix32((f + _P_FRAME) & M32))
        base = fmix32(pix ^ hf)
        u = base & 0xFFFF
        ci = (u >= thr0).long() + (u >= thr1).long() + (u >= thr2).long()
        if spec.bimodal_frac > 0.0:
            bi = ((f + phase) % spec.bimodal_period >= 4).long()
            ci = torch.where(bimodal, bi, ci)
        c = pal_flat[pal_base + ci]                        # [H, W, 3]
        s = drift_scale_q16(spec, f)
        if s != 65536:
            c = torch.clamp((c * s + 32768) >> 16, max=255)
        h2 = fmix32(base ^ _P_NOISE_A)
        h3 = fmix32(base ^ _P_NOISE_B)
        n = torch.stack([ntab[h2 & 0xFFFF], ntab[h2 >> 16], ntab[h3 & 0xFFFF]], dim=-1)
        c = torch.clamp(c + n, 0, 255)
        fgm, fcol = _foreground(spec, f, ys, xs)
        c = torch.where(fgm.unsqueeze(-1), fcol, c)
        out[i, :, : 3 * W] = c.to(torch.uint8).view(H, 3 * W)
        if with_truth:
            truth[i] = fgm
    if with_truth:
        return out, truth
    return out


# ---------------------------------------------------------------------------
# The five workloads.  Shapes, counts and merge thresholds are the workload
# definitions; generator parameters (palette, noise, drift, bimodal fraction,
# foreground) follow the same definitions.

@dataclass
class Workload:
    name: str
    streams: List[StreamSpec]
    depth: List[int]              # per stream
    thr: List[tuple]              # per stream (num, den)
    region: tuple = (0, 0)        # (region_w, region_h); (0, 0) = one tree per frame


def cfg0(seed: int = 0) -> Workload:
    s = StreamSpec(160, 120, 20, 20, seed=seed, fg="rect")
    return Workload("plain-160x120-d4-T20", [s], [4], [(1, 2)])


def cfg1(seed: int = 1, n_test: int = 1000) -> Workload:
    s = StreamSpec(1920, 1080, 50, n_test, seed=seed, bimodal_frac=0.2, drift_amp=0.1,
                   fg="ellipses", fg_coverage=0.05)
    return Workload("plain-1920x1080-d5-T50", [s], [5], [(1, 2)])


def cfg2(seed: int = 2, n_test: int = 500) -> Workload:
    s = StreamSpec(3840, 2160, 30, n_test, seed=seed, bimodal_frac=0.2, drift_amp=0.1,
                   fg="ellipses", fg_coverage=0.10)
    return Workload("region32-3840x2160-d4-T30", [s], [4], [(1, 2)], region=(32, 32))


MIX_RES = [(320, 240), (640, 480), (1280, 720), (1920, 1080), (3840, 2160)]
MIX_THR = [(3, 10), (1, 2), (7, 10)]


def mixed_streams(n_streams: int, seed: int, n_test: int = 200):
    """The uneven multi-stream mix: resolution, depth, T and threshold per stream."""
    rng = random.Random(f"mix/{seed}")
    streams, depths, thrs = [], [], []
    for s in range(n_streams):
        w, h = MIX_RES[rng.randrange(len(MIX_RES))]
        d = rng.choice([3, 4, 5, 6])
        T = rng.randint(20, 100)
        thr = MIX_THR[rng.randrange(len(MIX_THR))]
        streams.append(StreamSpec(w, h, T, n_test, seed=seed, stream=s, bimodal_frac=0.2,
                                  drift_amp=0.1, fg="ellipses", fg_coverage=0.05))
        depths.append(d)
        thrs.append(thr)
    return streams, depths, thrs


def cfg3(seed: int = 3, n_streams: int = 64, n_test: int = 200) -> Workload:
    st, d, t = mixed_streams(n_streams, seed, n_test)
    return Workload("batched-64-streams-mixed", st, d, t)


def cfg4(seed: int = 4, n_streams: int = 256):
    """The served mix: the batched resolution / depth / T / threshold mix plus a
    Poisson frame rate per stream drawn uniformly from 5-30 fps.  Frames are
    indexed from 0 without end; how many arrive depends on the duration."""
    specs, depths, thrs = mixed_streams(n_streams, seed, n_test=0)
    rng = random.Random(f"rates/{seed}")
    rates = [rng.uniform(5.0, 30.0) for _ in range(n_streams)]
    return specs, depths, thrs, rates


def scaled(spec: StreamSpec, **kw) -> StreamSpec:
    """Same stream with some fields replaced (objects recomputed)."""
    kw.setdefault("objects", [])
    return replace(spec, **kw)
