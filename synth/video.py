"""Seeded synthetic video shaped like the paper's surveillance workloads.

The paper evaluates on surveillance videos (Wallflower, CDW-2014) that are not
available here.  These streams stand in for them: a smooth colour-gradient
background, per-pixel Gaussian camera noise, bimodal (sinusoidally
alternating) background regions, an optional slow global illumination wave
and a low-occupancy moving foreground (the paper's operating point: mostly
static surveillance scenes with little foreground, §1 and §3.2).

Determinism: every random draw comes from a Philox generator keyed by the
stream seed plus a purpose index (scene layout, motion) or the frame index
(noise), so any frame range can be regenerated on its own.

Nothing here implements any part of the background-subtraction method.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass
from typing import Iterator, Optional, Tuple

import numpy as np

BASE_SEED = 170509339

_LAYOUT_KEY = 2**31
_MOTION_KEY = 2**31 + 1


def _rng(*keys: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(np.random.SeedSequence(list(keys))))


@dataclass(frozen=True)
class StreamSpec:
    """Parameters of one synthetic RGB u8 stream (frames are HWC, tight)."""

    name: str
    width: int
    height: int
    frames: int
    n_train: int
    K: int
    seed: int
    noise_sigma: float = 4.0
    # bimodal background: squares whose colour swings between two colours
    dyn_regions: int = 1
    dyn_size: int = 30          # side in pixels (ignored when dyn_area_frac > 0)
    dyn_area_frac: float = 0.0  # if > 0, the regions together cover this area fraction
    dyn_periods: Tuple[int, ...] = (17,)
    # foreground
    const_rects: int = 3        # sides U[8,16] px, constant velocity |v| <= 2 px/frame
    rw_rects: int = 0           # random-walk rectangles of side rw_size
    rw_size: int = 28
    rw_vmax: float = 4.0
    ellipse_occ: float = 0.0    # random-walk ellipses; count solved for this mean occupancy
    # global additive illumination triangle wave, applied before noise
    illum_amp: float = 0.0
    illum_period: int = 400

    @property
    def pixels(self) -> int:
        return self.width * self.height

    def with_(self, **kw) -> "StreamSpec":
        return dataclasses.replace(self, **kw)


PRESETS = {
    # 160x120, 200 frames, prior over the first 50, K=3: one 30x30 bimodal
    # square (period 17) and three constant-velocity rectangles (~2 % FG).
    "surveil-160x120-k3": StreamSpec(
        name="surveil-160x120-k3", width=160, height=120, frames=200, n_train=50, K=3,
        seed=BASE_SEED + 1, const_rects=3),
    # 640x480, 1000 frames, prior over 100, K=5: as above plus a +-20 level
    # illumination wave over 400 frames and 20 random-walk 28x28 rectangles (~5 % FG).
    "surveil-640x480-k5": StreamSpec(
        name="surveil-640x480-k5", width=640, height=480, frames=1000, n_train=100, K=5,
        seed=BASE_SEED + 2, const_rects=3, rw_rects=20, rw_size=28,
        illum_amp=20.0, illum_period=400),
}
for _occ in (1, 5, 10, 30):
    # 1920x1080, 500 frames, prior over 100, K=5: bimodal regions on 10 % of the
    # area (periods 13/17/23) and random-walk ellipses at the given occupancy.
    PRESETS[f"surveil-1920x1080-k5-occ{_occ:02d}"] = StreamSpec(
        name=f"surveil-1920x1080-k5-occ{_occ:02d}", width=1920, height=1080, frames=500,
        n_train=100, K=5, seed=BASE_SEED + 3 + 100 * _occ, const_rects=0,
        dyn_regions=8, dyn_area_frac=0.10, dyn_periods=(13, 17, 23),
        ellipse_occ=_occ / 100.0)


def preset(name: str) -> StreamSpec:
    return PRESETS[name]


@dataclass
class _Obj:
    kind: str            # "rect" | "ellipse"
    w: float             # rect width / ellipse semi-axis x
    h: float             # rect height / ellipse semi-axis y
    x: float
    y: float
    vx: float
    vy: float
    color: np.ndarray    # (3,) float32
    walk: bool


class _Scene:
    def __init__(self, spec: StreamSpec):
        self.spec = spec
        W, H = spec.width, spec.height
        r = _rng(spec.seed, _LAYOUT_KEY)
        corners = r.uniform(40.0, 215.0, size=(2, 2, 3)).astype(np.float64)
        u = (np.arange(W, dtype=np.float64) + 0.5) / W
        v = (np.arange(H, dtype=np.float64) + 0.5) / H
        top = corners[0, 0][None, :] * (1 - u)[:, None] + corners[0, 1][None, :] * u[:, None]
        bot = corners[1, 0][None, :] * (1 - u)[:, None] + corners[1, 1][None, :] * u[:, None]
        self.bg = (top[None, :, :] * (1 - v)[:, None, None]
                   + bot[None, :, :] * v[:, None, None]).astype(np.float32)

        # bimodal regions
        self.dyn = []
        if spec.dyn_regions > 0:
            if spec.dyn_area_frac > 0:
                side = int(round(math.sqrt(spec.dyn_area_frac * W * H / spec.dyn_regions)))
            else:
                side = spec.dyn_size
            side = max(1, min(side, W, H))
            for i in range(spec.dyn_regions):
                x0 = int(r.integers(0, W - side + 1))
                y0 = int(r.integers(0, H - side + 1))
                while True:
                    ca = r.uniform(0.0, 255.0, size=3)
                    cb = r.uniform(0.0, 255.0, size=3)
                    if np.linalg.norm(ca - cb) >= 60.0:
                        break
                period = spec.dyn_periods[i % len(spec.dyn_periods)]
                self.dyn.append((y0, x0, side, ca.astype(np.float32), cb.astype(np.float32), period))

        objs = []
        for _ in range(spec.const_rects):
            w = min(int(r.integers(8, 17)), W)
            h = min(int(r.integers(8, 17)), H)
            ang = r.uniform(0, 2 * math.pi)
            spd = r.uniform(0.5, 2.0)
            objs.append(_Obj("rect", w, h, r.uniform(0, W - w), r.uniform(0, H - h),
                             spd * math.cos(ang), spd * math.sin(ang),
                             r.uniform(0, 255, size=3).astype(np.float32), False))
        for _ in range(spec.rw_rects):
            s = min(spec.rw_size, W, H)
            ang = r.uniform(0, 2 * math.pi)
            spd = r.uniform(0.5, spec.rw_vmax)
            objs.append(_Obj("rect", s, s, r.uniform(0, W - s), r.uniform(0, H - s),
                             spd * math.cos(ang), spd * math.sin(ang),
                             r.uniform(0, 255, size=3).astype(np.float32), True))
        if spec.ellipse_occ > 0:
            # semi-axes U[15,45]: mean area pi*30*30; Poisson coverage gives
            # union fraction 1-exp(-n*A/(W*H)), solved here for n.
            mean_area = math.pi * 30.0 * 30.0
            n = int(round(-math.log(1.0 - spec.ellipse_occ) * W * H / mean_area))
            for _ in range(max(n, 1)):
                a = r.uniform(15, 45)
                b = r.uniform(15, 45)
                ang = r.uniform(0, 2 * math.pi)
                spd = r.uniform(0.5, spec.rw_vmax)
                objs.append(_Obj("ellipse", a, b, r.uniform(a, W - a), r.uniform(b, H - b),
                                 spd * math.cos(ang), spd * math.sin(ang),
                                 r.uniform(0, 255, size=3).astype(np.float32), True))
        self.objs = objs
        self.motion = _rng(spec.seed, _MOTION_KEY)
        self.t = 0

    def _bounds(self, o: _Obj):
        W, H = self.spec.width, self.spec.height
        if o.kind == "rect":
            return 0.0, W - o.w, 0.0, H - o.h
        return o.w, W - o.w, o.h, H - o.h

    def snapshot(self):
        """Copies of the objects at the current frame (render() of a frame
        reads nothing else that advance() changes)."""
        return [dataclasses.replace(o) for o in self.objs]

    def advance(self):
        """Move every object by one frame."""
        vmax = self.spec.rw_vmax
        n_walk = sum(1 for o in self.objs if o.walk)
        jit = self.motion.normal(0.0, 0.5, size=(n_walk, 2)) if n_walk else None
        i = 0
        for o in self.objs:
            if o.walk:
                o.vx += jit[i, 0]
                o.vy += jit[i, 1]
                i += 1
                sp = math.hypot(o.vx, o.vy)
                if sp > vmax:
                    o.vx *= vmax / sp
                    o.vy *= vmax / sp
            x0, x1, y0, y1 = self._bounds(o)
            o.x += o.vx
            o.y += o.vy
            if o.x < x0 or o.x > x1:
                o.vx = -o.vx
                o.x = min(max(o.x, x0), x1)
            if o.y < y0 or o.y > y1:
                o.vy = -o.vy
                o.y = min(max(o.y, y0), y1)
        self.t += 1

    def render(self, t: int, objs=None) -> Tuple[np.ndarray, np.ndarray]:
        """Frame t with the objects where they are now (or at `objs`, a
        snapshot taken by `snapshot()` when the scene was at frame t)."""
        spec = self.spec
        objs = self.objs if objs is None else objs
        W, H = spec.width, spec.height
        img = self.bg.copy()
        lvl = np.float32(0.0)
        if spec.illum_amp != 0.0:
            ph = (t / spec.illum_period) % 1.0
            lvl = np.float32(spec.illum_amp * (4.0 * abs(ph - 0.5) - 1.0))
            img += lvl
        for (y0, x0, side, ca, cb, period) in self.dyn:
            f = np.float32((1.0 + math.sin(2.0 * math.pi * t / period)) / 2.0)
            img[y0:y0 + side, x0:x0 + side] = ca + (cb - ca) * f + lvl
        gt = np.zeros((H, W), dtype=bool)
        for o in objs:
            if o.kind == "rect":
                xa, ya = int(round(o.x)), int(round(o.y))
                xb, yb = min(W, xa + int(o.w)), min(H, ya + int(o.h))
                xa, ya = max(0, xa), max(0, ya)
                img[ya:yb, xa:xb] = o.color + lvl
                gt[ya:yb, xa:xb] = True
            else:
                xa, xb = max(0, int(math.floor(o.x - o.w))), min(W, int(math.ceil(o.x + o.w)) + 1)
                ya, yb = max(0, int(math.floor(o.y - o.h))), min(H, int(math.ceil(o.y + o.h)) + 1)
                # the same float64 terms as over a full coordinate grid, formed
                # once per column and per row and summed by broadcasting
                ex = ((np.arange(xa, xb) + 0.5 - o.x) / o.w) ** 2
                ey = ((np.arange(ya, yb) + 0.5 - o.y) / o.h) ** 2
                inside = ex[None, :] + ey[:, None] <= 1.0
                sub = img[ya:yb, xa:xb]
                sub[inside] = o.color + lvl
                gt[ya:yb, xa:xb] |= inside
        noise = _rng(spec.seed, t).standard_normal((H, W, 3), dtype=np.float32)
        img += noise * np.float32(spec.noise_sigma)
        np.rint(img, out=img)
        np.clip(img, 0.0, 255.0, out=img)
        return img.astype(np.uint8), gt


def iter_frames(spec: StreamSpec, start: int = 0, stop: Optional[int] = None
                ) -> Iterator[Tuple[int, np.ndarray, np.ndarray]]:
    """Yield (t, frame[H,W,3] u8, gt[H,W] bool) for t in [start, stop)."""
    stop = spec.frames if stop is None else stop
    sc = _Scene(spec)
    for t in range(stop):
        if t >= start:
            f, g = sc.render(t)
            yield t, f, g
        sc.advance()


def make_stream(spec: StreamSpec, start: int = 0, stop: Optional[int] = None,
                with_gt: bool = False, threads: int = 1):
    """Frames [start, stop) as one u8 array [n, H, W, 3] (and GT masks [n, H, W]).

    With threads > 1 the object motion is stepped through first (it is
    sequential and cheap) and the frames are drawn by a thread pool; every
    frame's noise has its own generator, so the result is the same array."""
    stop = spec.frames if stop is None else stop
    n = stop - start
    frames = np.empty((n, spec.height, spec.width, 3), dtype=np.uint8)
    gts = np.empty((n, spec.height, spec.width), dtype=bool) if with_gt else None
    if threads <= 1:
        for t, f, g in iter_frames(spec, start, stop):
            frames[t - start] = f
            if with_gt:
                gts[t - start] = g
        return (frames, gts) if with_gt else frames
    from concurrent.futures import ThreadPoolExecutor

    sc = _Scene(spec)
    snaps = {}
    for t in range(stop):
        if t >= start:
            snaps[t] = sc.snapshot()
        sc.advance()

    def draw(t):
        f, g = sc.render(t, snaps.pop(t))
        frames[t - start] = f
        if with_gt:
            gts[t - start] = g

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(draw, range(start, stop)))
    return (frames, gts) if with_gt else frames


# ---- micro streams for unit tests ------------------------------------------------

def constant_stream(n: int, h: int, w: int, c: int, value) -> np.ndarray:
    v = np.broadcast_to(np.asarray(value, dtype=np.uint8), (c,))
    return np.broadcast_to(v, (n, h, w, c)).copy()


def random_stream(n: int, h: int, w: int, c: int, seed: int, lo: int = 0, hi: int = 256) -> np.ndarray:
    return _rng(seed, 7).integers(lo, hi, size=(n, h, w, c), dtype=np.uint8)


def alternating_stream(n: int, h: int, w: int, c: int, a, b) -> np.ndarray:
    out = np.empty((n, h, w, c), dtype=np.uint8)
    out[0::2] = np.asarray(a, dtype=np.uint8)
    out[1::2] = np.asarray(b, dtype=np.uint8)
    return out


def step_stream(n: int, h: int, w: int, c: int, v0, v1, t_step: int) -> np.ndarray:
    out = np.empty((n, h, w, c), dtype=np.uint8)
    out[:t_step] = np.asarray(v0, dtype=np.uint8)
    out[t_step:] = np.asarray(v1, dtype=np.uint8)
    return out


# ---- latent-map streams ----------------------------------------------------------

def latent_stream(n: int, channels: int = 64, h: int = 30, w: int = 40, seed: int = BASE_SEED + 4,
                  noise: float = 0.1, drift_amp: float = 0.5, blob: bool = True,
                  start: int = 0) -> np.ndarray:
    """Frames [start, start + n) of a stream of f32 latent maps, flattened so
    that every (channel, y, x) element is one single-channel pixel:
    array [n, channels * h * w], element index (ch * h + y) * w + x.

    Each channel is a fixed Gaussian spatial pattern plus a slow sinusoidal
    drift of its own (period 300..900 frames, amplitude drift_amp) plus
    per-frame N(0, noise^2) noise; with blob, a 6x6 patch moving along a
    diagonal adds +2 to a quarter of the channels (a foreground object in
    latent space).  Values stay roughly within [-5, 5].
    """
    lay = _rng(seed, _LAYOUT_KEY)
    base = lay.normal(0.0, 1.0, size=(channels, h, w)).astype(np.float32)
    period = lay.uniform(300.0, 900.0, size=channels)
    phase = lay.uniform(0.0, 2.0 * math.pi, size=channels)
    fg_ch = lay.permutation(channels)[: max(1, channels // 4)]
    out = np.empty((n, channels * h * w), dtype=np.float32)
    for i in range(n):
        t = start + i
        d = (drift_amp * np.sin(2.0 * math.pi * t / period + phase)).astype(np.float32)
        fr = base + d[:, None, None]
        fr = fr + _rng(seed, t).normal(0.0, noise, size=(channels, h, w)).astype(np.float32)
        if blob:
            y0 = (t // 2) % max(1, h - 6)
            x0 = t % max(1, w - 6)
            fr[fg_ch, y0:y0 + 6, x0:x0 + 6] += np.float32(2.0)
        out[i] = fr.reshape(-1)
    return out
