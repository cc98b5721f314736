"""Seeded synthetic surveillance frames drawn on the GPU with torch.

For workloads too large to draw on the host in reasonable time (many
streams at up to 1280x720): the same kind of scene as synth.video (bilinear
colour-gradient background, a bimodal square alternating between two colours,
moving flat-colour rectangles for the foreground, per-pixel Gaussian noise
rounded and clipped to u8), drawn with torch on the device.  The results
depend on the torch version's random-number kernels, so these frames serve
timing runs, and the one parity test whose frames are too large to draw on
the host (the maximum frame size), which hands the oracle the same bytes.

Nothing here implements any part of the background-subtraction method.
"""
from __future__ import annotations

import math

import numpy as np


class DeviceScene:
    """One RGB u8 stream of width x height pixels drawn on `device`."""

    def __init__(self, width: int, height: int, seed: int, device="cuda", fg_occ: float = 0.05,
                 n_rects: int = 8, noise_sigma: float = 4.0, dyn_period: int = 17):
        import torch
        self.torch = torch
        self.w, self.h, self.seed, self.device = width, height, seed, device
        self.noise = noise_sigma
        self.period = dyn_period
        rng = np.random.default_rng([seed, 1])
        corners = rng.uniform(40.0, 215.0, size=(4, 3)).astype(np.float32)
        ys = torch.linspace(0.0, 1.0, height, device=device).view(height, 1, 1)
        xs = torch.linspace(0.0, 1.0, width, device=device).view(1, width, 1)
        c = torch.from_numpy(corners).to(device)
        self.bg = ((1 - ys) * (1 - xs) * c[0] + (1 - ys) * xs * c[1] + ys * (1 - xs) * c[2]
                   + ys * xs * c[3]).contiguous()
        # bimodal square: side 1/8 of the shorter edge, colours >= 60 apart
        self.dsz = max(2, min(width, height) // 8)
        self.dpos = (int(rng.integers(0, max(1, height - self.dsz))),
                     int(rng.integers(0, max(1, width - self.dsz))))
        ca = rng.uniform(40.0, 120.0, size=3)
        self.dcol = (torch.tensor(ca, dtype=torch.float32, device=device),
                     torch.tensor(ca + rng.uniform(60.0, 90.0, size=3), dtype=torch.float32,
                                  device=device))
        # moving rectangles sized for the foreground occupancy
        side = max(2, int(round(math.sqrt(fg_occ * width * height / max(1, n_rects)))))
        side = min(side, width, height)
        self.rects = []
        for _ in range(n_rects):
            col = torch.tensor(rng.uniform(0.0, 255.0, size=3), dtype=torch.float32, device=device)
            self.rects.append(dict(s=side, y=float(rng.uniform(0, height - side)),
                                   x=float(rng.uniform(0, width - side)),
                                   vy=float(rng.uniform(-2.0, 2.0)), vx=float(rng.uniform(-2.0, 2.0)),
                                   col=col))

    def _pos(self, r, t):
        """Position at frame t of a rectangle bouncing at the borders."""
        def bounce(p0, v, lim):
            if lim <= 0:
                return 0
            q = (p0 + v * t) % (2 * lim)
            return int(q if q <= lim else 2 * lim - q)
        return bounce(r["y"], r["vy"], self.h - r["s"]), bounce(r["x"], r["vx"], self.w - r["s"])

    def frames(self, t0: int, n: int, out=None):
        """Frames t0 .. t0+n-1 as a u8 tensor [n, H, W, 3] on the device."""
        torch = self.torch
        if out is None:
            out = torch.empty((n, self.h, self.w, 3), dtype=torch.uint8, device=self.device)
        g = torch.Generator(device=self.device)
        for i in range(n):
            t = t0 + i
            g.manual_seed(self.seed * 1000003 + t)
            f = self.bg.clone()
            y0, x0 = self.dpos
            a = 0.5 * (1.0 + math.sin(2.0 * math.pi * t / self.period))
            f[y0:y0 + self.dsz, x0:x0 + self.dsz] = self.dcol[0] + (self.dcol[1] - self.dcol[0]) * a
            for r in self.rects:
                y, x = self._pos(r, t)
                f[y:y + r["s"], x:x + r["s"]] = r["col"]
            f += torch.randn(f.shape, generator=g, device=self.device) * self.noise
            out[i] = f.round_().clamp_(0.0, 255.0).to(torch.uint8)
        return out
