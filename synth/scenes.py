"""Analytic clean scenes and the low-SPP noise model (inputs only).

Scenes are evaluated at absolute pixel coordinates (t, y, x), so a window
(t0, y0, x0, T, H, W) of a large clip is regenerated exactly by asking for
that window.  Everything is computed with torch on the requested device, in
float32 for the scene and float64 for the noise logarithms.

The paper renders its frames with a Monte-Carlo path tracer at a low sample
count (Sec. 3.2); no renderer is available here, so the noise model stands in
for it: a pixel estimated from n samples of a path tracer whose per-sample
throughput is exponentially distributed around the clean radiance is the
clean radiance times Gamma(n, 1)/n.  One set of n draws per (t, y, x) is
shared by R, G and B (a path carries all three channels).
"""

from __future__ import annotations

import math

import numpy as np
import torch

_M32 = 0xFFFFFFFF


def _mix32(h: torch.Tensor) -> torch.Tensor:
    # 32-bit integer finaliser (xor-shift / multiply); every product stays
    # below 2**63 so int64 arithmetic never overflows on any device.
    h = h ^ (h >> 16)
    h = (h * 0x045D9F3B) & _M32
    h = h ^ (h >> 16)
    h = (h * 0x045D9F3B) & _M32
    h = h ^ (h >> 16)
    return h


def hash_u32(seed: int, *coords: torch.Tensor) -> torch.Tensor:
    """Counter-based hash of (seed, coords...) to uint32 values held in int64."""
    shape = torch.broadcast_shapes(*[c.shape for c in coords])
    dev = coords[0].device
    h = torch.full(shape, (seed * 0x27D4EB2D + 0x165667B1) & _M32, dtype=torch.int64, device=dev)
    for c in coords:
        c = c.to(torch.int64) & _M32
        h = _mix32((h ^ ((c * 0x27D4EB2D + 0x3C6EF372) & _M32)) & _M32)
    return h


def hash_uniform(seed: int, *coords: torch.Tensor) -> torch.Tensor:
    """Uniform (0, 1) float64 values, a pure function of (seed, coords)."""
    return (hash_u32(seed, *coords).to(torch.float64) + 0.5) * (1.0 / 4294967296.0)


def _grid(T, H, W, t0, y0, x0, device):
    t = torch.arange(t0, t0 + T, device=device, dtype=torch.int64).view(T, 1, 1)
    y = torch.arange(y0, y0 + H, device=device, dtype=torch.int64).view(1, H, 1)
    x = torch.arange(x0, x0 + W, device=device, dtype=torch.int64).view(1, 1, W)
    return t, y, x


def moving_disc(T: int, H: int = 64, W: int = 64, t0: int = 0, y0: int = 0, x0: int = 0,
                device="cpu") -> torch.Tensor:
    """Clean frames [T,3,H,W] of a disc moving over a grey background.

    Background radiance 0.2 in all channels; disc of radius 10 px with
    radiance (1.0, 0.7, 0.4); its centre moves 2.5 px/frame along x from
    x = 14 with a sinusoidal +-8 px wobble in y around y = 32 (period 16
    frames).  Edge coverage is the fraction of a 4x4 grid of sub-samples per
    pixel that falls inside the disc.
    """
    t, y, x = _grid(T, H, W, t0, y0, x0, device)
    tf = t.to(torch.float64)
    cx = 14.0 + 2.5 * tf
    cy = 32.0 + 8.0 * torch.sin(2.0 * math.pi * tf / 16.0)
    cover = torch.zeros(T, H, W, dtype=torch.float64, device=device)
    for i in range(4):
        for j in range(4):
            sy = y.to(torch.float64) + (i + 0.5) / 4.0
            sx = x.to(torch.float64) + (j + 0.5) / 4.0
            inside = ((sx - cx) ** 2 + (sy - cy) ** 2) <= 100.0
            cover = cover + inside.to(torch.float64)
    cover = cover / 16.0
    bg = 0.2
    disc = torch.tensor([1.0, 0.7, 0.4], dtype=torch.float64, device=device).view(1, 3, 1, 1)
    out = bg + cover.unsqueeze(1) * (disc - bg)
    return out.to(torch.float32).contiguous()


def _plane_params(seed: int, n_planes: int = 4):
    rng = np.random.default_rng(seed)
    planes = []
    lo, hi = math.log(0.02), math.log(4.0)
    for p in range(n_planes):
        speed = rng.uniform(0.0, 20.0)
        ang = rng.uniform(0.0, 2.0 * math.pi)
        gratings = []
        for _ in range(3):
            period = rng.uniform(8.0, 64.0)
            theta = rng.uniform(0.0, math.pi)
            phase = rng.uniform(0.0, 2.0 * math.pi)
            gratings.append((2.0 * math.pi / period * math.cos(theta),
                             2.0 * math.pi / period * math.sin(theta), phase))
        col_a = rng.uniform(lo, hi, size=3)
        col_b = rng.uniform(lo, hi, size=3)
        mask = None
        if p > 0:
            mask = (rng.uniform(0.0, 1280.0), rng.uniform(0.0, 720.0),
                    rng.uniform(100.0, 300.0), rng.uniform(2.0, 12.0))
        planes.append(dict(vx=speed * math.cos(ang), vy=speed * math.sin(ang),
                           gratings=gratings, col_a=col_a, col_b=col_b, mask=mask,
                           noise_seed=int(rng.integers(0, 2**31 - 1))))
    return planes


def _value_noise(seed, qy, qx, cell=16.0):
    gy = torch.floor(qy / cell)
    gx = torch.floor(qx / cell)
    fy = qy / cell - gy
    fx = qx / cell - gx
    fy = fy * fy * (3.0 - 2.0 * fy)
    fx = fx * fx * (3.0 - 2.0 * fx)
    iy = gy.to(torch.int64)
    ix = gx.to(torch.int64)
    h00 = hash_uniform(seed, iy, ix).to(qy.dtype)
    h01 = hash_uniform(seed, iy, ix + 1).to(qy.dtype)
    h10 = hash_uniform(seed, iy + 1, ix).to(qy.dtype)
    h11 = hash_uniform(seed, iy + 1, ix + 1).to(qy.dtype)
    top = h00 + (h01 - h00) * fx
    bot = h10 + (h11 - h10) * fx
    return top + (bot - top) * fy


def textured_planes(T: int, H: int, W: int, seed: int = 1, t0: int = 0, y0: int = 0,
                    x0: int = 0, device="cpu", chunk: int = 16) -> torch.Tensor:
    """Clean HDR frames [T,3,H,W] of four translating textured planes.

    Plane 0 fills the frame; planes 1-3 are soft-edged discs (radius
    100-300 px) composited front over back.  Each plane translates at
    |v| ~ U[0, 20] px/frame in a random direction.  Its texture m in [0, 1]
    mixes three oriented gratings (periods 8-64 px) with hashed value noise,
    and its radiance interpolates geometrically between two colours drawn
    log-uniformly in [0.02, 4] per channel, so radiance is log-spread over
    that HDR range.
    """
    planes = _plane_params(seed)
    out = torch.empty(T, 3, H, W, dtype=torch.float32, device=device)
    ys = (torch.arange(y0, y0 + H, device=device, dtype=torch.float32) + 0.5).view(1, H, 1)
    xs = (torch.arange(x0, x0 + W, device=device, dtype=torch.float32) + 0.5).view(1, 1, W)
    for c0 in range(0, T, chunk):
        c1 = min(T, c0 + chunk)
        tt = torch.arange(t0 + c0, t0 + c1, device=device, dtype=torch.float32).view(-1, 1, 1)
        acc = None
        for p in planes:
            qy = ys - p["vy"] * tt
            qx = xs - p["vx"] * tt
            g = torch.zeros(c1 - c0, H, W, dtype=torch.float32, device=device)
            for (ky, kx, ph) in p["gratings"]:
                g = g + torch.cos(ky * qy + kx * qx + ph)
            m = 0.5 * (g / 3.0 + 1.0)
            m = 0.6 * m + 0.4 * _value_noise(p["noise_seed"], qy, qx)
            m = m.clamp(0.0, 1.0).unsqueeze(1)
            la = torch.tensor(p["col_a"], dtype=torch.float32, device=device).view(1, 3, 1, 1)
            lb = torch.tensor(p["col_b"], dtype=torch.float32, device=device).view(1, 3, 1, 1)
            rad = torch.exp(la + (lb - la) * m)
            if p["mask"] is None:
                acc = rad
            else:
                mx, my, r, soft = p["mask"]
                d = torch.sqrt((qy - my) ** 2 + (qx - mx) ** 2)
                alpha = torch.sigmoid((r - d) / soft).unsqueeze(1)
                acc = alpha * rad + (1.0 - alpha) * acc
        out[c0:c1] = acc
    return out


def spp_noise(clean: torch.Tensor, spp: int, seed: int, t0: int = 0, y0: int = 0,
              x0: int = 0) -> torch.Tensor:
    """Low-SPP estimate: clean * Gamma(spp, 1)/spp, draws shared across RGB."""
    T, C, H, W = clean.shape
    t, y, x = _grid(T, H, W, t0, y0, x0, clean.device)
    g = torch.zeros(T, H, W, dtype=torch.float64, device=clean.device)
    for k in range(spp):
        kk = torch.full((1, 1, 1), k, dtype=torch.int64, device=clean.device)
        g = g - torch.log(hash_uniform(seed, t, y, x, kk))
    g = (g / spp).to(torch.float32).unsqueeze(1)
    return (clean * g).contiguous()
