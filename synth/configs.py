"""Registry of the named EvSNet workloads and their input recipes.

Each workload fixes the clip shape, the network's channel list, the BiLIF
threshold and leak, the noise level and every seed.  ``make_clip`` builds the
noisy input of any window of a workload on any torch device.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from .scenes import moving_disc, spp_noise, textured_planes
from .weights import he_weights


@dataclass(frozen=True)
class Workload:
    name: str
    T: int
    H: int
    W: int
    channels: tuple
    spp: int = 1
    scene: str = "planes"         # "disc" | "planes"
    scene_seed: int = 1
    noise_seed: int = 2
    weight_seed: int = 0
    theta: float = 0.5
    leak: float = 0.9
    N: int = 1
    note: str = field(default="", compare=False)

    def weights(self):
        return he_weights(self.channels, self.weight_seed)

    @property
    def px_frames(self) -> int:
        return self.N * self.T * self.H * self.W


WORKLOADS = {
    "disc64": Workload(
        "disc64", T=16, H=64, W=64, channels=(3, 8, 2), spp=4, scene="disc",
        scene_seed=0, noise_seed=1, weight_seed=0,
        note="plain FP32 forward, moving disc, 4-SPP noise, 3->8->2"),
    "planes720": Workload(
        "planes720", T=1000, H=720, W=1280, channels=(3, 16, 16, 2), spp=1,
        scene="planes", scene_seed=1, noise_seed=2, weight_seed=0,
        note="plain FP32 forward, 1000 frames of 720p textured planes, 1-SPP, 3->16->16->2"),
    "planes720_w32": Workload(
        "planes720_w32", T=1000, H=720, W=1280, channels=(3, 32, 2), spp=1,
        scene="planes", scene_seed=1, noise_seed=2, weight_seed=0,
        note="precision form: 3->32->2 on the same 720p clip, FP32 and BF16 MFMA"),
    "train256": Workload(
        "train256", T=64, H=256, W=256, channels=(3, 16, 16, 2), spp=1,
        scene="planes", scene_seed=1, noise_seed=2, weight_seed=0, N=4,
        note="training step: 4 crops 256x256, T=64, EMD loss, BPTT with checkpoints every 16"),
}


def make_clip(wl: Workload, device="cpu", t0: int = 0, T: int | None = None,
              y0: int = 0, x0: int = 0, H: int | None = None, W: int | None = None,
              spp: int | None = None, scene_seed: int | None = None,
              noise_seed: int | None = None, clean: bool = False, out: torch.Tensor | None = None,
              chunk_pixels: int = 1 << 24) -> torch.Tensor:
    """Input window [T,3,H,W] float32 of workload ``wl`` at absolute offsets.

    Frames are generated in chunks of about ``chunk_pixels`` pixels (bounded
    temporaries) and written into ``out`` if given."""
    T = wl.T if T is None else T
    H = wl.H if H is None else H
    W = wl.W if W is None else W
    spp = wl.spp if spp is None else spp
    ss = wl.scene_seed if scene_seed is None else scene_seed
    ns = wl.noise_seed if noise_seed is None else noise_seed
    out = torch.empty(T, 3, H, W, dtype=torch.float32, device=device) if out is None else out
    step = max(1, chunk_pixels // (H * W))
    for c0 in range(0, T, step):
        c1 = min(T, c0 + step)
        if wl.scene == "disc":
            c = moving_disc(c1 - c0, H, W, t0=t0 + c0, y0=y0, x0=x0, device=device)
        else:
            c = textured_planes(c1 - c0, H, W, seed=ss, t0=t0 + c0, y0=y0, x0=x0, device=device)
        out[c0:c1] = c if clean else spp_noise(c, spp, ns, t0=t0 + c0, y0=y0, x0=x0)
    return out


def train_crops(wl: Workload, device="cpu", seed: int = 3, n: int | None = None):
    """Crop windows (t0, y0, x0) of the training batch, drawn from a 720p,
    1000-frame textured-planes clip."""
    rng = np.random.default_rng(seed)
    n = wl.N if n is None else n
    out = []
    for _ in range(n):
        t0 = int(rng.integers(0, 1000 - wl.T + 1))
        y0 = int(rng.integers(0, 720 - wl.H + 1))
        x0 = int(rng.integers(0, 1280 - wl.W + 1))
        out.append((t0, y0, x0))
    return out


def batch_clip_table(seed: int = 4, n_clips: int = 12):
    """Uneven clip batch: (H, W, T, spp, scene_seed, noise_seed) per clip.

    Resolution uniform over {320x240, 640x480, 1280x720, 1920x1080}, length
    uniform over the integers 100..2000 and SPP uniform over 1..8.
    """
    rng = np.random.default_rng(seed)
    res = [(240, 320), (480, 640), (720, 1280), (1080, 1920)]
    out = []
    for i in range(n_clips):
        H, W = res[int(rng.integers(0, 4))]
        T = int(rng.integers(100, 2001))
        spp = int(rng.integers(1, 9))
        out.append(dict(H=H, W=W, T=T, spp=spp, scene_seed=100 + i, noise_seed=200 + i))
    return out
