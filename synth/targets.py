"""Target events for the training workload (inputs only).

The paper trains against events that an external event simulator derives
from noiseless high-SPP renders (Sec. 3.3, loss functions); neither the
simulator nor the renders exist here.  The stand-in is the idealised event
camera the paper describes in Sec. 3.1: a pixel emits one event each time its
log luminance moves by the contrast threshold C from the level at its last
event.  The luminance weights and the linear-below-knee logarithm follow
Eq. (1), on a 0-255 luminance scale with knee rho = 20 so that the linear
branch is continuous and increasing.
"""

from __future__ import annotations

import math

import torch


def contrast_events(clean: torch.Tensor, C: float = 0.2, knee: float = 20.0) -> torch.Tensor:
    """ON/OFF event counts [T, 2, H, W] int8 from clean frames [T, 3, H, W].

    Channel 0 counts ON (positive) crossings and channel 1 OFF crossings.
    Frame 0 sets the reference level and emits nothing; counts are clamped
    to 127.
    """
    c = clean.to(torch.float64)
    L = 255.0 * (0.2126 * c[:, 0] + 0.7152 * c[:, 1] + 0.0722 * c[:, 2])
    lin = (math.log(knee) / knee) * L
    logl = torch.where(L >= knee, torch.log(torch.clamp(L, min=1e-300)), lin)
    T = clean.shape[0]
    out = torch.zeros(T, 2, clean.shape[2], clean.shape[3], dtype=torch.int8, device=clean.device)
    ref = logl[0].clone()
    for t in range(1, T):
        d = logl[t] - ref
        n = torch.sign(d) * torch.floor(torch.abs(d) / C)
        ref = ref + n * C
        out[t, 0] = torch.clamp(n, min=0, max=127).to(torch.int8)
        out[t, 1] = torch.clamp(-n, min=0, max=127).to(torch.int8)
    return out
