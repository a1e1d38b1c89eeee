"""FP64 oracle of the network input (Eq. 1) and of the contrast-crossing
target events.  Test infrastructure only (see the package docstring).

Eq. (1), Sec. 3.2: per pixel, the luminance of the linear RGB frame

    L = 0.2126 R + 0.7152 G + 0.0722 B

is mapped to log space with a linear toe below the knee rho,

    L_log = ln L              if L >= rho
            (ln rho / rho) L  if L <  rho,

and the network input is its temporal difference X_k = L_log[k] - L_log[k-1]
(k = 1..K from frames 0..K).  Reading: L is taken on a 0-255 scale
(L = lum_scale * (weights . rgb), lum_scale = 255) with rho = 20, for which
the two branches meet at L = rho and the map is increasing (with rho < 1 the
linear branch would decrease).

Targets (the stand-in for the external simulator the paper trains against):
an ideal contrast-threshold camera on the clean frames.  Per pixel the
reference level starts at L_log of frame 0; at every later frame the change
d = L_log[t] - ref emits n = sgn(d) floor(|d| / C) events, ref moves by n C,
and ON = max(n, 0), OFF = max(-n, 0) are stored (clamped to 127).  Frame 0
emits nothing.
"""

from __future__ import annotations

import numpy as np

LUMA = (0.2126, 0.7152, 0.0722)


def luminance(rgb: np.ndarray, lum_scale: float = 255.0) -> np.ndarray:
    """[..., 3, H, W] -> [..., H, W], scaled."""
    rgb = np.asarray(rgb, dtype=np.float64)
    return lum_scale * (LUMA[0] * rgb[..., 0, :, :] + LUMA[1] * rgb[..., 1, :, :] + LUMA[2] * rgb[..., 2, :, :])


def linlog(L: np.ndarray, knee: float = 20.0) -> np.ndarray:
    L = np.asarray(L, dtype=np.float64)
    lin = (np.log(knee) / knee) * L
    return np.where(L >= knee, np.log(np.maximum(L, knee)), lin)


def logdiff(rgb: np.ndarray, lum_scale: float = 255.0, knee: float = 20.0) -> np.ndarray:
    """Network input of Eq. (1): [K+1, 3, H, W] frames -> X [K, 1, H, W]."""
    l = linlog(luminance(rgb, lum_scale), knee)
    return (l[1:] - l[:-1])[:, None]


def contrast_events(rgb: np.ndarray, C: float = 0.2, lum_scale: float = 255.0, knee: float = 20.0):
    """Target events [T, 2, H, W] (int8 ON, OFF counts) of clean frames [T, 3, H, W]."""
    l = linlog(luminance(rgb, lum_scale), knee)
    T = l.shape[0]
    out = np.zeros((T, 2) + l.shape[1:], dtype=np.int8)
    ref = l[0].copy()
    for t in range(1, T):
        d = l[t] - ref
        n = np.sign(d) * np.floor(np.abs(d) / C)
        ref = ref + n * C
        out[t, 0] = np.clip(n, 0, 127)
        out[t, 1] = np.clip(-n, 0, 127)
    return out


def contrast_margin(rgb: np.ndarray, C: float = 0.2, lum_scale: float = 255.0, knee: float = 20.0) -> np.ndarray:
    """Per pixel, the smallest distance of q = |d| / C to a boundary of
    floor(q), i.e. to an integer >= 1, over all frames (along the oracle's own
    trajectory): where it is tiny, a rounding of a different precision may
    decide the event count differently."""
    l = linlog(luminance(rgb, lum_scale), knee)
    ref = l[0].copy()
    m = np.full(l.shape[1:], np.inf)
    for t in range(1, l.shape[0]):
        d = l[t] - ref
        q = np.abs(d) / C
        m = np.minimum(m, np.abs(q - np.maximum(np.round(q), 1.0)))
        ref = ref + np.sign(d) * np.floor(q) * C
    return m
