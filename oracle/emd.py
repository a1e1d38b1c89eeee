"""FP64 oracle of the bidirectional, polarity-split EMD loss (Sec. 3.3).

Test infrastructure only (see the package docstring).  Time is axis 0.

* Eq. (7): the 1-D EMD between equal-length sequences is the L1 norm of the
  difference of their cumulative sums, averaged over the K = T time steps.
* Eq. (8): the same quantity on the time-reversed sequences is added and the
  two are averaged, so an unmatched event costs the same wherever it lies.
* Eq. (9): positive and negative parts are scored separately.  With a
  single bipolar output channel S the parts are S*[S>0] and -S*[S<0]; with
  the two-channel net (channel 0 = ON stream, channel 1 = OFF stream) each
  channel is scored, with its signed spikes, against the matching target
  count E_on or E_off.
* Eq. (10-11): optional per-pixel spike-count term weighted by lambda.

Norm reading: the L1 norm sums over pixels (and clips); the loss returned is
that sum.  The subgradient of |z| at z = 0 is taken as 0.
"""

from __future__ import annotations

import numpy as np


def emd_forward_dir(S: np.ndarray, E: np.ndarray) -> np.ndarray:
    """Eq. (7) per sequence (all axes but 0 are independent sequences)."""
    T = S.shape[0]
    return np.abs(np.cumsum(np.asarray(S, np.float64) - np.asarray(E, np.float64), axis=0)).sum(axis=0) / T


def emd_bidir(S: np.ndarray, E: np.ndarray) -> np.ndarray:
    """Eq. (8) per sequence: mean of the forward and time-reversed EMD."""
    return 0.5 * (emd_forward_dir(S, E) + emd_forward_dir(S[::-1], E[::-1]))


def emd_bidir_grad(S: np.ndarray, E: np.ndarray) -> np.ndarray:
    """d emd_bidir / dS: (1/2T) [sum_{i>=j} sgn D_i + sum_{m<=j} sgn R_m],

    with D the prefix sums and R the suffix sums of S - E.
    """
    T = S.shape[0]
    d = np.asarray(S, np.float64) - np.asarray(E, np.float64)
    D = np.cumsum(d, axis=0)
    R = np.cumsum(d[::-1], axis=0)[::-1]
    gD = np.cumsum(np.sign(D)[::-1], axis=0)[::-1]
    gR = np.cumsum(np.sign(R), axis=0)
    return (gD + gR) / (2.0 * T)


def split_polarity(S: np.ndarray, E: np.ndarray | None = None):
    """Eq. (9) split for single-channel bipolar sequences: (S+, S-)."""
    S = np.asarray(S, np.float64)
    return S * (S > 0), -S * (S < 0)


def loss_and_grad(S: np.ndarray, E_on: np.ndarray, E_off: np.ndarray, lam: float = 0.0):
    """Total loss L_EMD + lam * L_count and dL/dS.

    S      [T, C, ...] with C = 2 (ON, OFF channels) or C = 1 (bipolar)
    E_on   [T, ...] ON counts (>= 0);  E_off [T, ...] OFF counts (>= 0)
    """
    S = np.asarray(S, np.float64)
    E_on = np.asarray(E_on, np.float64)
    E_off = np.asarray(E_off, np.float64)
    C = S.shape[1]
    g = np.zeros_like(S)
    if C == 2:
        sp, sn = S[:, 0], S[:, 1]
        loss = emd_bidir(sp, E_on).sum() + emd_bidir(sn, E_off).sum()
        g[:, 0] = emd_bidir_grad(sp, E_on)
        g[:, 1] = emd_bidir_grad(sn, E_off)
        count = np.abs(S[:, 0]).sum(0) + np.abs(S[:, 1]).sum(0) - (E_on + E_off).sum(0)
        if lam:
            loss += lam * np.abs(count).sum()
            g[:, 0] += lam * np.sign(count)[None] * np.sign(S[:, 0])
            g[:, 1] += lam * np.sign(count)[None] * np.sign(S[:, 1])
    elif C == 1:
        s = S[:, 0]
        sp, sn = split_polarity(s)
        loss = emd_bidir(sp, E_on).sum() + emd_bidir(sn, E_off).sum()
        g[:, 0] = emd_bidir_grad(sp, E_on) * (s > 0) - emd_bidir_grad(sn, E_off) * (s < 0)
        count = np.abs(s).sum(0) - (E_on + E_off).sum(0)
        if lam:
            loss += lam * np.abs(count).sum()
            g[:, 0] += lam * np.sign(count)[None] * np.sign(s)
    else:
        raise ValueError("C must be 1 or 2")
    return float(loss), g
