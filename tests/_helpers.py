"""Shared helpers of the GPU parity tests (not collected by pytest)."""

from __future__ import annotations

import numpy as np
import torch

import synth
from oracle import evsnet

F32 = np.float32

# Gate of the BF16 nets' gradients against the FP64 oracle (on the
# bf16-rounded x and W the forward multiplied).  Their backward keeps the
# adjoint g_h of every layer in bf16 between kernels (relative rounding
# <= 2^-9 per value) and the segment potentials in fp16 (the surrogate then
# moves by at most alpha |h| 2^-11 relative); layer 1's adjoint carries the
# roundings of the three layers above it.  Five units of 2^-9: 1e-2
# (measured 0.7e-3 .. 2.9e-3 on the small cases, max-normalised).
BF16_GRAD_TOL = 1e-2


def grad_tol(prec):
    return BF16_GRAD_TOL if prec == "bf16" else 1e-4


def f32(v):
    return float(np.float32(v))


def make_inputs(channels, T, H, W, N=1, seed=0, scale=1.0, y0=37, x0=51):
    """Seeded synthetic clip batch [N,T,C,H,W] (textured planes, 1-SPP noise)
    and He weights; for Cin = 1 the luminance-like mean of the RGB is used."""
    wl = synth.WORKLOADS["planes720"]
    xs = []
    for n in range(N):
        x = synth.make_clip(wl, T=T, H=H, W=W, y0=y0 + 97 * n, x0=x0 + 131 * n, noise_seed=2 + n)
        if channels[0] == 1:
            x = x.mean(dim=1, keepdim=True)
        xs.append(x * scale)
    x = torch.stack(xs).contiguous()
    ws = synth.he_weights(channels, seed)
    return x, ws


def split_layers(h, channels):
    """[T, sumC, H, W] -> list of per-layer [T, C_l, H, W]."""
    out, o = [], 0
    for c in channels[1:]:
        out.append(h[:, o:o + c])
        o += c
    return out


def fire32(h, theta):
    h = np.asarray(h, np.float32)
    th = np.float32(theta)
    return (h >= th).astype(np.float64) - (h <= -th).astype(np.float64)


def teacher_forced_report(x, ws, theta, leak, h_dev_layers, band=1e-3, v_init=None, quant_ws=None,
                          quant_x=None):
    """Teacher-forced one-step parity of a device trajectory.

    Returns dict with, per layer, the relative membrane error (against the
    unquantised FP64 step) and spike mismatches against the (optionally
    BF16-quantised) FP64 step, plus how many of those fall outside the
    near-threshold band.
    """
    x64 = np.asarray(x, np.float64)
    refs = evsnet.teacher_forced(x64, ws, theta, leak, h_dev_layers, v_init=v_init)
    if quant_ws is not None:
        qrefs = evsnet.teacher_forced(quant_x, quant_ws, theta, leak, h_dev_layers, v_init=v_init)
    else:
        qrefs = refs
    rep = []
    for hd, r, qr in zip(h_dev_layers, refs, qrefs):
        hd = np.asarray(hd, np.float64)
        rel = np.abs(hd - r).max() / max(np.abs(r).max(), 1e-30)
        qrel = np.abs(hd - qr).max() / max(np.abs(qr).max(), 1e-30)
        sd = evsnet.fire(hd, theta)
        sq = evsnet.fire(qr, theta)
        mism = sd != sq
        outside = mism & (evsnet.spike_margin(qr, theta) >= band)
        rep.append(dict(rel=rel, qrel=qrel, mism=int(mism.sum()), outside=int(outside.sum()),
                        n=int(sd.size), spikes=int(np.abs(sd).sum())))
    return rep
