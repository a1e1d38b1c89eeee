"""Seeded synthetic inputs for EvSNet workloads.

This package generates inputs only: analytic clean scenes, a low-SPP path
tracing noise model, He-initialised weights and the registry of named
workloads.  It contains none of the method's arithmetic (no Eq. 1 input or
target events, no convolution, no BiLIF, no loss), so both the FP64 oracle
and the HIP path can consume its outputs without sharing any method code;
target events come from the oracle (tests) or the library (benchmark).

Every random quantity is a pure function of (seed, coordinates) through a
32-bit integer hash, so a crop of a large clip can be regenerated exactly on
its own and the generators run on any torch device.
"""

from .scenes import moving_disc, textured_planes, spp_noise, hash_uniform
from .weights import he_weights
from .configs import WORKLOADS, Workload, make_clip, batch_clip_table, train_crops

__all__ = [
    "moving_disc", "textured_planes", "spp_noise", "hash_uniform",
    "he_weights", "WORKLOADS", "Workload", "make_clip",
    "batch_clip_table", "train_crops",
]
