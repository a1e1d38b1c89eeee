"""EvSNet on MI355X: conv3x3 + bipolar LIF event spiking network (arXiv 2508.18071).

The compute lives in libevs.so (hand-written HIP for gfx950, C ABI in
include/evs.h); this package only marshals torch tensors into it.
"""

from .api import (Net, TNet, Graph, pack_weights, forward, forward_batched, backward, emd_loss,
                  compact_events, logdiff, contrast_events, tnet_forward, tnet_weight_floats, autotune, set_tile,
                  tile_count, tile_name, status_word)
from ._lib import lib, EvsError, LIB_PATH, EXPORTED

__all__ = ["Net", "TNet", "Graph", "pack_weights", "forward", "forward_batched", "backward", "emd_loss",
           "compact_events", "logdiff", "contrast_events", "tnet_forward", "tnet_weight_floats", "autotune",
           "set_tile", "tile_count", "tile_name", "status_word", "lib", "EvsError", "LIB_PATH", "EXPORTED"]
