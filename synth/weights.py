"""He-initialised conv3x3 weights (inputs only).

Layer l gets W ~ N(0, 2 / (Cin * 9)) of shape [Cout][Cin][3][3], drawn layer
by layer from numpy's default_rng(seed) in float64 and rounded to float32.
The weights are inputs to both the oracle and the HIP path.
"""

from __future__ import annotations

import numpy as np


def he_weights(channels, seed: int = 0):
    rng = np.random.default_rng(seed)
    ws = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        std = np.sqrt(2.0 / (cin * 9))
        ws.append(rng.normal(0.0, std, size=(cout, cin, 3, 3)).astype(np.float32))
    return ws
