"""FP64 CPU oracle of the EvSNet hot path -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously-correct reference that the HIP
path is checked against.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does, and
it shares no code with the HIP library (no kernels, headers, tables or
helpers).  It is written from the paper (arXiv 2508.18071):

* ``evsnet``  -- conv3x3 layers feeding bipolar LIF units (Sec. 3.3, Eq. 2-3),
  the surrogate-gradient BPTT backward (Eq. 4) with segment checkpointing,
  and teacher-forced one-step checks.
* ``emd``     -- the 1-D EMD as a difference of cumulative sums (Eq. 7), its
  bidirectional form (Eq. 8), the polarity split (Eq. 9) and the spike-count
  term (Eq. 10-11), with their (sub)gradients.
* ``prologue`` -- the network input of Eq. 1 (luminance, lin-log map, temporal
  difference) and contrast-crossing target events.
* ``tnet``    -- the paper's own temporal EvSNet (Sec. 3.3, Eq. 5-6): a
  kernel-7 Conv1d encoder with residual blocks, a point-wise projection and
  one BiLIF unit per pixel.

Every function is pinned by tests that do not re-type its formula: closed
forms, invariants, library special cases, brute force and finite
differences.  Nothing here is parity-unpinned.
"""

from . import evsnet, emd, prologue, tnet

__all__ = ["evsnet", "emd", "prologue", "tnet"]
