"""FP64 CPU oracle for the contrastive-RL update.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU path is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path (the HIP
library and its Python binding) never does, and this package imports nothing
from the product path.  It is written from the paper, in the paper's order
and notation, with numpy in float64 and Python integers for the random
stream.
"""
from . import philox, relabel, replay, critic, objectives, adam  # noqa: F401
