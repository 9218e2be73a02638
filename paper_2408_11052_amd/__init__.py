"""MI355X-native contrastive-RL update hot path (HIP kernels behind a C ABI).

The compute lives in ``libcrl.so`` (built from ``csrc/`` by
``python -m paper_2408_11052_amd.build``); this package only marshals
arguments to it.  Importing the package does not load the library; the first
call does, and fails loudly if it has not been built.
"""
from ._lib import lib, CRLError, LIB_PATH  # noqa: F401
from .critic import (Critic, CriticLoss, crl_adam_step, crl_cast_bf16,  # noqa: F401
                     crl_check_finite, crl_counter_add, crl_peak_rate, crl_replay_insert,
                     crl_timing_enable, crl_timing_read, crl_timing_reset, make_config)
from .replay import ReplayRing  # noqa: F401
