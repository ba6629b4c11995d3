"""Seeded synthetic exposure stacks shaped like the paper's workloads.

This module is shared by the tests, the benchmark and the smoke check. It
holds only scene synthesis (Gaussian blobs, texture, a planted homography,
planted per-tile integer shifts, exposure scaling, sensor noise): none of the
registration method's arithmetic lives here, so neither the CPU oracle nor the
GPU path depends on the other through it.
"""
from .scenes import (  # noqa: F401
    Frame,
    Stack,
    make_pair,
    make_stack,
    make_config_pair,
    make_batch_pair,
    make_sweep_pair,
    SWEEP_SIZES,
    make_planted_shift_pair,
    make_texture,
    CONFIGS,
)
from .proposal import proposal_params, N_PARAMS  # noqa: F401
