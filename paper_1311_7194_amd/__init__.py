"""Block-sparse TSDF fusion and raycasting for AMD Instinct MI355X (gfx950).

The compute path is libtsdf.so (hand-written HIP kernels behind a C ABI,
``include/tsdf.h``); this package is its thin Python binding over torch
device tensors.
"""

from .tsdf import (  # noqa: F401
    F16, F32, NOISE_CONSTANT, NOISE_MLP, NOISE_QUADRATIC, RULE_KALMAN, RULE_RUNNING, RULE_WEIGHTED,
    WEIGHT_CONSTANT, WEIGHT_INV_VARIANCE, Batch, Icp, TsdfError, Volume, lib, LIB_PATH,
)
