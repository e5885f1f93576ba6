"""MI355X-native kernel-independent FMM for 3D elastostatics (Kelvin kernels) and the BEM it drives.

The compute path is the HIP library ``libkfmm.so`` (C ABI in ``include/kfmm.h``); this package only
marshals torch tensors (device memory, streams) into that ABI.
"""
from .kfmm import (  # noqa: F401
    DISP, STRESS, FP64, FP32, FP32_M2L_BF16, KfmmError, FmmOpts, FmmPlan, load_library, moduli,
)
