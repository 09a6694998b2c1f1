"""MI355X-native FX correlation hot path of the MWAX correlator (Morrison et al. 2023).

The compute lives in ``libmwax.so`` (hand-written HIP for gfx950, C ABI in
``include/mwax.h``); :mod:`paper_2303_11557_amd.mwax` is its ctypes binding.
"""
from .mwax import (  # noqa: F401
    Config, Dims, MwaxError, Plan, derive, lib, make_config, pair_index,
    X_FP16, X_FP32, X_INT8, ORDER_CHAN_TRI, ORDER_TILE_BL, FAMILY_F, FAMILY_X, FAMILY_PACK,
)
