"""MI355X-native hybrid-snapshot adaptive ROM step (arXiv 2301.01718).

The computational path is the HIP library ``libhsrom.so`` (C ABI in
``include/hsrom.h``); this package is its thin Python binding, the
Algorithm-1 driver that sequences the calls, and the checkpointed trajectory
adjoint (``paper_2301_01718_amd.adjoint``).
"""
from ._lib import (Context, Samples, Tape, HsError, hybrid_params, lib, exported_symbols,  # noqa: F401
                   BURGERS_1D, BURGERS_2D, EULER_2D, FP64, MIXED_FP32, RULE_FRACTION, RULE_RRE,
                   TAPE_RECORD, TAPE_REPLAY, BASIS_PENDING, PAPER_BC_FIXED, PAPER_BC_WALL, PaperHDM, paper_hdm)
