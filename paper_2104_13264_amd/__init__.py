"""MI355X (gfx950) tensor-network Metropolis-Hastings sampler for 2D Ising
and q-state Potts models (arXiv:2104.13264): boundary-MPS environments,
sequential proposals with their log-probability, MH acceptance and d ln Z~ / dJ,
as HIP kernels behind the C ABI of include/tnmh.h.
"""
from .tnmh import (BF16, FP32, FP64, FP64_MFMA, PREC, LogZ, Sampler, TNError, exported_symbols, lib,
                   log_z, LIB_PATH, PEAK_KINDS, peak_probe)

__all__ = ["Sampler", "TNError", "LogZ", "log_z", "FP64", "FP32", "BF16", "FP64_MFMA", "PREC", "lib",
           "LIB_PATH", "exported_symbols", "PEAK_KINDS", "peak_probe"]
