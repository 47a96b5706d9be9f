"""MI355X-native (gfx950) PDE signature kernel.

Hot path of Salvi et al., "The Signature Kernel is the solution of a Goursat
PDE" (arXiv 2006.14794), Section 3.1: increment inner products of two
piecewise-linear paths, their dyadic refinement, and the explicit
finite-difference sweep of the Goursat problem to the terminal corner -- as
hand-written HIP kernels behind a C ABI (include/sigkernel.h).  This package
is the thin Python binding; it never computes anything on the CPU.
"""
from ._lib import SK_NO_DIAG, SK_SYMMETRIC, SigKernelError, load, status_string, version
from .api import (RaggedPaths, SigKernelGram, SigKernelGramSymmetric, SigKernelMMD2, gram, mmd2,
                  sigkernel_gram, sigkernel_gram_backward, sigkernel_increment_gram, sigkernel_mmd2,
                  sigkernel_gram_lifted, sigkernel_pair, sigkernel_pair_lifted,
                  reduced_measure, reduced_measure_support, workspace_bytes)
from . import corrector
from .corrector import Corrector
from .graph import CapturedCalls, capture_gram, capture_mmd2, capture_pair
from .tuning import autotune, load_cache, save_cache, tune_clear, tune_get, tune_key, tune_list, tune_set

__all__ = [
    "RaggedPaths", "SigKernelError", "SigKernelGram", "SigKernelGramSymmetric", "gram", "load",
    "SigKernelMMD2", "mmd2", "sigkernel_mmd2", "sigkernel_increment_gram",
    "sigkernel_gram", "sigkernel_gram_backward", "sigkernel_pair",
    "sigkernel_gram_lifted", "sigkernel_pair_lifted",
    "reduced_measure", "reduced_measure_support",
    "status_string", "version", "workspace_bytes",
    "SK_SYMMETRIC", "SK_NO_DIAG",
    "Corrector", "corrector",
    "CapturedCalls", "capture_gram", "capture_mmd2", "capture_pair",
    "autotune", "load_cache", "save_cache", "tune_clear", "tune_get", "tune_key", "tune_list",
    "tune_set",
]
