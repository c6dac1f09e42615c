"""FP64 CPU oracle for sparse FastTucker SGD (FastTuckerPlus, arXiv 2404.10087).

Test infrastructure: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use this package. It shares no code with the HIP library.
"""
from .oracle import (  # noqa: F401
    build, lib_path, use_library, predict, residual_stats, loss,
    factor_minibatch,
    factor_epoch, core_grad, core_epoch, set_threads,
)
