"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package draws coordinates, values, initial parameters and epoch orders
from seeds. It holds no part of the SGD sweep: nothing here computes a
gradient, an update, a residual or a loss.
"""
from .gen import (  # noqa: F401
    Tensor, make_tensor, uniform_distinct, zipf_distinct, init_params,
    epoch_perm, planted_values, build,
)
from .configs import CONFIGS, Workload, get  # noqa: F401
