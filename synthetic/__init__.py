"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package draws random numbers and evaluates the source fields the paper's
benchmark uses; it holds none of the solver's or the network's arithmetic.
"""
from .rhs import DriftingGaussians, RandomBlob, RandomDipoles, grid_coords, system_sizes_batched  # noqa: F401
from .params import fluid_net_params, guess_net_params  # noqa: F401
