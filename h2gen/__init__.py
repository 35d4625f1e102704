"""Seeded synthetic inputs: points, kernels, cluster trees, H^2 construction, blob files.

Both the oracle and the GPU path consume what this package produces; it
contains no factorization or solve arithmetic.
"""
