"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package draws random numbers and lays arrays out; it contains none of the
solver's arithmetic, so both the CPU oracle and the HIP path may consume its arrays.
"""

from .gen import *  # noqa: F401,F403
