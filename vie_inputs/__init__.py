"""Seeded synthetic inputs for the volume-integral-equation solver.

This module is shared by the CPU oracle (test infrastructure) and the GPU
harness.  It produces *inputs only*: grid coordinates, medium tensors
eps(x) / eps^{-1}(x) / mu(x), incident fields and random densities.  It holds
none of the method's arithmetic (no contrast, no kernel, no convolution).
"""

from .generators import *  # noqa: F401,F403
