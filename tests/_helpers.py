"""Shared test helpers: oracle construction and GPU plan construction."""

import math

import numpy as np

from oracle import operator as op
from oracle import tables as tb
from vie_inputs import generators as gen


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def medium(kind: int, n: int, seed_item: int = 0, full: bool = False, sheared: bool = False):
    """(coef, mu, omega) of a small test problem of the given kind.  sheared:
    non-symmetric tensors (a rotation composed with a shear; for full Maxwell
    both eps and mu), so that H and H^T differ at every point of the bump."""
    rng = gen.rng_for(gen.CONFIG_IDS["test"], 100 + seed_item)
    if sheared:
        coef = gen.sheared_medium(n, rng)
        if kind == op.KIND_LAPLACE:
            return coef, None, 0.0
        mu = gen.sheared_medium(n, rng, norm=0.3) if full else None
        return coef, mu, 3.0 * math.pi
    if kind == op.KIND_LAPLACE:
        return gen.laplace_medium(n, rng), None, 0.0
    if kind == op.KIND_HELMHOLTZ:
        return gen.helmholtz_medium(n, rng), None, 3.0 * math.pi
    eps, mu = gen.maxwell_medium(n, rng)
    return eps, (mu if full else None), 3.0 * math.pi


def oracle_octant_tables(kind_sym: str, n: int, h: float, omega: float):
    """Oracle transform of the windowed kernel on the 2n grid at q in [0, n]^3,
    scaled by (2n)^-3, in the GPU's [qz][qy][entry][qx] order."""
    P = 2 * n
    idx = np.arange(-(n - 1), n) % P
    out = []
    for K in tb.kernel_tables(kind_sym, n, h, omega):
        Kp = np.zeros((P, P, P), dtype=np.complex128)
        Kp[np.ix_(idx, idx, idx)] = K
        out.append(np.fft.fftn(Kp)[: n + 1, : n + 1, : n + 1] / P ** 3)
    return np.stack(out, axis=2)  # [qz][qy][e][qx]
