"""Windowed real-space kernel tables of the truncated-kernel method.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 5 describes the discretisation in three steps: (a) truncate the
kernel at the range of the computational box, (b) transform the truncated
kernel, (c) cut frequencies off at the resolution of the grid.  The readings
of the steps the paper leaves open (cut-off radius R, oversampling M, grid
placement, treatment of the Nyquist plane) are:

* R = sqrt(3) n h: the diameter of the box, so every pair of grid points is
  inside the truncation ball;
* frequencies s_k = 2 pi k / (M h), k in {-M/2, ..., M/2 - 1}^3 with M = 4n
  (a cube cut-off at |s_a| <= pi/h);
* on a plane k_a = -M/2 the sample is replaced by the average of the symbol
  over s_a = -pi/h and s_a = +pi/h (on edges and corners: over all sign
  choices of the Nyquist axes);
* the real-space kernel is the trapezoidal inverse transform
      K_m = M^{-3} sum_k F(s_k) exp(2 pi i k.m / M),   m in [-(n-1), n-1]^3,
  and the discrete convolution is U_a(i) = sum_b sum_j K^{ab}_{i-j} J_b(j).

Arrays are indexed [z][y][x]; symbol component (a, b) refers to vector
components x = 0, y = 1, z = 2.
"""

from __future__ import annotations

import itertools
import math
import os

import numpy as np
import scipy.fft

from . import symbol as sym

# scipy's pocketfft with every host core the process may use (capped at 16)
WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))


def fftn(a):
    return scipy.fft.fftn(a, workers=WORKERS)


def ifftn(a):
    return scipy.fft.ifftn(a, workers=WORKERS)


def default_R(n: int, h: float) -> float:
    return math.sqrt(3.0) * n * h


def default_M(n: int) -> int:
    return 4 * n


def freq_integers(M: int) -> np.ndarray:
    """k in FFT order: 0..M/2-1, -M/2..-1."""
    return np.fft.fftfreq(M, d=1.0 / M).round().astype(np.int64)


def sampled_symbol(kind: str, n: int, h: float, omega: float, R: float = None, M: int = None,
                   entries=None):
    """Samples of the symbol entries on the M^3 frequency grid, Nyquist planes averaged.

    Returns a list of complex arrays [M][M][M] in FFT order (only the listed
    entries when ``entries`` is given).
    """
    return list(iter_sampled_symbol(kind, n, h, omega, R, M, entries))


def iter_sampled_symbol(kind: str, n: int, h: float, omega: float, R: float = None, M: int = None,
                        entries=None):
    """Yields the sampled entries one at a time; G^(|s|) is evaluated once."""
    R = default_R(n, h) if R is None else R
    M = default_M(n) if M is None else M
    fn = sym.symbol_set(kind)
    nent = 3 if kind == "curl" else 6
    entries = list(range(nent)) if entries is None else list(entries)
    k = freq_integers(M)
    s1 = 2.0 * math.pi * k / (M * h)
    nyq1 = k == -(M // 2)
    SZ, SY, SX = np.meshgrid(s1, s1, s1, indexing="ij")
    g = sym.ghat(np.sqrt(SX * SX + SY * SY + SZ * SZ), omega, R)
    NZ, NY, NX = np.meshgrid(nyq1, nyq1, nyq1, indexing="ij")
    nyq = (NX, NY, NZ)
    scale = 1.0 / (2.0 ** (NX.astype(np.int64) + NY + NZ))
    # points on Nyquist planes, and the symbol there at every sign choice of those axes
    flips = []
    for r in (1, 2, 3):
        for T in itertools.combinations(range(3), r):
            mask = np.logical_and.reduce([nyq[a] for a in T])
            if mask.any():
                comp = [SX[mask].copy(), SY[mask].copy(), SZ[mask].copy()]
                for a in T:
                    comp[a] = -comp[a]          # -pi/h -> +pi/h
                flips.append((mask, comp))
    for e in entries:
        F = np.array(fn(SX, SY, SZ, omega, R, g=g, entries=[e])[0], dtype=np.complex128)
        for mask, comp in flips:
            F[mask] += fn(comp[0], comp[1], comp[2], omega, R, entries=[e])[0]
        F *= scale
        yield F


def window_indices(n: int, M: int) -> np.ndarray:
    return np.arange(-(n - 1), n) % M


def kernel_tables(kind: str, n: int, h: float, omega: float, R: float = None, M: int = None):
    """Windowed tables K_m, m in [-(n-1), n-1]^3, for every entry of the symbol set.

    Returns a list of arrays [(2n-1)]^3 indexed by m + n - 1 (axes z, y, x).
    """
    M = default_M(n) if M is None else M
    idx = window_indices(n, M)
    tabs = []
    for F in iter_sampled_symbol(kind, n, h, omega, R, M):   # one M^3 entry at a time
        K = ifftn(F)                     # M^{-3} sum_k F_k exp(+2 pi i k m / M)
        del F
        tabs.append(np.ascontiguousarray(K[np.ix_(idx, idx, idx)]))
        del K
    return tabs


def kernel_entry_direct(kind: str, index: int, m, n: int, h: float, omega: float,
                        R: float = None, M: int = None) -> complex:
    """K_m of one table entry by summing the definition term by term (no FFT)."""
    M = default_M(n) if M is None else M
    samples = sampled_symbol(kind, n, h, omega, R, M)[index]
    k = freq_integers(M).astype(np.float64)
    mz, my, mx = m
    ez = np.exp(2j * math.pi * k * mz / M)
    ey = np.exp(2j * math.pi * k * my / M)
    ex = np.exp(2j * math.pi * k * mx / M)
    phase = ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
    return complex(np.sum(samples * phase) / M ** 3)
