"""Fourier transform of the truncated Green's function and the operator symbols.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Conventions: forward transform f^(s) = int f(x) exp(-i s.x) dx, so that a
derivative d/dx_a has symbol i s_a.

Truncated kernel (Section 5, step (a) of the truncated-kernel method): the
Helmholtz kernel exp(i omega r)/(4 pi r) of eq. Vw (omega = 0 gives the
Laplace kernel of eq. Vo) is cut off at r = R.  Its transform is radial:

    G^(s) = (1/s) int_0^R exp(i omega r) sin(s r) dr,         s = |s| > 0
    G^(0) = int_0^R r exp(i omega r) dr.

Writing sin(sr) = (e^{isr} - e^{-isr})/(2i) and phi1(z) = (e^z - 1)/z,

    G^(s) = R / (2 i s) * [phi1(i(omega + s)R) - phi1(i(omega - s)R)],

which is finite at s = omega.  G^(0) is [e^{i omega R}(1 - i omega R) - 1]/omega^2,
or its Taylor series sum_k (i omega)^k R^{k+2} / (k! (k+2)) when omega R < 1/2
(the closed form cancels catastrophically as omega R -> 0).

Operator symbols (eqs. Todef, Vw, represent_Maxwell):
    grad div V          :  F_ab = -s_a s_b G^
    (grad div + w^2) V  :  D_ab = (omega^2 delta_ab - s_a s_b) G^
    curl V              :  (C m)_a = sum_bc eps_abc (i s_b G^) m_c
"""

from __future__ import annotations

import math

import numpy as np

# symmetric 3x3 entries in storage order
SYM_ENTRIES = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def phi1(z):
    """(exp(z) - 1)/z, with its Taylor series for |z| < 1e-3."""
    z = np.asarray(z, dtype=np.complex128)
    out = np.empty_like(z)
    small = np.abs(z) < 1e-3
    zs = z[small]
    out[small] = 1.0 + zs / 2.0 + zs ** 2 / 6.0 + zs ** 3 / 24.0 + zs ** 4 / 120.0
    zl = z[~small]
    out[~small] = np.expm1(zl) / zl
    return out


def ghat_zero(omega: float, R: float) -> complex:
    """G^(0) = int_0^R r exp(i omega r) dr."""
    wR = omega * R
    if abs(wR) < 0.5:
        total = 0.0 + 0.0j
        term = 1.0 + 0.0j  # (i omega)^k / k!
        for k in range(24):
            total += term * R ** (k + 2) / (k + 2)
            term *= 1j * omega / (k + 1)
        return complex(total)
    e = complex(math.cos(wR), math.sin(wR))
    return complex((e * (1.0 - 1j * wR) - 1.0) / (omega * omega))


def ghat(s, omega: float, R: float) -> np.ndarray:
    """Transform of the truncated kernel at radial frequencies s >= 0."""
    s = np.asarray(s, dtype=np.float64)
    out = np.empty(s.shape, dtype=np.complex128)
    pos = s > 0
    sp = s[pos]
    if sp.size and np.min(sp) * R < 1e-2:
        raise ValueError("0 < s R < 1e-2 is not supported by the oracle (cancellation)")
    out[pos] = R / (2j * sp) * (phi1(1j * (omega + sp) * R) - phi1(1j * (omega - sp) * R))
    out[~pos] = ghat_zero(omega, R)
    return out


def _g(sx, sy, sz, omega, R, g):
    return ghat(np.sqrt(sx * sx + sy * sy + sz * sz), omega, R) if g is None else g


def symbol_grad(sx, sy, sz, omega: float, R: float, g=None, entries=None):
    """Entries (xx, yy, zz, xy, xz, yz) of -s s^T G^ (grad div V).

    g: G^(|s|) when already known; entries: indices of the entries wanted."""
    s = (sx, sy, sz)
    g = _g(sx, sy, sz, omega, R, g)
    idx = range(6) if entries is None else entries
    return [-(s[SYM_ENTRIES[e][0]] * s[SYM_ENTRIES[e][1]]) * g for e in idx]


def symbol_maxwell_D(sx, sy, sz, omega: float, R: float, g=None, entries=None):
    """Entries (xx, yy, zz, xy, xz, yz) of (omega^2 I - s s^T) G^."""
    s = (sx, sy, sz)
    g = _g(sx, sy, sz, omega, R, g)
    idx = range(6) if entries is None else entries
    out = []
    for e in idx:
        a, b = SYM_ENTRIES[e]
        out.append(((omega * omega if a == b else 0.0) - s[a] * s[b]) * g)
    return out


def symbol_curl(sx, sy, sz, omega: float, R: float, g=None, entries=None):
    """The vector i s_b G^ (b = x, y, z): curl V m has symbol (i s G^) x m."""
    s = (sx, sy, sz)
    g = _g(sx, sy, sz, omega, R, g)
    idx = range(3) if entries is None else entries
    return [1j * s[b] * g for b in idx]


def symbol_set(kind: str):
    """kind: 'grad' (Laplace, Helmholtz), 'D' (Maxwell), 'curl' (Maxwell)."""
    return {"grad": symbol_grad, "D": symbol_maxwell_D, "curl": symbol_curl}[kind]


# parity of each table entry in (s_x, s_y, s_z): +1 even, -1 odd
def parity(kind: str, index: int):
    if kind in ("grad", "D"):
        a, b = SYM_ENTRIES[index]
        p = [1, 1, 1]
        if a != b:
            p[a] = -1
            p[b] = -1
        return tuple(p)
    p = [1, 1, 1]
    p[index] = -1
    return tuple(p)
