"""Potentials and fields after the solve: on the grid, at user points, far away.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

On the grid (the truncated-kernel discretisation of Section 5, as the
operator):
* phi_scat = div V_omega J (the summary of Section 3: F = V_omega J solves
  the vector problem and phi_scat = div F the anisotropic scalar one); its
  symbol is sum_b (i s_b G^) J^_b, the same vector i s G^ as the curl;
* H_scat = -i omega curl V_omega J for Maxwell with mu = I (eq.
  represent_Maxwell_reduced).

At points x away from the support of J, with the free-space kernel
G(r) = e^{i omega r} / (4 pi r) and the trapezoidal rule (weights h^3) over
the grid points y (this is the representation itself, not its truncated
discretisation):
* Laplace / Helmholtz: phi(x) = sum h^3 grad_x G(x - y) . J(y) and
  grad phi(x) = sum h^3 (grad grad G)(x - y) J(y);
* Maxwell (eq. represent_Maxwell): E = sum h^3 [(grad grad G + omega^2 G) J
  + i omega grad G x M], H = sum h^3 [(grad grad G + omega^2 G) M
  - i omega grad G x J].
Derivatives of G: G' = (i omega r - 1) e^{i omega r} / (4 pi r^2),
G'' = (2 - 2 i omega r - omega^2 r^2) e^{i omega r} / (4 pi r^3),
grad G = G' rh, grad grad G = G'' rh rh^T + (G' / r)(I - rh rh^T).

Far-field patterns (omega > 0), defined by f(r xh) = e^{i omega r} / r
f_inf(xh) + O(1/r^2): with J^(xh) = sum h^3 e^{-i omega xh.y} J(y),
phi_inf = (i omega / 4 pi) xh . J^, E_inf = (omega^2 / 4 pi) [(I - xh xh^T) J^
- xh x M^], H_inf = (omega^2 / 4 pi) [(I - xh xh^T) M^ + xh x J^].
"""

from __future__ import annotations

import math

import numpy as np

from . import operator as op
from . import tables as tb


def grid_points(n: int, h: float, origin):
    """Cell-centred coordinates x_i = origin + (i + 1/2) h, arrays [n][n][n] (z, y, x)."""
    c = [origin[a] + (np.arange(n) + 0.5) * h for a in range(3)]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    return X, Y, Z


def potential(J: np.ndarray, omega: float, h: float = None, R: float = None, M: int = None) -> np.ndarray:
    """phi_scat = div V_omega J on the grid: sum_b (i s_b G^) * J_b by window tables."""
    n = J.shape[-1]
    h = 2.0 / n if h is None else h
    conv = op.Convolver("curl", n, h, omega, "window", R=R, M=M)
    return sum(op.conv_fft_window_hat(conv.sym[b], J[b]) for b in range(3))


def field_h_reduced(J: np.ndarray, omega: float, h: float = None) -> np.ndarray:
    """H_scat = -i omega curl V_omega J on the grid (Maxwell, mu = I)."""
    n = J.shape[-1]
    h = 2.0 / n if h is None else h
    conv = op.Convolver("curl", n, h, omega, "window")
    W = np.zeros(J.shape, dtype=np.complex128)
    for (a, b, c), sgn in op.LEVI.items():
        W[a] += sgn * op.conv_fft_window_hat(conv.sym[b], J[c])
    return -1j * omega * W


def _green(r, omega):
    """(G, G', G'') of e^{i omega r} / (4 pi r) at r > 0."""
    e = np.exp(1j * omega * r) / (4.0 * math.pi)
    g = e / r
    g1 = (1j * omega * r - 1.0) * e / (r * r)
    g2 = (2.0 - 2j * omega * r - (omega * r) ** 2) * e / (r ** 3)
    return g, g1, g2


def fields_at(kind: int, density: np.ndarray, omega: float, points, h: float = None, origin=(-1.0, -1.0, -1.0)):
    """Scattered fields at points away from the support, by direct sums.

    Laplace / Helmholtz: [npts][4] = (phi, d_x phi, d_y phi, d_z phi);
    Maxwell: [npts][6] = (E, H) (density [3] for mu = I, [6] otherwise).
    """
    n = density.shape[-1]
    h = 2.0 / n if h is None else h
    X, Y, Z = grid_points(n, h, origin)
    w3 = h ** 3
    J = density[:3]
    Mv = density[3:] if density.shape[0] == 6 else None
    out = []
    for p in np.asarray(points, dtype=np.float64):
        d = (p[0] - X, p[1] - Y, p[2] - Z)
        r = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
        rh = [d[a] / r for a in range(3)]
        g, g1, g2 = _green(r, omega)

        def hess_dot(v):
            rv = rh[0] * v[0] + rh[1] * v[1] + rh[2] * v[2]
            return [(g2 - g1 / r) * rh[a] * rv + (g1 / r) * v[a] for a in range(3)]

        def grad_cross(v):  # grad G x v
            gr = [g1 * rh[a] for a in range(3)]
            return [gr[1] * v[2] - gr[2] * v[1], gr[2] * v[0] - gr[0] * v[2], gr[0] * v[1] - gr[1] * v[0]]

        if kind != op.KIND_MAXWELL:
            phi = np.sum(g1 * (rh[0] * J[0] + rh[1] * J[1] + rh[2] * J[2])) * w3
            gp = [np.sum(t) * w3 for t in hess_dot(J)]
            out.append([phi] + gp)
        else:
            HJ = hess_dot(J)
            E = [HJ[a] + omega ** 2 * g * J[a] for a in range(3)]
            Hf = [-1j * omega * t for t in grad_cross(J)]
            if Mv is not None:
                HM = hess_dot(Mv)
                CM = grad_cross(Mv)
                E = [E[a] + 1j * omega * CM[a] for a in range(3)]
                Hf = [Hf[a] + HM[a] + omega ** 2 * g * Mv[a] for a in range(3)]
            out.append([np.sum(t) * w3 for t in E] + [np.sum(t) * w3 for t in Hf])
    return np.array(out, dtype=np.complex128)


def far_field(kind: int, density: np.ndarray, omega: float, dirs, h: float = None, origin=(-1.0, -1.0, -1.0)):
    """Far-field patterns: Helmholtz [ndirs][1] = phi_inf; Maxwell [ndirs][6] = (E_inf, H_inf)."""
    n = density.shape[-1]
    h = 2.0 / n if h is None else h
    X, Y, Z = grid_points(n, h, origin)
    w3 = h ** 3
    out = []
    for xh in np.asarray(dirs, dtype=np.float64):
        ph = np.exp(-1j * omega * (xh[0] * X + xh[1] * Y + xh[2] * Z))
        Jh = np.array([np.sum(ph * density[a]) * w3 for a in range(3)])
        if kind != op.KIND_MAXWELL:
            out.append([1j * omega / (4.0 * math.pi) * np.dot(xh, Jh)])
            continue
        Mh = (np.array([np.sum(ph * density[3 + a]) * w3 for a in range(3)])
              if density.shape[0] == 6 else np.zeros(3, dtype=np.complex128))
        c = omega ** 2 / (4.0 * math.pi)
        E = c * (Jh - xh * np.dot(xh, Jh) - np.cross(xh, Mh))
        Hf = c * (Mh - xh * np.dot(xh, Mh) + np.cross(xh, Jh))
        out.append(list(E) + list(Hf))
    return np.array(out, dtype=np.complex128)
