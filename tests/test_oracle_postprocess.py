"""Pins of oracle/postprocess.py against closed forms (CPU).

For J = c rho with the Gaussian rho = exp(-|x - x0|^2 / (2 sigma^2)) and a
constant vector c, u = V_omega rho is radial (closed_forms.gaussian_*), so
  div V J = c . grad u = u' (rh . c),       grad div V J = (Hess u) c,
  E = (Hess u) c + omega^2 u c,             curl V J = u' rh x c,
and the far field involves rho^(k) = (2 pi sigma^2)^{3/2} exp(-sigma^2 |k|^2 / 2)
exp(-i k . x0).  The grid sums are trapezoidal rules of a Gaussian that is
1e-12 at the box faces: spectrally accurate.
"""

import math

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import operator as op
from oracle import postprocess as pp

N = 32
SIGMA = 0.12
X0 = np.array([0.1, -0.05, 0.0])
C = np.array([0.3, -0.7, 0.5 + 0.2j])


def density(n=N, half="J"):
    X, Y, Z = pp.grid_points(n, 2.0 / n, (-1.0, -1.0, -1.0))
    rho = np.exp(-((X - X0[0]) ** 2 + (Y - X0[1]) ** 2 + (Z - X0[2]) ** 2) / (2 * SIGMA ** 2))
    J = np.stack([C[a] * rho for a in range(3)])
    if half == "J":
        return J
    z = np.zeros_like(J)
    return np.concatenate([J, z]) if half == "JM_J" else np.concatenate([z, J])


def closed(points, omega):
    """(u, u', Hess u, rh) at the points."""
    d = np.asarray(points) - X0
    r = np.linalg.norm(d, axis=1)
    u, up, upp = cf.gaussian_u_derivs(r, SIGMA, omega)
    rh = d / r[:, None]
    hess = np.einsum("p,pa,pb->pab", upp - up / r, rh, rh) + (up / r)[:, None, None] * np.eye(3)[None]
    return u, up, hess, rh


POINTS = np.array([[2.0, 0.3, -0.4], [-1.5, -1.2, 0.8], [0.2, 2.5, 1.1], [-0.3, 0.1, -3.0]])


@pytest.mark.parametrize("kind,omega", [(op.KIND_LAPLACE, 0.0), (op.KIND_HELMHOLTZ, 3 * math.pi)])
def test_scalar_fields_at_points(kind, omega):
    got = pp.fields_at(kind, density(), omega, POINTS)
    u, up, hess, rh = closed(POINTS, omega)
    phi = up * (rh @ C)
    grad = np.einsum("pab,b->pa", hess, C)
    assert np.max(np.abs(got[:, 0] - phi)) < 1e-9 * np.max(np.abs(phi))
    assert np.max(np.abs(got[:, 1:] - grad)) < 1e-9 * np.max(np.abs(grad))


@pytest.mark.parametrize("half", ["J", "JM_J", "JM_M"])
def test_maxwell_fields_at_points(half):
    omega = 3 * math.pi
    got = pp.fields_at(op.KIND_MAXWELL, density(half=half), omega, POINTS)
    u, up, hess, rh = closed(POINTS, omega)
    D = np.einsum("pab,b->pa", hess, C) + omega ** 2 * u[:, None] * C[None]   # (grad div + omega^2) V (c rho)
    Cu = up[:, None] * np.cross(rh, C[None])                                   # curl V (c rho)
    if half in ("J", "JM_J"):
        E, H = D, -1j * omega * Cu
    else:
        E, H = 1j * omega * Cu, D
    ref = np.concatenate([E, H], axis=1)
    assert np.max(np.abs(got - ref)) < 1e-9 * np.max(np.abs(ref))


def far_closed(dirs, omega):
    k = omega * np.asarray(dirs)
    rho_hat = (2 * math.pi * SIGMA ** 2) ** 1.5 * np.exp(-0.5 * SIGMA ** 2 * omega ** 2) * np.exp(-1j * k @ X0)
    return rho_hat


DIRS = np.array([[1.0, 0, 0], [0, 0.6, 0.8], [-0.48, 0.6, -0.64]])


def test_far_field_closed_forms():
    omega = 3 * math.pi
    rho_hat = far_closed(DIRS, omega)
    got = pp.far_field(op.KIND_HELMHOLTZ, density(), omega, DIRS)
    ref = 1j * omega / (4 * math.pi) * (DIRS @ C) * rho_hat
    assert np.max(np.abs(got[:, 0] - ref)) < 1e-10 * np.max(np.abs(ref))
    got = pp.far_field(op.KIND_MAXWELL, density(), omega, DIRS)
    c = omega ** 2 / (4 * math.pi)
    E = c * rho_hat[:, None] * (C[None] - DIRS * (DIRS @ C)[:, None])
    H = c * rho_hat[:, None] * np.cross(DIRS, C[None])
    ref = np.concatenate([E, H], axis=1)
    assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("kind", [op.KIND_HELMHOLTZ, op.KIND_MAXWELL])
def test_far_field_is_the_limit_of_the_field(kind):
    """r e^{-i omega r} f(r xh) -> f_inf(xh), with an O(1/r) remainder."""
    omega = 3 * math.pi
    J = density()
    inf = pp.far_field(kind, J, omega, DIRS)
    for r in (1e3, 1e4):
        near = pp.fields_at(kind, J, omega, r * DIRS)
        f = near[:, :1] if kind != op.KIND_MAXWELL else near
        lim = r * np.exp(-1j * omega * r) * f
        assert np.max(np.abs(lim - inf)) < 20.0 / r * np.max(np.abs(inf))


def test_potential_on_grid_closed_form():
    omega = 3 * math.pi
    phi = pp.potential(density(), omega)
    X, Y, Z = pp.grid_points(N, 2.0 / N, (-1.0, -1.0, -1.0))
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    u, up, hess, rh = closed(pts, omega)
    ref = (up * (rh @ C)).reshape(N, N, N)
    # the truncated-kernel discretisation at 32^3 (not a rounding-level identity)
    assert np.max(np.abs(phi - ref)) < 5e-9 * np.max(np.abs(ref))


def test_reduced_maxwell_h_on_grid_closed_form():
    omega = 3 * math.pi
    H = pp.field_h_reduced(density(), omega)
    X, Y, Z = pp.grid_points(N, 2.0 / N, (-1.0, -1.0, -1.0))
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    u, up, hess, rh = closed(pts, omega)
    ref = (-1j * omega * up[:, None] * np.cross(rh, C[None])).T.reshape(3, N, N, N)
    assert np.max(np.abs(H - ref)) < 5e-9 * np.max(np.abs(ref))
