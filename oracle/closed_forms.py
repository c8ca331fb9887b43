"""Closed-form fields used to pin the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

1. Potential of a Gaussian density.  For rho(x) = exp(-|x|^2 / (2 sigma^2))
   the volume potential u = V_omega rho (eq. Vw; omega = 0 is eq. Vo) is
   radial, u = v(r)/r, with
     Laplace:   v  = sigma^3 sqrt(pi/2) erf(r / (sqrt2 sigma)),
                v' = sigma^2 exp(-r^2 / (2 sigma^2));
     Helmholtz: v  = (sigma^3/2) sqrt(pi/2) e^{-omega^2 sigma^2/2} [E+ - E-],
                v' = sigma^2 e^{-r^2/(2 sigma^2)} + i omega (sigma^3/2) sqrt(pi/2) e^{-omega^2 sigma^2/2} [E+ + E-],
                E+ = e^{i omega r} erfc(-(r + i omega sigma^2)/(sqrt2 sigma)),
                E- = e^{-i omega r} erfc((r - i omega sigma^2)/(sqrt2 sigma));
     both:      v'' = -omega^2 v - r rho   (the radial form of (Delta + omega^2) u = -rho).
   Derivatives: u' = v'/r - v/r^2, u'' = v''/r - 2v'/r^2 + 2v/r^3,
   d_a d_b u = u'' xh_a xh_b + (u'/r)(delta_ab - xh_a xh_b),  curl(u c) = u' xh x c.
   ``radial_potential_quadrature`` evaluates u(r) = (1/r) int_0^inf t rho(t)
   e^{i omega r_>} sin(omega r_<)/omega dt by adaptive quadrature, an
   independent check of these formulas.

2. Dielectric ball.  A ball of constant (anisotropic) eps in a uniform
   applied gradient E0 has the uniform interior field grad phi_tot =
   3 (eps + 2I)^{-1} E0 (depolarisation factor 1/3 of a sphere), the
   electrostatic problem of Section 2 with a piecewise-constant medium.
"""

from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special


def gaussian_v(r, sigma: float, omega: float):
    """(v, v', v'') of the radial potential u = v / r."""
    r = np.asarray(r, dtype=np.float64)
    rho = np.exp(-r * r / (2.0 * sigma * sigma))
    if omega == 0.0:
        v = sigma ** 3 * math.sqrt(math.pi / 2.0) * special.erf(r / (math.sqrt(2.0) * sigma))
        v = v.astype(np.complex128)
        vp = (sigma ** 2 * rho).astype(np.complex128)
    else:
        pref = 0.5 * sigma ** 3 * math.sqrt(math.pi / 2.0) * math.exp(-0.5 * (omega * sigma) ** 2)
        s2 = math.sqrt(2.0) * sigma
        Ep = np.exp(1j * omega * r) * special.erfc(-(r + 1j * omega * sigma ** 2) / s2)
        Em = np.exp(-1j * omega * r) * special.erfc((r - 1j * omega * sigma ** 2) / s2)
        v = pref * (Ep - Em)
        vp = sigma ** 2 * rho + 1j * omega * pref * (Ep + Em)
    vpp = -omega * omega * v - r * rho
    return v, vp, vpp


def gaussian_u_derivs(r, sigma: float, omega: float):
    """(u, u', u'') of u = V_omega rho at radii r > 0."""
    v, vp, vpp = gaussian_v(r, sigma, omega)
    u = v / r
    up = vp / r - v / r ** 2
    upp = vpp / r - 2.0 * vp / r ** 2 + 2.0 * v / r ** 3
    return u, up, upp


def radial_potential_quadrature(r: float, sigma: float, omega: float) -> complex:
    """u(r) = (1/r) int_0^inf t rho(t) G_rad(r, t) dt by adaptive quadrature."""
    def kern(t):
        lo, hi = min(r, t), max(r, t)
        if omega == 0.0:
            return lo
        return np.exp(1j * omega * hi) * math.sin(omega * lo) / omega

    def f_re(t):
        return (t * math.exp(-t * t / (2 * sigma * sigma)) * kern(t)).real

    def f_im(t):
        return complex(t * math.exp(-t * t / (2 * sigma * sigma)) * kern(t)).imag

    top = 12.0 * sigma + r
    re = integrate.quad(f_re, 0.0, r, epsabs=0, epsrel=1e-13, limit=200)[0] + \
        integrate.quad(f_re, r, top, epsabs=0, epsrel=1e-13, limit=200)[0]
    im = integrate.quad(f_im, 0.0, r, epsabs=0, epsrel=1e-13, limit=200)[0] + \
        integrate.quad(f_im, r, top, epsabs=0, epsrel=1e-13, limit=200)[0]
    return complex(re, im) / r


def gaussian_hessian(X, Y, Z, sigma: float, omega: float, center=(0.0, 0.0, 0.0)):
    """d_a d_b u at the points, returned as [3][3][...] complex."""
    dx, dy, dz = X - center[0], Y - center[1], Z - center[2]
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    _, up, upp = gaussian_u_derivs(r, sigma, omega)
    xh = (dx / r, dy / r, dz / r)
    out = np.empty((3, 3) + r.shape, dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            out[a, b] = upp * xh[a] * xh[b] + (up / r) * ((1.0 if a == b else 0.0) - xh[a] * xh[b])
    return out


def gaussian_potential(X, Y, Z, sigma: float, omega: float, center=(0.0, 0.0, 0.0)):
    dx, dy, dz = X - center[0], Y - center[1], Z - center[2]
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    u, _, _ = gaussian_u_derivs(r, sigma, omega)
    return u


def gaussian_curl(X, Y, Z, sigma: float, omega: float, c, center=(0.0, 0.0, 0.0)):
    """curl(u c) = u' xh x c for a constant vector c, as [3][...]."""
    dx, dy, dz = X - center[0], Y - center[1], Z - center[2]
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    _, up, _ = gaussian_u_derivs(r, sigma, omega)
    xh = np.stack([dx / r, dy / r, dz / r])
    cr = np.cross(xh, np.asarray(c, dtype=np.float64)[:, None, None, None], axis=0)
    return up[None] * cr


def sphere_interior_field(eps_const: np.ndarray, E0) -> np.ndarray:
    """3 (eps + 2I)^{-1} E0."""
    return 3.0 * np.linalg.solve(np.asarray(eps_const) + 2.0 * np.eye(3), np.asarray(E0, dtype=np.complex128))
