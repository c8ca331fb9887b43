"""Pins for the oracle's truncated-kernel transform (CPU only).

The transform G^(s) = (1/s) int_0^R e^{i omega r} sin(s r) dr of the kernel of
eqs. Vo / Vw cut off at r = R is checked against adaptive quadrature of that
integral (an independent route), including the removable singularities at
s = 0 and s = omega and the static limit omega = 2 pi 1e-50 used by the
paper's "size 1e-50" rows (Section 5, Tables 2-5).
"""

import math

import numpy as np
import pytest
from scipy import integrate

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")

from oracle import symbol as sym


def ghat_quadrature(s, omega, R):
    if s == 0.0:
        def f(r):
            return r * np.exp(1j * omega * r)
    else:
        def f(r):
            return np.exp(1j * omega * r) * math.sin(s * r) / s
    opts = dict(epsabs=1e-17, epsrel=1e-13, limit=800)
    re = integrate.quad(lambda r: f(r).real, 0.0, R, **opts)[0]
    im = integrate.quad(lambda r: f(r).imag, 0.0, R, **opts)[0]
    return complex(re, im)


@pytest.mark.parametrize("omega", [4 * math.pi, 8 * math.pi, 1.0, 1e-3])
@pytest.mark.parametrize("s_frac", [0.0, 0.08, 0.5, 0.999, 1.0, 1.001, 2.7, 9.0])
def test_ghat_matches_quadrature(omega, s_frac):
    R = 2.0 * math.sqrt(3.0)
    s = s_frac * omega if omega > 0.5 else s_frac * 10.0
    if 0 < s * R < 1e-2:
        pytest.skip("below the oracle's supported range")
    got = sym.ghat(np.array([s]), omega, R)[0]
    ref = ghat_quadrature(s, omega, R)
    assert abs(got - ref) <= 1e-11 * max(abs(ref), 1e-3)


def test_ghat_exact_resonance_is_finite():
    # s == omega exactly (samples land there on the configuration grids)
    R, omega = 2.0 * math.sqrt(3.0), 4 * math.pi
    got = sym.ghat(np.array([omega]), omega, R)[0]
    assert np.isfinite(got)
    assert abs(got - ghat_quadrature(omega, omega, R)) < 1e-12


@pytest.mark.parametrize("s", [0.0, 0.3, 1.7, 12.0, 55.0])
def test_laplace_limit_closed_form(s):
    # omega -> 0: G^ = 2 sin^2(sR/2)/s^2, G^(0) = R^2/2 (elementary integral of sin)
    R = 3.3
    ref = R * R / 2 if s == 0 else 2 * math.sin(s * R / 2) ** 2 / s ** 2
    # omega = 2 pi 1e-10 moves G^ by O(omega R) ~ 1e-9 relative
    for omega, tol in ((0.0, 1e-13), (2 * math.pi * 1e-50, 1e-13), (2 * math.pi * 1e-10, 1e-8)):
        got = sym.ghat(np.array([s]), omega, R)[0]
        assert abs(got - ref) <= tol * abs(ref) + 1e-15


def test_ghat_zero_series_branch_continuity():
    # both branches of G^(0) agree with quadrature near the switch at omega R = 1/2
    R = 2.0
    for wR in (1e-3, 0.49, 0.51, 3.0):
        omega = wR / R
        ref = ghat_quadrature(0.0, omega, R)
        assert abs(sym.ghat_zero(omega, R) - ref) < 1e-13 * abs(ref)


def test_phi1_series_and_direct_agree():
    z = np.array([0.99e-3j, 1.01e-3j, 0.5e-3 + 0.7e-3j])
    direct = np.expm1(z) / z
    assert np.allclose(sym.phi1(z), direct, rtol=1e-15, atol=0)


def test_symbol_parities():
    # grad-div entries: xy odd in s_x and s_y; curl entry b odd in s_b only
    rng = np.random.default_rng(1)
    s = rng.standard_normal(3) * 3
    for kind, fn in (("grad", sym.symbol_grad), ("D", sym.symbol_maxwell_D), ("curl", sym.symbol_curl)):
        base = fn(*[np.array([v]) for v in s], 4.0, 3.0)
        for axis in range(3):
            t = s.copy()
            t[axis] = -t[axis]
            flipped = fn(*[np.array([v]) for v in t], 4.0, 3.0)
            for e in range(len(base)):
                par = sym.parity(kind, e)[axis]
                assert np.allclose(flipped[e], par * base[e], rtol=1e-14, atol=0)
