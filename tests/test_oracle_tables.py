"""Pins for the oracle's windowed kernel tables and convolution routes (CPU only).

* the table from the inverse FFT equals the defining sum
  K_m = M^{-3} sum_k F(s_k) e^{2 pi i k.m/M} evaluated term by term;
* direct O(n^6) sum == FFT on the 2n grid == FFT on the M grid (the three
  routes compute the same discrete operator exactly);
* the Gaussian closed forms of ``oracle.closed_forms`` (themselves checked
  against quadrature here) equal the discrete grad div V, (grad div + w^2) V
  and curl V applied to a sampled Gaussian to the accuracy the
  truncated-kernel method promises for resolved data (Section 5).
"""

import itertools
import math

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import operator as op
from oracle import tables as tb
from vie_inputs import generators as gen


@pytest.mark.parametrize("kind,omega", [("grad", 0.0), ("grad", 3.0), ("D", 5.0), ("curl", 5.0)])
def test_table_equals_defining_sum(kind, omega):
    n, h = 5, 0.4
    tabs = tb.kernel_tables(kind, n, h, omega)
    for m in [(0, 0, 0), (1, -2, 3), (-4, 4, -1), (4, 0, -4)]:
        for e in range(len(tabs)):
            ref = tb.kernel_entry_direct(kind, e, m, n, h, omega)
            got = tabs[e][m[0] + n - 1, m[1] + n - 1, m[2] + n - 1]
            assert abs(got - ref) <= 1e-13 * np.abs(tabs[e]).max()


@pytest.mark.parametrize("kind,omega", [("grad", 0.0), ("grad", 2.5), ("D", 2.5), ("curl", 2.5)])
def test_routes_agree(kind, omega):
    n, h = 6, 2.0 / 6
    tabs = tb.kernel_tables(kind, n, h, omega)
    F = tb.sampled_symbol(kind, n, h, omega)
    rng = np.random.default_rng(3)
    f = gen.random_density((n, n, n), rng)
    for e in range(len(tabs)):
        a = op.conv_direct(tabs[e], f)
        b = op.conv_fft_window(tabs[e], f)
        c = op.conv_fft_mgrid(F[e], f)
        assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)
        assert np.linalg.norm(a - c) <= 1e-13 * np.linalg.norm(a)


@pytest.mark.parametrize("kind,omega", [("grad", 0.0), ("grad", 2.5), ("D", 2.5)])
def test_vector_routes_agree(kind, omega):
    """The window route's vector apply (each component transformed once,
    U_a = crop IFFT(sum_b K^_ab J^_b)) equals the direct sum of every (a, b)
    pair; the same for the curl W_a = sum_bc eps_abc C_b * J_c."""
    n, h = 6, 2.0 / 6
    J = gen.random_density((3, n, n, n), np.random.default_rng(8))
    curl = kind == "D"
    win = op.Convolver(kind, n, h, omega, "window", with_curl=curl)
    dsum = op.Convolver(kind, n, h, omega, "direct", with_curl=curl)
    a, b = win.sym_apply(J), dsum.sym_apply(J)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)
    if curl:
        a, b = win.curl_apply(J), dsum.curl_apply(J)
        assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)


def test_direct_sum_at_single_point():
    n, h = 6, 1.0 / 3
    K = tb.kernel_tables("grad", n, h, 2.0)[3]
    f = gen.random_density((n, n, n), np.random.default_rng(4))
    full = op.conv_direct(K, f)
    for p in [(0, 0, 0), (5, 2, 1), (3, 5, 4)]:
        assert abs(op.conv_direct_at(K, f, p) - full[p]) < 1e-13 * np.abs(full).max()


@pytest.mark.parametrize("kind,omega", [("grad", 0.0), ("grad", 3.0), ("D", 3.0), ("curl", 3.0)])
def test_nyquist_samples_are_averages(kind, omega):
    """Reading of Section 5's cut-off: a sample on a plane k_a = -M/2 is the
    average of the symbol over s_a = -pi/h and s_a = +pi/h (edges: over the 4
    sign choices, the corner: over 8).  Evaluated point by point from the
    symbol functions (themselves pinned by quadrature), at plane, edge and
    corner samples; the entries odd in a Nyquist axis come out zero there."""
    from oracle import symbol as sym
    n, h = 5, 0.4
    M = tb.default_M(n)
    R = tb.default_R(n, h)
    F = tb.sampled_symbol(kind, n, h, omega)
    fn = sym.symbol_set(kind)
    ds = 2.0 * math.pi / (M * h)
    k = tb.freq_integers(M)
    nyq = M // 2                              # FFT index of k = -M/2
    cases = [(3, 7, nyq), (nyq, 2, 15), (11, nyq, 4),        # planes (z, y, x index)
             (nyq, nyq, 6), (1, nyq, nyq), (nyq, 9, nyq),    # edges
             (nyq, nyq, nyq)]                                  # corner
    for iz, iy, ix in cases:
        base = np.array([k[ix], k[iy], k[iz]], dtype=np.float64) * ds      # (s_x, s_y, s_z)
        axes = [a for a, i in enumerate((ix, iy, iz)) if i == nyq]
        ref = np.zeros(len(F), dtype=np.complex128)
        for signs in itertools.product((-1.0, 1.0), repeat=len(axes)):
            s = base.copy()
            for a, sg in zip(axes, signs):
                s[a] = sg * math.pi / h
            vals = fn(np.array([s[0]]), np.array([s[1]]), np.array([s[2]]), omega, R)
            ref += np.array([v[0] for v in vals])
        ref /= 2 ** len(axes)
        got = np.array([F[e][iz, iy, ix] for e in range(len(F))])
        mag = max(abs(v[0]) for v in fn(np.array([base[0]]), np.array([base[1]]), np.array([base[2]]),
                                        omega, R))
        assert np.allclose(got, ref, rtol=1e-14, atol=1e-14 * mag)
        par = [sym.parity(kind, e) for e in range(len(F))]
        for e in range(len(F)):
            if any(par[e][a] < 0 for a in axes):
                assert abs(got[e]) <= 1e-15 * mag
            else:
                # an even entry is unchanged by the averaging: F(-pi/h) itself
                s = base.copy()
                vals = fn(np.array([s[0]]), np.array([s[1]]), np.array([s[2]]), omega, R)
                assert abs(got[e] - vals[e][0]) <= 1e-14 * max(abs(vals[e][0]), 1e-300)


@pytest.mark.parametrize("kind", ["grad", "D", "curl"])
def test_table_parity(kind):
    # Nyquist averaging makes the samples symmetric, so K_{-m} = +-K_m exactly
    from oracle import symbol as sym
    n, h = 6, 1.0 / 3
    tabs = tb.kernel_tables(kind, n, h, 4.0)
    for e, K in enumerate(tabs):
        par = sym.parity(kind, e)
        for axis in range(3):
            flipped = np.flip(K, axis=2 - axis)      # vector axis x is array axis 2
            assert np.allclose(flipped, par[axis] * K, rtol=0, atol=1e-14 * np.abs(K).max())


def test_table_axis_permutation():
    # K^{xx}(m) with the x and y displacement swapped equals K^{yy}(m); same for xz/yz
    n, h = 6, 1.0 / 3
    t = tb.kernel_tables("grad", n, h, 3.0)
    xx, yy, zz, xy, xz, yz = t
    tol = 1e-14 * np.abs(xx).max()
    # array axes are (z, y, x): swapping vector x <-> y swaps array axes 2 <-> 1
    assert np.allclose(np.transpose(xx, (0, 2, 1)), yy, rtol=0, atol=tol)
    assert np.allclose(np.transpose(xx, (2, 1, 0)), zz, rtol=0, atol=tol)
    assert np.allclose(np.transpose(xz, (0, 2, 1)), yz, rtol=0, atol=tol)
    assert np.allclose(np.transpose(xy, (0, 2, 1)), xy, rtol=0, atol=tol)
    assert not np.allclose(np.transpose(xz, (1, 0, 2)), yz, rtol=0, atol=tol)


@pytest.mark.parametrize("r", [0.03, 0.2, 0.45, 0.9])
@pytest.mark.parametrize("omega", [0.0, 4 * math.pi, 8 * math.pi])
def test_gaussian_closed_form_matches_quadrature(r, omega):
    sigma = 0.15
    u = cf.gaussian_u_derivs(np.array([r]), sigma, omega)[0][0]
    q = cf.radial_potential_quadrature(r, sigma, omega)
    assert abs(u - q) <= 1e-12 * abs(q)


def test_gaussian_derivatives_by_finite_difference():
    # u', u'' of the closed form against central differences of u
    r = np.array([0.3, 0.6])
    for omega in (0.0, 4 * math.pi):
        d = 1e-4
        u0, up, upp = cf.gaussian_u_derivs(r, 0.15, omega)
        um = cf.gaussian_u_derivs(r - d, 0.15, omega)[0]
        uq = cf.gaussian_u_derivs(r + d, 0.15, omega)[0]
        assert np.allclose((uq - um) / (2 * d), up, rtol=1e-7)
        assert np.allclose((uq - 2 * u0 + um) / d ** 2, upp, rtol=1e-5)


@pytest.mark.parametrize("omega,tol", [(0.0, 5e-11), (4 * math.pi, 1e-10)])
def test_operator_matches_gaussian_closed_forms(omega, tol):
    n, sigma = 32, 0.15
    h = 2.0 / n
    X, Y, Z = gen.grid_coords(n)
    rho = gen.gaussian(n, sigma)
    hess = cf.gaussian_hessian(X, Y, Z, sigma, omega)
    u = cf.gaussian_potential(X, Y, Z, sigma, omega)
    for kind in ("grad", "D"):
        conv = op.Convolver(kind, n, h, omega, "window", with_curl=(kind == "D"))
        for b in range(3):
            J = np.zeros((3, n, n, n), dtype=np.complex128)
            J[b] = rho
            U = conv.sym_apply(J)
            ref = np.stack([hess[a, b] + (omega ** 2 * u if (kind == "D" and a == b) else 0.0)
                            for a in range(3)])
            assert np.linalg.norm(U - ref) <= tol * np.linalg.norm(ref)
        if kind == "D":
            for c in range(3):
                J = np.zeros((3, n, n, n), dtype=np.complex128)
                J[c] = rho
                cvec = np.eye(3)[c]
                ref = cf.gaussian_curl(X, Y, Z, sigma, omega, cvec)
                W = conv.curl_apply(J)
                assert np.linalg.norm(W - ref) <= tol * np.linalg.norm(ref)


@pytest.mark.slow
def test_operator_gaussian_superalgebraic_at_48():
    n, sigma, omega = 48, 0.11, 4 * math.pi
    X, Y, Z = gen.grid_coords(n)
    rho = gen.gaussian(n, sigma)
    hess = cf.gaussian_hessian(X, Y, Z, sigma, omega)
    conv = op.Convolver("grad", n, 2.0 / n, omega, "window")
    J = np.zeros((3, n, n, n), dtype=np.complex128)
    J[2] = rho
    U = conv.sym_apply(J)
    ref = hess[:, 2]
    assert np.linalg.norm(U - ref) <= 1e-13 * np.linalg.norm(ref)
