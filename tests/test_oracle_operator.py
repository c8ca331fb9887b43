"""Pins for the oracle's contrast, matvec and solves (CPU only).

Each test checks the oracle against a fact fixed by the paper or by the
mathematics, chosen so that a plausible mistake (sign, transposed operand,
dropped term, wrong index) fails at least one of them:

* Lemma 1: ||H(x)||_2 < 1 for the media of the configurations;
* Lemma 2 (proof): 2 T_0 maps gradients g to -g and divergence-free fields to
  themselves, i.e. grad div V_0 grad(rho) = -grad(rho), grad div V_0 curl = 0;
* bilinear symmetry x^T K y = y^T K x and equivariance under axis
  permutations and reflections of the cell-centred cube;
* omega -> 0 (the paper's "size 1e-50" rows): Helmholtz = Laplace, reduced
  Maxwell = Laplace;
* eps = I gives J = 0 and the incident field;
* dense LU == GMRES == Bi-CGStab == Neumann series (Laplace, eq. intLap);
* manufactured solution from the Gaussian closed forms;
* dielectric ball: interior field 3 (eps + 2I)^{-1} E0 to first order in h,
  and the "+" sign printed in eq. intH fails this test while "-" passes;
* full Maxwell duality (eq. intM): solve(mu, eps, H_inc, -E_inc) = (M, -J).
"""

import math

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import operator as op
from oracle import solve as sv
from vie_inputs import generators as gen


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ----------------------------------------------------------------------------
# contrast
# ----------------------------------------------------------------------------

def test_contrast_diagonal_closed_form():
    n = 4
    a = np.array([0.5, 2.0, 3.0 + 0.2j])
    coef = gen.tensor_field(0.0, np.ones((n, n, n)), np.diag(a))
    H = op.contrast(coef).reshape(3, 3, n, n, n)
    for i in range(3):
        assert np.allclose(H[i, i], (a[i] - 1) / (a[i] + 1), rtol=1e-15)
        for j in range(3):
            if i != j:
                assert np.all(H[i, j] == 0)


def test_contrast_rotation_covariant():
    rng = np.random.default_rng(5)
    Q = gen.random_rotation(rng)
    d = np.array([0.7, 1.9, 2.6])
    n = 2
    coef = gen.tensor_field(0.0, np.ones((n, n, n)), Q @ np.diag(d) @ Q.T)
    H = op.contrast(coef).reshape(3, 3, -1)[:, :, 0]
    assert np.allclose(H, Q @ np.diag((d - 1) / (d + 1)) @ Q.T, atol=1e-15)


def shear_field(n):
    """a = I + e_x e_y^T at every point: the hand-computed contrast (eq. rhodef) is
    H = (a + I)^{-1}(a - I) = [[1/2, -1/4, 0], [0, 1/2, 0], [0, 0, 1/2]] e_x e_y^T
      = (1/2) e_x e_y^T,
    so H v = (v_y / 2, 0, 0) while H^T v = (0, v_x / 2, 0)."""
    a = np.eye(3)
    a[0, 1] = 1.0
    return gen.tensor_field(0.0, np.ones((n, n, n)), a.astype(np.complex128))


def test_contrast_orientation_hand_computed():
    n = 6
    H = op.contrast(shear_field(n))
    want = np.zeros((3, 3))
    want[0, 1] = 0.5
    assert np.array_equal(H.reshape(3, 3, -1)[:, :, 17], want)
    v = np.zeros((3, n, n, n), dtype=np.complex128)
    v[1] = 2.0 - 4.0j                        # v = (0, 2 - 4i, 0)
    v[0] = 1.0                               # ... + (1, 0, 0): H^T would pick this one
    Hv = op.pointwise(H, v)
    assert np.array_equal(Hv[0], np.full((n, n, n), 1.0 - 2.0j))
    assert np.array_equal(Hv[1], np.zeros((n, n, n))) and np.array_equal(Hv[2], np.zeros((n, n, n)))


@pytest.mark.parametrize("kind,full", [(op.KIND_LAPLACE, False), (op.KIND_HELMHOLTZ, False),
                                       (op.KIND_MAXWELL, False), (op.KIND_MAXWELL, True)])
def test_operator_orientation_of_contrast(kind, full):
    """With H = (1/2) e_x e_y^T, A J = J - H (J + 2 U) leaves the y and z
    components of J untouched and changes x by -(J_y + 2 U_y)/2; the right-hand
    side 2 H g is (g_y, 0, 0).  Full Maxwell: the same for the M half with
    H_mu = (1/2) e_x e_y^T."""
    n = 8
    coef = shear_field(n)
    omega = 0.0 if kind == op.KIND_LAPLACE else 2.0
    A = op.Operator(kind, coef, omega, mu=coef if full else None)
    c = 6 if full else 3
    x = gen.random_density((c, n, n, n), np.random.default_rng(11))
    y = A.apply(x)
    Z = A.field(x, np.zeros_like(x)) if full else A.conv.sym_apply(x)
    for h in range(c // 3):
        J, Y, U = x[3 * h:3 * h + 3], y[3 * h:3 * h + 3], Z[3 * h:3 * h + 3]
        assert np.array_equal(Y[1], J[1]) and np.array_equal(Y[2], J[2])
        assert rel(Y[0], J[0] - 0.5 * (J[1] + 2.0 * U[1])) < 1e-15
    g = gen.random_density((c, n, n, n), np.random.default_rng(12))
    b = A.rhs(g)
    for h in range(c // 3):
        assert np.array_equal(b[3 * h], g[3 * h + 1])
        assert not b[3 * h + 1].any() and not b[3 * h + 2].any()


def _field_of(mats):
    """[9][n][1][1] field holding one 3x3 matrix per x point."""
    m = np.stack(mats, axis=-1)              # [3][3][n]
    return m.reshape(9, 1, 1, -1).astype(np.complex128)


def test_contrast_norm_is_spectral_norm():
    """Lemma 1 is stated for ||H(x)||_2.  For normal H (unitarily
    diagonalisable) the norm is max |lambda|; for the nilpotent (1/2) e_x e_y^T
    it is 1/2 although every eigenvalue is 0; for a rank-one u v^H it is
    |u| |v|.  The largest entry, the Frobenius norm or the spectral radius
    each fail at least one of these."""
    rng = np.random.default_rng(21)
    g = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    U, _ = np.linalg.qr(g)                   # unitary
    lam = np.array([0.3 * np.exp(0.4j), -0.7, 0.55j])
    normal = U @ np.diag(lam) @ U.conj().T
    assert abs(op.contrast_norm_max(_field_of([normal])) - 0.7) < 1e-14
    nil = np.zeros((3, 3))
    nil[0, 1] = 0.5
    assert abs(op.contrast_norm_max(_field_of([nil])) - 0.5) < 1e-15
    u = np.array([0.3, 0.4j, 0.0])
    v = np.array([0.6, 0.0, 0.8j])
    assert abs(op.contrast_norm_max(_field_of([np.outer(u, v.conj())])) - 0.5) < 1e-15
    # the maximum over points
    assert abs(op.contrast_norm_max(_field_of([nil, normal, 0.1 * np.eye(3)])) - 0.7) < 1e-14


def test_lemma1_accretive_and_not():
    """H = (a + I)^{-1}(a - I) is a contraction exactly when the Hermitian part
    of a is positive definite (Lemma 1's hypothesis): a sheared non-symmetric
    medium passes; a tensor with an indefinite Hermitian part does not."""
    n = 10
    c = gen.sheared_medium(n, gen.rng_for(gen.CONFIG_IDS["test"], 3))
    assert op.contrast_norm_max(op.contrast(c)) < 1.0
    a = np.array([[1.0, 3.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])   # a + a^T indefinite
    assert op.contrast_norm_max(op.contrast(_field_of([a]))) > 1.0


@pytest.mark.parametrize("name", ["laplace", "helmholtz", "maxwell"])
def test_lemma1_contrast_is_contraction(name):
    n = 20
    if name == "laplace":
        coefs = [gen.laplace_medium(n, gen.rng_for(1, 0))]
    elif name == "helmholtz":
        coefs = [gen.helmholtz_medium(n, gen.rng_for(2, 0))]
    else:
        coefs = list(gen.maxwell_medium(n, gen.rng_for(3, 0)))
    for c in coefs:
        assert op.contrast_norm_max(op.contrast(c)) < 1.0


# ----------------------------------------------------------------------------
# operator identities
# ----------------------------------------------------------------------------

def test_lemma2_reflection_of_gradients_and_curls():
    n, sigma = 32, 0.15
    X, Y, Z = gen.grid_coords(n)
    rho = gen.gaussian(n, sigma)
    conv = op.Convolver("grad", n, 2.0 / n, 0.0, "window")
    grad = np.stack([-(X / sigma ** 2) * rho, -(Y / sigma ** 2) * rho, -(Z / sigma ** 2) * rho]).astype(complex)
    U = conv.sym_apply(grad)
    assert rel(grad + 2 * U, -grad) < 1e-9           # 2 T0 grad = -grad (resolution-limited)
    # curl(rho e_z) = (d_y rho, -d_x rho, 0) is divergence free: 2 T0 J = J
    curl = np.stack([grad[1], -grad[0], np.zeros_like(rho)]).astype(complex)
    U = conv.sym_apply(curl)
    assert np.linalg.norm(U) < 1e-10 * np.linalg.norm(curl)


@pytest.mark.parametrize("kind", ["grad", "D", "curl"])
def test_bilinear_symmetry(kind):
    n = 7
    conv = op.Convolver("D" if kind == "curl" else kind, n, 2.0 / n, 3.0, "window", with_curl=True)
    rng = np.random.default_rng(11)
    x = gen.random_density((3, n, n, n), rng)
    y = gen.random_density((3, n, n, n), rng)
    f = conv.curl_apply if kind == "curl" else conv.sym_apply
    a = np.sum(x * f(y))
    b = np.sum(y * f(x))
    assert abs(a - b) < 1e-13 * abs(a)


def test_equivariance_permutation_and_reflection():
    n = 8
    conv = op.Convolver("D", n, 2.0 / n, 4.0, "window", with_curl=True)
    rng = np.random.default_rng(12)
    J = gen.random_density((3, n, n, n), rng)
    U = conv.sym_apply(J)
    W = conv.curl_apply(J)
    # swap vector components x <-> y and array axes x <-> y
    Jp = np.transpose(J[[1, 0, 2]], (0, 1, 3, 2))
    assert rel(conv.sym_apply(Jp), np.transpose(U[[1, 0, 2]], (0, 1, 3, 2))) < 1e-13
    # a swap is orientation reversing: the curl changes sign
    assert rel(conv.curl_apply(Jp), -np.transpose(W[[1, 0, 2]], (0, 1, 3, 2))) < 1e-13
    # reflect x -> -x: index i -> n-1-i and the x component flips
    def refl(v):
        out = np.flip(v, axis=3).copy()
        out[0] = -out[0]
        return out
    assert rel(conv.sym_apply(refl(J)), refl(U)) < 1e-13
    # curl of a reflected field is minus the reflected curl (pseudo-vector)
    assert rel(conv.curl_apply(refl(J)), -refl(W)) < 1e-13


def test_static_limits():
    n = 8
    coef = gen.laplace_medium(n, gen.rng_for(7, 1))
    x = gen.random_density((3, n, n, n), np.random.default_rng(13))
    lap = op.Operator(op.KIND_LAPLACE, coef, 0.0).apply(x)
    # size 1e-50: identical to Laplace to rounding; size 1e-10: the first-order
    # term i omega R is ~1e-9 relative in the kernel and still below the rows' digits
    for w, tol in ((2 * math.pi * 1e-50, 1e-14), (2 * math.pi * 1e-10, 1e-9)):
        hel = op.Operator(op.KIND_HELMHOLTZ, coef, w).apply(x)
        mxr = op.Operator(op.KIND_MAXWELL, coef, w).apply(x)
        assert rel(hel, lap) < tol
        assert rel(mxr, lap) < tol


def test_identity_medium():
    n = 8
    coef = gen.identity_field(n)
    A = op.Operator(op.KIND_HELMHOLTZ, coef, 3.0)
    inc = gen.plane_wave_gradient(n, 3.0, np.array([0.0, 0.6, 0.8]))
    b = A.rhs(inc)
    assert np.all(b == 0)
    x = gen.random_density((3, n, n, n), np.random.default_rng(2))
    assert np.allclose(A.apply(x), x, rtol=0, atol=0)
    assert np.allclose(A.field(np.zeros_like(inc), inc), inc)


# ----------------------------------------------------------------------------
# solves
# ----------------------------------------------------------------------------

def test_dense_lu_equals_gmres_and_bicgstab():
    n = 6
    coef = gen.helmholtz_medium(n, gen.rng_for(7, 2))
    A = op.Operator(op.KIND_HELMHOLTZ, coef, 2.0)
    b = A.rhs(gen.plane_wave_gradient(n, 2.0, np.array([0.0, 0.0, 1.0])))
    x_lu = sv.dense_solve(A.apply, b)
    x_gm, info = sv.gmres(A.apply, b, tol=1e-13)
    assert info["converged"]
    assert rel(x_gm, x_lu) < 1e-12
    x_bi, info = sv.bicgstab(A.apply, b, tol=1e-13)
    assert rel(x_bi, x_lu) < 1e-11


def test_neumann_series_laplace():
    n = 12
    coef = gen.laplace_medium(n, gen.rng_for(7, 3))
    A = op.Operator(op.KIND_LAPLACE, coef, 0.0)
    b = A.rhs(gen.constant_field(n, (0.0, 0.0, 1.0)))
    x_n, info = sv.neumann(A.apply, b, tol=1e-12)
    assert info["rel_residual"] < 1e-12
    x_g, _ = sv.gmres(A.apply, b, tol=1e-13)
    assert rel(x_n, x_g) < 1e-11


def test_manufactured_solution_helmholtz():
    n, sigma, omega = 32, 0.15, 4 * math.pi
    X, Y, Z = gen.grid_coords(n)
    coef = gen.helmholtz_medium(n, gen.rng_for(2, 0))
    A = op.Operator(op.KIND_HELMHOLTZ, coef, omega)
    rho = gen.gaussian(n, sigma)
    c = np.array([0.3 + 0.1j, -0.5, 0.8j])
    Jstar = c[:, None, None, None] * rho[None]
    hess = cf.gaussian_hessian(X, Y, Z, sigma, omega)
    Ustar = np.einsum("ab...,b->a...", hess, c)
    b = Jstar - op.pointwise(A.H, Jstar + 2 * Ustar)
    x, info = sv.gmres(A.apply, b, tol=1e-13)
    assert info["converged"]
    assert rel(x, Jstar) < 1e-9


class FlippedSignOperator(op.Operator):
    """The '+' reading of eq. intH: J + H (J + 2U) (planted mistake)."""

    def apply(self, x):
        U = self.conv.sym_apply(x)
        return x + op.pointwise(self.H, x + 2.0 * U)

    def rhs(self, inc):
        return -super().rhs(inc)


def _ball_error(cls, n, a_const):
    """Interior field error of the dielectric ball solved with coefficient a = eps^{-1}."""
    coef = gen.sphere_medium(n, a_const, radius=0.5)
    E0 = np.array([0.2, -0.3, 1.0])
    A = cls(op.KIND_HELMHOLTZ, coef, 2 * math.pi * 1e-50)
    inc = gen.constant_field(n, E0)
    x, info = sv.gmres(A.apply, A.rhs(inc), tol=1e-10)
    fld = A.field(x, inc)
    X, Y, Z = gen.grid_coords(n)
    inner = (X * X + Y * Y + Z * Z) < 0.3 ** 2
    ref = cf.sphere_interior_field(a_const, E0)
    got = fld[:, inner]
    return float(np.max(np.abs(got - ref[:, None])) / np.linalg.norm(ref))


@pytest.mark.slow
def test_dielectric_ball_first_order_and_sign():
    rng = gen.rng_for(7, 4)
    Q = gen.random_rotation(rng)
    a_const = Q @ np.diag([1.5, 2.5, 3.5]) @ Q.T
    e16 = _ball_error(op.Operator, 16, a_const)
    e32 = _ball_error(op.Operator, 32, a_const)
    assert e32 < 0.06
    assert e32 < 0.75 * e16
    bad = _ball_error(FlippedSignOperator, 16, a_const)
    assert bad > 2 * e16


def test_maxwell_duality():
    n, omega = 8, 3.0
    eps, mu = gen.maxwell_medium(n, gen.rng_for(3, 0))
    inc = gen.plane_wave_em(n, omega, np.array([0.0, 0.6, 0.8]), np.array([1.0, 0.0, 0.0]))
    A = op.Operator(op.KIND_MAXWELL, eps, omega, mu=mu)
    x, _ = sv.gmres(A.apply, A.rhs(inc), tol=1e-13)
    B = op.Operator(op.KIND_MAXWELL, mu, omega, mu=eps)
    inc2 = np.concatenate([inc[3:], -inc[:3]])
    y, _ = sv.gmres(B.apply, B.rhs(inc2), tol=1e-13)
    assert rel(y[:3], x[3:]) < 1e-11
    assert rel(y[3:], -x[:3]) < 1e-11


def test_maxwell_field_is_incident_plus_scattered():
    # field() of full Maxwell with M = 0 and mu = I reduces to the reduced form
    n, omega = 8, 3.0
    eps, _ = gen.maxwell_medium(n, gen.rng_for(3, 0))
    full = op.Operator(op.KIND_MAXWELL, eps, omega, mu=gen.identity_field(n))
    red = op.Operator(op.KIND_MAXWELL, eps, omega)
    inc = gen.plane_wave_em(n, omega, np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0]))
    xr, _ = sv.gmres(red.apply, red.rhs(inc[:3]), tol=1e-13)
    xf, _ = sv.gmres(full.apply, full.rhs(inc), tol=1e-13)
    assert rel(xf[:3], xr) < 1e-11
    assert np.linalg.norm(xf[3:]) < 1e-11 * np.linalg.norm(xr)
    assert rel(full.field(xf, inc)[:3], red.field(xr, inc[:3])) < 1e-11
