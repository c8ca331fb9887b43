"""Potentials and fields after the solve (GPU, through the C ABI) against
oracle/postprocess.py on the same densities."""

import math

import numpy as np
import pytest

from oracle import operator as op
from oracle import postprocess as pp
from vie_inputs import generators as gen

from _helpers import medium, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vie():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_04791_amd import vie as v
    v.load_library()
    return v


def density(n, comps, item):
    return gen.random_density((2, comps, n, n, n), gen.rng_for(gen.CONFIG_IDS["test"], 1200 + item))


POINTS = np.array([[1.6, 0.2, -0.3], [-0.4, -1.9, 0.5], [0.3, 0.4, 2.5], [-3.0, 2.0, 1.0], [40.0, -25.0, 10.0]])
DIRS = np.array([[1.0, 0.0, 0.0], [0.0, 0.6, -0.8], [-0.36, 0.48, 0.8], [0.0, 0.0, -1.0]])


@pytest.mark.parametrize("kind", [op.KIND_LAPLACE, op.KIND_HELMHOLTZ])
@pytest.mark.parametrize("n", [16, 24])
def test_potential_on_grid(vie, kind, n):
    coef, _, omega = medium(kind, n, 30)
    plan = vie.Plan(kind, coef, omega=omega, precision=vie.PREC_MIXED, max_rhs=2)
    x = density(n, 3, n)
    phi = plan.potential(x).cpu().numpy()
    for r in range(2):
        assert rel(phi[r], pp.potential(x[r], omega)) < 1e-12
    plan.close()


def test_reduced_maxwell_h_on_grid(vie):
    n = 16
    coef, _, omega = medium(op.KIND_MAXWELL, n, 31)
    plan = vie.Plan(op.KIND_MAXWELL, coef, omega=omega, precision=vie.PREC_MIXED, max_rhs=2)
    x = density(n, 3, 1)
    hinc = density(n, 3, 2)
    hs = plan.field_h(x).cpu().numpy()
    ht = plan.field_h(x, hinc).cpu().numpy()
    for r in range(2):
        ref = pp.field_h_reduced(x[r], omega)
        assert rel(hs[r], ref) < 1e-12
        assert rel(ht[r], hinc[r] + ref) < 1e-12
    plan.close()


@pytest.mark.parametrize("kind,full", [(op.KIND_LAPLACE, False), (op.KIND_HELMHOLTZ, False),
                                       (op.KIND_MAXWELL, False), (op.KIND_MAXWELL, True)])
def test_fields_at_points_and_far_field_after_solve(vie, kind, full):
    """Solve, then evaluate the scattered fields outside the support and the
    far-field patterns of the GPU density; compare with the oracle's sums on
    the same density."""
    n = 16
    coef, mu, omega = medium(kind, n, 32, full)
    rng = gen.rng_for(gen.CONFIG_IDS["test"], 1300)
    d = gen.random_unit(rng)
    if kind == op.KIND_LAPLACE:
        inc = gen.constant_field(n, d)[None]
    elif kind == op.KIND_HELMHOLTZ:
        inc = gen.plane_wave_gradient(n, omega, d)[None]
    else:
        f = gen.plane_wave_em(n, omega, d, gen.random_polarisation(rng, d))
        inc = (f if full else f[:3])[None]
    plan = vie.Plan(kind, coef, omega=omega, mu=mu, precision=vie.PREC_MIXED, max_rhs=1)
    dens, _, st, rc = plan.solve(inc, tol=1e-10, fp64=True, want_field=False)
    assert rc == vie.OK
    dens_np = dens.cpu().numpy()
    got = plan.fields_at(dens, POINTS).cpu().numpy()[0]
    ref = pp.fields_at(kind, dens_np[0], omega, POINTS)
    assert rel(got, ref) < 1e-12
    if kind != op.KIND_LAPLACE:
        far = plan.far_field(dens, DIRS).cpu().numpy()[0]
        assert rel(far, pp.far_field(kind, dens_np[0], omega, DIRS)) < 1e-12
    plan.close()


def test_postprocess_argument_errors(vie):
    n = 16
    coef, _, omega = medium(op.KIND_HELMHOLTZ, n, 33)
    plan = vie.Plan(op.KIND_HELMHOLTZ, coef, omega=omega)
    x = density(n, 3, 5)[:1]
    with pytest.raises(vie.VieError) as e:
        plan.fields_at(x, [[0.0, 0.0, 0.0]])          # inside the support box
    assert e.value.code == vie.E_ARG
    with pytest.raises(vie.VieError) as e:
        plan.far_field(x, [[1.0, 1.0, 0.0]])          # not a unit vector
    assert e.value.code == vie.E_ARG
    with pytest.raises(vie.VieError) as e:
        plan.field_h(x)                               # not a Maxwell plan
    assert e.value.code == vie.E_STATE
    plan.close()
    lap, _, _ = medium(op.KIND_LAPLACE, n, 34)
    plan = vie.Plan(op.KIND_LAPLACE, lap)
    with pytest.raises(vie.VieError) as e:
        plan.far_field(x, DIRS)                       # omega = 0
    assert e.value.code == vie.E_STATE
    plan.close()
    mx, _, w = medium(op.KIND_MAXWELL, n, 35)
    plan = vie.Plan(op.KIND_MAXWELL, mx, omega=w)
    with pytest.raises(vie.VieError) as e:
        plan.potential(x)                             # Maxwell
    assert e.value.code == vie.E_STATE
    plan.close()


def offcentre(coef, n):
    """The medium restricted to an off-centre box (x > 0.1, y < 0.3)."""
    X, Y, Z = gen.grid_coords(n)
    mask = ((X > 0.1) & (Y < 0.3)).astype(np.float64)
    eye = np.eye(3, dtype=np.complex128).reshape(9, 1, 1, 1)
    return eye + mask[None] * (coef - eye)


@pytest.mark.parametrize("kind,full,n", [(op.KIND_LAPLACE, False, 24), (op.KIND_HELMHOLTZ, False, 48),
                                         (op.KIND_MAXWELL, False, 32), (op.KIND_MAXWELL, True, 24)])
def test_batched_sums_over_an_off_centre_support_box(vie, kind, full, n):
    """Five right-hand sides (not a multiple of the kernels' groups of
    right-hand sides or directions), densities that vanish outside the
    plan's support box, 37 points and 21 directions, against the oracle's sums."""
    coef, mu, omega = medium(kind, n, 36, full)
    coef = offcentre(coef, n)
    if mu is not None:
        mu = offcentre(mu, n)
    plan = vie.Plan(kind, coef, omega=omega, mu=mu, precision=vie.PREC_MIXED, max_rhs=5)
    x0, y0, z0, bx, by, bz = plan.info()["box"]
    assert (bx, by) != (n, n)
    C = 6 if full else 3
    x = density(n, C, 40 + n)
    x = np.concatenate([x, density(n, C, 41 + n), density(n, C, 42 + n)[:1]])
    inside = np.zeros((n, n, n))
    inside[z0:z0 + bz, y0:y0 + by, x0:x0 + bx] = 1.0
    x = x * inside
    rng = gen.rng_for(gen.CONFIG_IDS["test"], 1500 + n)
    pts = rng.standard_normal((37, 3))
    pts = 2.6 * pts / np.linalg.norm(pts, axis=1, keepdims=True)
    dirs = rng.standard_normal((21, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    got = plan.fields_at(x, pts).cpu().numpy()
    far = plan.far_field(x, dirs).cpu().numpy() if kind != op.KIND_LAPLACE else None
    for r in range(5):
        assert rel(got[r], pp.fields_at(kind, x[r], omega, pts)) < 1e-12, r
        if far is not None:
            assert rel(far[r], pp.far_field(kind, x[r], omega, dirs)) < 1e-12, r
    plan.close()
