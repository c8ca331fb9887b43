"""Host logic of the replication study (CPU): check points, inputs, errors, tables."""

import math

import numpy as np

from paper_1805_04791_amd import study
from vie_inputs import generators as gen


def test_check_points_lie_outside_the_unit_box():
    pts = study.check_points()
    assert pts.shape == (26, 3)
    assert np.allclose(np.linalg.norm(pts, axis=1), 1.5)
    # outside [-1/2, 1/2]^3 by more than 2h at every supported grid >= 32
    assert np.min(np.max(np.abs(pts), axis=1)) > 0.5 + 2.0 / 32
    assert len({tuple(np.round(p, 12)) for p in pts}) == 26


def test_invert_tensor_is_the_pointwise_inverse():
    eps = gen.paper_medium("epsdense", 8)
    inv = study.invert_tensor(eps)
    m = eps.reshape(3, 3, -1)
    mi = inv.reshape(3, 3, -1)
    prod = np.einsum("abp,bcp->acp", m, mi)
    assert np.max(np.abs(prod - np.eye(3)[:, :, None])) < 1e-13


def test_static_limit_inputs_are_uniform_fields():
    for eq in ("helmholtz", "maxwell"):
        kind, coef, omega, h, inc = study.problem(eq, "eps222", 8, 1e-50)
        assert h == 1.0 / 8 and omega == 2 * math.pi * 1e-50
        assert inc.shape == (1, 3, 8, 8, 8)
        want = study.DIRECTION if eq == "helmholtz" else study.POLARISATION
        assert np.max(np.abs(inc[0] - want[:, None, None, None])) < 1e-15
    # the incident fields are plane waves along d at finite frequency
    kind, coef, omega, h, inc = study.problem("maxwell", "eps234", 8, 1.0)
    X, Y, Z = gen.grid_coords(8, -0.5, 1.0 / 8)
    ph = np.exp(1j * omega * (0.48 * X + 0.6 * Y + 0.64 * Z))
    assert np.max(np.abs(inc[0, 0] - 0.8 * ph)) < 1e-14
    assert abs(np.dot(study.DIRECTION, study.POLARISATION)) < 1e-15


def test_errors_against_the_finest_grid():
    rows = []
    ref = np.array([[1.0, 2.0], [3.0, -4.0]], dtype=complex)
    for n, f in ((32, ref * (1 + 1e-3)), (64, ref)):
        rows.append({"equation": "maxwell", "medium": "eps222", "size": 1.0, "solver": "bicgstab", "n": n,
                     "fields": f, "tol": 1e-14, "unknowns": 3 * n ** 3, "support_unknowns": 3 * n ** 3,
                     "matvecs": 10, "converged": True, "iters": 5, "solve_s": 0.1, "plan_s": 0.2})
    study.add_errors(rows)
    assert rows[1]["E2"] is None and rows[1]["reference_n"] is None
    assert abs(rows[0]["E2"] - 1e-3) < 1e-12 and abs(rows[0]["Einf"] - 1e-3) < 1e-12
    md = study.markdown(rows)
    assert "| 1 | 32 |" in md and "1.0e-03" in md and "—" in md


def test_paper_sizes():
    assert tuple(study.sizes_for("eps222")) == (1e-50, 1e-10, 1.0, 20.0)
    for m in ("eps234", "epsdense", "eps444"):
        assert tuple(study.sizes_for(m)) == (1e-50, 1e-10, 1.0, 5.0)
