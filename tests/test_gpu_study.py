"""The qualitative claims of the paper's numerical study (Section 5, Tables
2-5 and the iteration-count figure) on small grids, through the C ABI:

* the rows at omega / 2 pi = 1e-50 and 1e-10 coincide (static limit);
* the iteration count is about constant as the grid is refined (a
  second-kind equation);
* it grows with the frequency and with the contrast (eps444 > eps222), and
  the rotation of the principal axes changes it little (eps234 ~ epsdense);
* the scattered field converges rapidly under refinement.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-12
_cache = {}


@pytest.fixture(scope="module")
def study():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_04791_amd import study as s
    from paper_1805_04791_amd import vie
    vie.load_library()
    return s


def case(study, equation, medium, n, size):
    key = (equation, medium, n, size)
    if key not in _cache:
        print(f"study case {key}", flush=True)
        _cache[key] = study.run_case(equation, medium, n, size, "bicgstab", TOL, 4000)
        assert _cache[key]["converged"], key
    return _cache[key]


@pytest.mark.parametrize("equation", ["helmholtz", "maxwell"])
@pytest.mark.parametrize("medium", ["eps222", "epsdense"])
def test_static_limit_rows_coincide(study, equation, medium):
    a = case(study, equation, medium, 32, 1e-50)
    b = case(study, equation, medium, 32, 1e-10)
    assert a["matvecs"] == b["matvecs"]
    # two solves to TOL of operators that differ by O(omega^2): the fields
    # agree to the solve tolerance times the conditioning, not to rounding
    e2, _ = study.field_errors(b["fields"], a["fields"])
    assert e2 < 1000 * TOL


@pytest.mark.parametrize("equation", ["helmholtz", "maxwell"])
def test_static_limit_operators_coincide(study, equation):
    """The FP64 applies at omega / 2 pi = 1e-50 and 1e-10 differ by O(omega):
    the kernel's first-order term i omega / 4 pi is a constant, which the
    derivatives annihilate in the continuum but not exactly on the grid for a
    rough (random) density, so the bound is omega itself."""
    from paper_1805_04791_amd import vie
    from vie_inputs import generators as gen
    n = 32
    x = gen.random_density((1, 3, n, n, n), gen.rng_for(gen.CONFIG_IDS["test"], 1400))
    y = []
    for size in (1e-50, 1e-10):
        kind, coef, omega, h, _ = study.problem(equation, "epsdense", n, size)
        plan = vie.Plan(kind, coef, omega=omega, h=h, precision=vie.PREC_FP64)
        y.append(plan.apply(x).cpu().numpy())
        plan.close()
    assert np.linalg.norm(y[1] - y[0]) < 2 * np.pi * 1e-10 * np.linalg.norm(y[0])


@pytest.mark.parametrize("medium,size", [("eps222", 1e-50), ("eps222", 1.0), ("eps444", 1.0)])
def test_iterations_about_constant_under_refinement(study, medium, size):
    m = [case(study, "maxwell", medium, n, size)["matvecs"] for n in (32, 48, 64)]
    assert max(m) <= 1.2 * min(m) + 2, m


def test_iterations_grow_with_frequency_and_contrast(study):
    mv = {(m, s): case(study, "maxwell", m, 48, s)["matvecs"]
          for m in ("eps222", "eps234", "epsdense", "eps444") for s in (1e-50, 1.0)}
    for m in ("eps222", "eps234", "epsdense", "eps444"):
        assert mv[(m, 1.0)] > mv[(m, 1e-50)], (m, mv)
    for s in (1e-50, 1.0):
        assert mv[("eps444", s)] > mv[("eps222", s)], mv
        # anisotropy with rotated axes vs the same eigenvalues unrotated
        a, b = mv[("eps234", s)], mv[("epsdense", s)]
        assert abs(a - b) <= 0.25 * max(a, b), mv


@pytest.mark.parametrize("medium", ["eps222", "eps444"])
def test_scattered_field_converges_under_refinement(study, medium):
    f = {n: case(study, "maxwell", medium, n, 1.0)["fields"] for n in (32, 48, 64)}
    e32, _ = study.field_errors(f[32], f[64])
    e48, _ = study.field_errors(f[48], f[64])
    assert e48 < 0.5 * e32, (e32, e48)
    assert e32 < 1e-2


def paper_counts():
    """{(medium, size): [(n, N_matvec), ...]} from the paper's Tables 2-5 (fixture)."""
    import os
    out = {}
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_tables_2_5_nmatvec.txt")
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            m, size, n, k = line.split()
            out.setdefault((m, float(size)), []).append((int(n), int(k)))
    return out


@pytest.mark.parametrize("medium", ["eps222", "eps234", "epsdense", "eps444"])
def test_iteration_counts_near_the_papers_tables(study, medium):
    """Reduced Maxwell at 64^3 (the compiled grid nearest the paper's coarsest,
    70 or 50 points) with Bi-CGStab to 1e-14: N_matvec within 25% of the
    count the paper prints for its coarsest grid, at every size of its table.
    The band covers what the tables leave unstated (incidence, whether the
    final residual check is counted); the counts differ by 2-23% here."""
    table = paper_counts()
    for size in study.sizes_for(medium):
        n_paper, k_paper = min(table[(medium, size)])
        print(f"paper table {medium} size {size:g}: n {n_paper}, N_matvec {k_paper}", flush=True)
        r = study.run_case("maxwell", medium, 64, size, "bicgstab", 1e-14, 20000)
        assert r["converged"]
        assert abs(r["matvecs"] / k_paper - 1.0) <= 0.25, (medium, size, r["matvecs"], k_paper)
