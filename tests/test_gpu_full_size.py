"""Full-size parity at the benchmark's configurations (GPU, through the C ABI).

The oracle is evaluated on the whole grid (window FFT route, FP64): its
kernel tables are built once per configuration (Section 5 with readings
R4-R6), and its GMRES solves run to a true residual of 1e-13.  Checks:

* the FP64 and FP32 applies of the whole grid against the oracle's apply,
  element by element (1e-12 and 2e-6 relative l2);
* the batched mixed solve of the 128^3 Helmholtz workload (8 right-hand
  sides in one launch, as the benchmark runs it): the oracle's true residual
  ||b - A x|| / ||b|| of every solution <= 2e-9 (twice the solver's 1e-9),
  and one oracle solve compared element by element with the mixed (1e-8) and
  the FP64 (1e-10) solutions; a right-hand side alone gives bitwise the
  batch's answer;
* reduced and full Maxwell 128^3: mixed and FP64 solutions against an oracle
  solve;
* the batched 96^3 workload with 64 right-hand sides: two of them against
  oracle solves, and alone against the batch;
* the largest grid (160^3): whole-grid applies and the oracle residual of a
  mixed solve.
"""

import math

import numpy as np
import pytest

from oracle import operator as op
from oracle import solve as sv
from vie_inputs import generators as gen

from _helpers import rel

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vie():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_04791_amd import vie as v
    v.load_library()
    return v


def oracle_residual(A, inc, x):
    b = A.rhs(inc)
    return float(np.linalg.norm(b - A.apply(x)) / np.linalg.norm(b))


def oracle_solution(A, inc):
    x, info = sv.gmres(A.apply, A.rhs(inc), tol=1e-13, restart=100)
    assert info["rel_residual"] <= 1e-13
    return x


class Helmholtz128:
    """The headline problem, its oracle operator and (computed once) the oracle
    solution of right-hand side 0."""

    def __init__(self):
        self.prob = gen.config_problem("helmholtz128", nrhs=8)
        print("[full-size] oracle setup at 128^3 (Helmholtz)", flush=True)
        self.A = op.Operator(self.prob.kind, self.prob.coef, self.prob.omega)
        self._x0 = None

    def __iter__(self):
        return iter((self.prob, self.A))

    def x0(self):
        if self._x0 is None:
            print("[full-size] oracle solve at 128^3 (Helmholtz, right-hand side 0)", flush=True)
            self._x0 = oracle_solution(self.A, self.prob.inc[0])
        return self._x0


@pytest.fixture(scope="module")
def helmholtz128():
    return Helmholtz128()


@pytest.mark.timeout(900)
def test_applies_128_match_oracle(vie, helmholtz128):
    prob, A = helmholtz128
    n = prob.n
    x = gen.random_density((1, 3, n, n, n), gen.rng_for(gen.CONFIG_IDS["test"], 800))
    plan = vie.Plan(prob.kind, prob.coef, omega=prob.omega, precision=vie.PREC_MIXED)
    y64 = plan.apply(x, vie.APPLY_FP64).cpu().numpy()[0]
    y32 = plan.apply(x, vie.APPLY_FP32).cpu().numpy()[0]
    ref = A.apply(x[0])
    assert rel(y64, ref) < 1e-12
    assert rel(y32, ref) < 2e-6
    plan.close()


@pytest.mark.timeout(900)
def test_batched_mixed_solve_128_matches_oracle(vie, helmholtz128):
    """The benchmark's step: 8 right-hand sides in one batched mixed solve."""
    prob, A = helmholtz128
    plan = vie.Plan(prob.kind, prob.coef, omega=prob.omega, precision=vie.PREC_MIXED, max_rhs=8)
    d, _, st, rc = plan.solve(prob.inc, tol=1e-9, want_field=False)
    assert rc == vie.OK
    d = d.cpu().numpy()
    d64, _, st64, rc64 = plan.solve(prob.inc[:1], tol=1e-12, fp64=True, want_field=False)
    assert rc64 == vie.OK
    d64 = d64.cpu().numpy()
    for r in range(8):
        assert st[r]["rel_residual"] <= 1e-9 and st[r]["matvecs_fp32"] > 0
        assert oracle_residual(A, prob.inc[r], d[r]) <= 2e-9
    x0 = helmholtz128.x0()
    assert rel(d[0], x0) < 1e-8
    assert rel(d64[0], x0) < 1e-10
    # a right-hand side alone: bitwise the batch's answer
    d3, _, st3, _ = plan.solve(prob.inc[3:4], tol=1e-9, want_field=False)
    assert np.array_equal(d3.cpu().numpy()[0], d[3])
    assert st3[0]["iters"] == st[3]["iters"]
    plan.close()


@pytest.mark.timeout(900)
def test_alternative_splits_128_match_oracle(vie, helmholtz128, monkeypatch):
    """Every pass on its alternative split (VIE_SPLITS): the whole-grid
    applies on 256 = 32 x 8 and the solver's 216 = 12 x 18 (x, y) and
    256 = 32 x 8 (z) against the oracle."""
    monkeypatch.setenv("VIE_SPLITS", "1,1,1,1,1")
    prob, A = helmholtz128
    n = prob.n
    x = gen.random_density((1, 3, n, n, n), gen.rng_for(gen.CONFIG_IDS["test"], 802))
    plan = vie.Plan(prob.kind, prob.coef, omega=prob.omega, precision=vie.PREC_MIXED, max_rhs=1)
    assert plan.info()["box_P"] == 216
    y64 = plan.apply(x, vie.APPLY_FP64).cpu().numpy()[0]
    y32 = plan.apply(x, vie.APPLY_FP32).cpu().numpy()[0]
    d, _, st, rc = plan.solve(prob.inc[:1], tol=1e-9, want_field=False)
    d64, _, st64, rc64 = plan.solve(prob.inc[:1], tol=1e-12, fp64=True, want_field=False)
    assert rc == vie.OK and rc64 == vie.OK
    plan.close()
    ref = A.apply(x[0])
    assert rel(y64, ref) < 1e-12
    assert rel(y32, ref) < 2e-6
    x0 = helmholtz128.x0()
    assert rel(d.cpu().numpy()[0], x0) < 1e-8
    assert rel(d64.cpu().numpy()[0], x0) < 1e-10


@pytest.mark.timeout(900)
@pytest.mark.parametrize("full", [False, True])
def test_maxwell_128_matches_oracle(vie, full):
    """Maxwell 128^3 (rotated anisotropic eps, and mu): the mixed solution to
    1e-9 and the FP64 solution to 1e-12 against an oracle solve."""
    prob = gen.config_problem("maxwell128", nrhs=1)
    mu = prob.mu if full else None
    inc = prob.inc[:1] if full else prob.inc[:1, :3]
    plan = vie.Plan(prob.kind, prob.coef, omega=prob.omega, mu=mu, precision=vie.PREC_MIXED, max_rhs=1)
    dm, _, sm, rc = plan.solve(inc, tol=1e-9, want_field=False)
    assert rc == vie.OK
    d64, _, s64, rc = plan.solve(inc, tol=1e-12, fp64=True, want_field=False)
    assert rc == vie.OK
    dm, d64 = dm.cpu().numpy(), d64.cpu().numpy()
    plan.close()
    print(f"[full-size] oracle setup and solve at 128^3 (Maxwell, mu {'given' if full else '= I'})", flush=True)
    A = op.Operator(prob.kind, prob.coef, prob.omega, mu=mu)
    x0 = oracle_solution(A, inc[0])
    assert rel(dm[0], x0) < 1e-8
    assert rel(d64[0], x0) < 1e-10


@pytest.mark.timeout(900)
def test_batched_96_64_rhs_matches_oracle(vie):
    """The batched 96^3 workload: 64 right-hand sides through fused launches
    (chunks of 16); right-hand sides 0 and 37 against oracle solves, and alone
    against the batch (bitwise); right-hand side 63 in FP64 against the mixed one."""
    prob = gen.config_problem("batched96")
    assert prob.inc.shape[0] == 64
    plan = vie.Plan(prob.kind, prob.coef, omega=prob.omega, precision=vie.PREC_MIXED, max_rhs=16)
    d, _, st, rc = plan.solve(prob.inc, tol=1e-9, want_field=False)
    assert rc == vie.OK and all(s["rel_residual"] <= 1e-9 for s in st)
    d = d.cpu().numpy()
    for r in (0, 37):
        ds, _, ss, _ = plan.solve(prob.inc[r:r + 1], tol=1e-9, want_field=False)
        assert np.array_equal(ds.cpu().numpy()[0], d[r])
    d64, _, _, _ = plan.solve(prob.inc[63:64], tol=1e-11, fp64=True, want_field=False)
    assert rel(d[63], d64.cpu().numpy()[0]) < 1e-8
    plan.close()
    print("[full-size] oracle setup and two solves at 96^3", flush=True)
    A = op.Operator(prob.kind, prob.coef, prob.omega)
    for r in (0, 37):
        assert rel(d[r], oracle_solution(A, prob.inc[r])) < 1e-8


@pytest.mark.timeout(900)
def test_largest_grid_160(vie):
    """The largest supported grid (160^3, the top of the serving mix): the
    Helmholtz recipe at omega = 10 pi.  The whole-grid apply runs on length
    320 along every axis with tables from the 640-point precompute, the solver
    on the support box (length 256 along every axis: the box is 128 points
    along z, and 256 has a square split).  FP64 and FP32
    applies against the oracle on the whole grid, and the oracle residual of a
    mixed solve of 2 right-hand sides."""
    n = 160
    prob = gen.helmholtz_problem(n, 10 * math.pi, "helmholtz128", nrhs=2)
    plan = vie.Plan(prob.kind, prob.coef, omega=prob.omega, precision=vie.PREC_MIXED, max_rhs=2)
    assert plan.info()["box_P"] == 256 and plan.info()["box_Pz"] == 256
    x = gen.random_density((1, 3, n, n, n), gen.rng_for(gen.CONFIG_IDS["test"], 801))
    y64 = plan.apply(x, vie.APPLY_FP64).cpu().numpy()[0]
    y32 = plan.apply(x).cpu().numpy()[0]
    d, _, st, rc = plan.solve(prob.inc, tol=1e-9, want_field=False)
    assert rc == vie.OK and all(s["rel_residual"] <= 1e-9 for s in st)
    d = d.cpu().numpy()
    plan.close()
    print("[full-size] oracle setup at 160^3", flush=True)
    A = op.Operator(prob.kind, prob.coef, prob.omega)
    ref = A.apply(x[0])
    assert rel(y64, ref) < 1e-12
    assert rel(y32, ref) < 2e-6
    for r in range(2):
        assert oracle_residual(A, prob.inc[r], d[r]) <= 2e-9
