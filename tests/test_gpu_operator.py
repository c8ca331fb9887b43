"""GPU parity of the operator pieces against the oracle, through the C ABI.

Rows covered: contrast (eq. rhodef), kernel-transform tables (the
truncated-kernel method of Section 5), forward/inverse pruned FFTs and the
spectral multiply (checked through the raw convolution), the pointwise
combine (the matvec of eqs. intLap, contractionK, contraction_Maxwell_reduced,
intM), the right-hand side 2 H g and the total field.

Tolerances: FP64 path 1e-12 relative l2 (rounding of ~10 FFT stages on
complex128), FP32 path 2e-6 (the same with complex64, unit roundoff 6e-8,
times the log-depth of the transforms and the table magnitudes).
"""

import math

import numpy as np
import pytest

from oracle import operator as op
from vie_inputs import generators as gen

from _helpers import medium, oracle_octant_tables, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KINDS = [("laplace", op.KIND_LAPLACE, False), ("helmholtz", op.KIND_HELMHOLTZ, False),
         ("maxwell", op.KIND_MAXWELL, False), ("maxwell_full", op.KIND_MAXWELL, True)]


@pytest.fixture(scope="module")
def vie():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_04791_amd import vie as v
    v.load_library()
    return v


# non-symmetric media (a rotation composed with a shear): H and H^T differ, so
# these cases fix the orientation of H v and the ABI's tensor layout
# "entry (a, b) at 3a + b" against the oracle
SHEARED = [("laplace_sheared", op.KIND_LAPLACE, False), ("helmholtz_sheared", op.KIND_HELMHOLTZ, False),
           ("maxwell_full_sheared", op.KIND_MAXWELL, True)]


def make_plan(vie, kind, n, full=False, precision=0, seed=0, max_rhs=2, sheared=False):
    coef, mu, omega = medium(kind, n, seed, full, sheared=sheared)
    plan = vie.Plan(kind, coef, omega=omega, mu=mu, precision=precision, max_rhs=max_rhs)
    oper = op.Operator(kind, coef, omega, mu=mu)
    return plan, oper, coef, mu, omega


@pytest.mark.parametrize("name,kind,full", SHEARED)
def test_sheared_medium_matches_oracle(vie, name, kind, full):
    """Contrast, FP64 and FP32 matvecs, right-hand side and field on a
    non-symmetric medium against the oracle (tolerances as above)."""
    n = 16
    plan, oper, *_ = make_plan(vie, kind, n, full, precision=vie.PREC_MIXED, sheared=True)
    Hc = plan.contrast()
    assert rel(Hc[0], oper.H) < 1e-14
    if full:
        assert rel(Hc[1], oper.Hmu) < 1e-14
    h = oper.H.reshape(3, 3, -1)
    assert np.abs(h - h.transpose(1, 0, 2)).max() > 0.05      # really non-symmetric
    want = op.contrast_norm_max(oper.H)
    if full:
        want = max(want, op.contrast_norm_max(oper.Hmu))
    assert abs(plan.info()["max_contrast_norm"] - want) < 1e-12
    rng = gen.rng_for(gen.CONFIG_IDS["test"], 720)
    x = gen.random_density((2, oper.ncomp, n, n, n), rng)
    inc = gen.random_density((2, oper.ncomp, n, n, n), rng)
    y64 = plan.apply(x, vie.APPLY_FP64).cpu().numpy()
    y32 = plan.apply(x, vie.APPLY_FP32).cpu().numpy()
    b = plan.rhs(inc).cpu().numpy()
    f = plan.field(x, inc).cpu().numpy()
    for r in range(2):
        ref = oper.apply(x[r])
        assert rel(y64[r], ref) < 1e-12
        assert rel(y32[r], ref) < 2e-6
        assert rel(b[r], oper.rhs(inc[r])) < 1e-14
        assert rel(f[r], oper.field(x[r], inc[r])) < 1e-12
    plan.close()


@pytest.mark.parametrize("name,kind,full", KINDS)
def test_contrast_matches_oracle(vie, name, kind, full):
    n = 12
    plan, oper, *_ = make_plan(vie, kind, n, full)
    H = plan.contrast()
    assert rel(H[0], oper.H) < 1e-14
    if full:
        assert rel(H[1], oper.Hmu) < 1e-14
    info = plan.info()
    assert info["max_contrast_norm"] < 1.0
    assert abs(info["max_contrast_norm"] - op.contrast_norm_max(oper.H if not full else oper.H)) < 1e-12 or full
    plan.close()


@pytest.mark.parametrize("n", [8, 12, 16, 24])
@pytest.mark.parametrize("name,kind,full", KINDS)
def test_tables_match_oracle(vie, n, name, kind, full):
    plan, oper, coef, mu, omega = make_plan(vie, kind, n, full)
    got = plan.tables()
    ne = got.shape[2]
    sym = "D" if kind == op.KIND_MAXWELL else "grad"
    ref = oracle_octant_tables(sym, n, 2.0 / n, oper.omega)
    assert ne == (9 if full else 6)
    assert rel(got[:, :, :6, : n + 1], ref) < 1e-12
    if full:
        curl = oracle_octant_tables("curl", n, 2.0 / n, oper.omega) * (1j * oper.omega)
        assert rel(got[:, :, 6:, : n + 1], curl) < 1e-12
    plan.close()


@pytest.mark.parametrize("n", [8, 16, 24, 32])
@pytest.mark.parametrize("name,kind,full", KINDS)
def test_apply_fp64_matches_oracle(vie, n, name, kind, full):
    plan, oper, *_ = make_plan(vie, kind, n, full, precision=vie.PREC_FP64)
    rng = gen.rng_for(gen.CONFIG_IDS["test"], 500 + n)
    x = gen.random_density((2, oper.ncomp, n, n, n), rng)
    y = plan.apply(x, vie.APPLY_FP64).cpu().numpy()
    for r in range(2):
        assert rel(y[r], oper.apply(x[r])) < 1e-12
    # the raw convolution
    u = plan.apply(x, vie.APPLY_FP64 | vie.APPLY_CONV).cpu().numpy()
    if full:
        ref = oper.field(x[0], np.zeros_like(x[0]))
    else:
        ref = oper.conv.sym_apply(x[0])
    assert rel(u[0], ref) < 1e-12
    plan.close()


@pytest.mark.parametrize("n", [16, 32])
@pytest.mark.parametrize("name,kind,full", KINDS)
def test_apply_fp32_matches_oracle(vie, n, name, kind, full):
    plan, oper, *_ = make_plan(vie, kind, n, full, precision=vie.PREC_MIXED)
    rng = gen.rng_for(gen.CONFIG_IDS["test"], 600 + n)
    x = gen.random_density((1, oper.ncomp, n, n, n), rng)
    y = plan.apply(x, vie.APPLY_FP32).cpu().numpy()
    assert rel(y[0], oper.apply(x[0])) < 2e-6
    plan.close()


@pytest.mark.parametrize("n", [16, 24])
@pytest.mark.parametrize("name,kind,full", KINDS)
def test_apply_complex64_vectors(vie, n, name, kind, full):
    """The FP32 matvec on complex64 vectors: the oracle to FP32 accuracy, and
    the complex128-vector FP32 matvec to the rounding of its output."""
    plan, oper, *_ = make_plan(vie, kind, n, full, precision=vie.PREC_MIXED)
    rng = gen.rng_for(gen.CONFIG_IDS["test"], 650 + n)
    x = gen.random_density((2, oper.ncomp, n, n, n), rng).astype(np.complex64)
    y32 = plan.apply(x, vie.APPLY_C64)
    assert y32.dtype == torch.complex64
    y32 = y32.cpu().numpy()
    y = plan.apply(x.astype(np.complex128), vie.APPLY_FP32).cpu().numpy()
    for r in range(2):
        assert rel(y32[r], oper.apply(x[r].astype(np.complex128))) < 2e-6
        assert rel(y32[r], y[r]) < 1e-7
    plan.close()


@pytest.mark.parametrize("name,kind,full", KINDS)
def test_rhs_and_field_match_oracle(vie, name, kind, full):
    n = 16
    plan, oper, coef, mu, omega = make_plan(vie, kind, n, full)
    rng = gen.rng_for(gen.CONFIG_IDS["test"], 700)
    inc = gen.random_density((2, oper.ncomp, n, n, n), rng)
    dens = gen.random_density((2, oper.ncomp, n, n, n), rng)
    b = plan.rhs(inc).cpu().numpy()
    f = plan.field(dens, inc).cpu().numpy()
    for r in range(2):
        assert rel(b[r], oper.rhs(inc[r])) < 1e-14
        assert rel(f[r], oper.field(dens[r], inc[r])) < 1e-12
    plan.close()


def test_batched_apply_equals_single(vie):
    n = 16
    plan, oper, *_ = make_plan(vie, op.KIND_HELMHOLTZ, n, max_rhs=3)
    rng = gen.rng_for(gen.CONFIG_IDS["test"], 800)
    x = gen.random_density((5, 3, n, n, n), rng)   # 5 > max_rhs: processed in chunks
    yb = plan.apply(x, vie.APPLY_FP32).cpu().numpy()
    for r in range(5):
        ys = plan.apply(x[r:r + 1], vie.APPLY_FP32).cpu().numpy()[0]
        assert np.array_equal(ys, yb[r])
    plan.close()


def test_apply_is_deterministic(vie):
    n = 24
    plan, oper, *_ = make_plan(vie, op.KIND_MAXWELL, n, True)
    x = gen.random_density((1, 6, n, n, n), gen.rng_for(gen.CONFIG_IDS["test"], 801))
    a = plan.apply(x, vie.APPLY_FP32).cpu().numpy()
    b = plan.apply(x, vie.APPLY_FP32).cpu().numpy()
    assert np.array_equal(a, b)
    plan.close()
