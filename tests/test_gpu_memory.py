"""Device memory of plans (GPU, through the C ABI): a destroyed plan's blocks
go to the library's cache, later plans reuse them with the same results as on
fresh memory, and vie_release_cached_memory empties the cache."""

import numpy as np
import pytest

from oracle import operator as op
from vie_inputs import generators as gen

from _helpers import medium

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vie():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_04791_amd import vie as v
    v.load_library()
    return v


def solve_once(vie, coef, omega, inc):
    """(density, device bytes held by the plan) of one mixed solve on a new plan."""
    with vie.Plan(op.KIND_HELMHOLTZ, coef, omega=omega, precision=vie.PREC_MIXED, max_rhs=2) as plan:
        d, _, st, rc = plan.solve(inc, tol=1e-10, want_field=False)
        assert rc == 0
        return d.cpu().numpy(), plan.info()["device_bytes"]


def test_released_blocks_are_cached_and_reused(vie):
    n = 32
    coef, _, omega = medium(op.KIND_HELMHOLTZ, n, 21)
    rng = gen.rng_for(gen.CONFIG_IDS["test"], 221)
    inc = np.stack([gen.plane_wave_gradient(n, omega, gen.random_unit(rng)) for _ in range(2)])
    vie.release_cached_memory()
    d_fresh, held = solve_once(vie, coef, omega, inc)
    # every block of the destroyed plan is cached (far below the cache limit)
    cached = vie.release_cached_memory()
    assert cached >= held > 0
    assert vie.release_cached_memory() == 0
    # a plan on reused blocks (the first plan's, released again) computes the same
    d_again, _ = solve_once(vie, coef, omega, inc)
    d_reused, _ = solve_once(vie, coef, omega, inc)
    assert np.array_equal(d_fresh, d_again)
    assert np.array_equal(d_fresh, d_reused)
    assert vie.release_cached_memory() >= held


def test_destroy_waits_for_the_plans_work_only(vie):
    """vie_destroy waits for the work of the plan's last call (an event recorded
    after it), not for later work of other callers on the same stream: after
    the plan's apply, a bounded spin kernel on that stream is still running
    when the destroy returns, and the apply's result is complete."""
    n = 16
    coef, _, omega = medium(op.KIND_HELMHOLTZ, n, 23)
    x = torch.from_numpy(gen.random_density((1, 3, n, n, n), gen.rng_for(gen.CONFIG_IDS["test"], 231))).cuda()
    s = torch.cuda.Stream()
    plan = vie.Plan(op.KIND_HELMHOLTZ, coef, omega=omega, precision=vie.PREC_FP64, stream=s)
    with torch.cuda.stream(s):
        y = plan.apply(x, vie.APPLY_FP64, stream=s)
        torch.cuda._sleep(int(5e7))  # bounded spin: tens of milliseconds
    plan.close()
    busy = not s.query()
    s.synchronize()
    assert busy, "the destroy waited for work queued after the plan's last call"
    ref = vie.Plan(op.KIND_HELMHOLTZ, coef, omega=omega, precision=vie.PREC_FP64)
    assert torch.equal(y, ref.apply(x, vie.APPLY_FP64))
    ref.close()
