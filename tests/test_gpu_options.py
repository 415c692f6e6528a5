"""GPU tests of the solver options and of admission under a tight budget.

* From x = 0 the library runs the iteration the oracle runs (Jacobi or no
  preconditioner): FP64 iteration counts agree within a few percent (the
  device applies A once per iteration with a single reduction and predicts
  its stopping point from the recurrence, the oracle checks its own
  recursive residual), and K and pressures agree with the oracle's solution.
* The linear initial guess solves a uniform network without an iteration
  (closed form, as in the oracle's pins).
* A context whose budget is held by an idle slab still admits a request that
  needs that budget: the pool releases the slab instead of waiting for it.
"""
import sys
import time

import numpy as np
import pytest

from paper_1908_03301_amd import binding as B
from paper_1908_03301_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = B.Context(0)
    yield c
    c.close()


NETS = [lambda: I.fbm_network(2, 200, 150, 1, H=0.7, sigma=1.5, occupancy=0.7, index=1400),
        lambda: I.fbm_network(2, 257, 129, 1, H=0.35, sigma=1.0, occupancy=1.0, index=1401, axis=1),
        lambda: I.fbm_network(3, 40, 33, 30, H=0.7, sigma=1.0, occupancy=0.5, index=1402),
        lambda: I.fbm_network(3, 70, 20, 24, H=0.8, sigma=1.5, occupancy=0.8, index=1403, axis=2)]


@pytest.mark.parametrize("case", range(len(NETS)))
@pytest.mark.parametrize("precond", [B.RN_JACOBI, B.RN_NONE])
def test_zero_guess_matches_oracle_iterations(ctx, oracle_mod, case, precond):
    net = NETS[case]()
    ref = oracle_mod.solve(net, tol=1e-13, want_mask=True)
    pc = oracle_mod.JACOBI if precond == B.RN_JACOBI else oracle_mod.NONE
    ora = oracle_mod.solve(net, tol=1e-10, x0=oracle_mod.X0_ZERO, precond=pc, want_pressure=False)
    say(f"case {case} precond {precond}: shape {net.shape} axis {net.axis}")
    res, P, M = B.solve_network(ctx, net, B.RN_FP64, 1e-10, 2_000_000, want_pressure=True, want_mask=True,
                                precond=precond, x0=B.RN_X0_ZERO)
    say(f"  device iters {res.iters}, oracle iters {ora.iters}, K {res.K!r} vs {ref.K!r}")
    assert res.status == 0 and res.converged
    np.testing.assert_array_equal(M, ref.mask)
    assert abs(res.iters - ora.iters) <= 2 + 0.03 * ora.iters
    assert res.K == pytest.approx(ref.K, rel=1e-9)
    live = ref.mask == 3
    np.testing.assert_array_equal(P[~live], ref.pressure[~live])
    # mixed precision from the same options reaches the mixed bar
    rm, Pm, _ = B.solve_network(ctx, net, B.RN_MIXED, 1e-8, 2_000_000, want_pressure=True, precond=precond,
                                x0=B.RN_X0_ZERO)
    assert rm.status == 0 and rm.converged
    assert rm.K == pytest.approx(ref.K, rel=1e-7)
    c = oracle_mod.check_pressure(net, Pm)
    assert c.rel_resid <= 1.01e-8


@pytest.mark.parametrize("dim,shape,axis", [(2, (300, 41, 1), 0), (3, (20, 33, 17), 2)])
@pytest.mark.parametrize("precision", [B.RN_FP64, B.RN_MIXED])
def test_linear_guess_exact_on_uniform(ctx, dim, shape, axis, precision):
    net = I.uniform_network(dim, *shape, g0=0.6, axis=axis)
    r, _, _ = B.solve_network(ctx, net, precision, 1e-10 if precision == B.RN_FP64 else 1e-8)
    assert r.converged and r.iters == 0
    assert r.K == pytest.approx(0.6, rel=1e-12)
    r0, _, _ = B.solve_network(ctx, net, precision, 1e-10 if precision == B.RN_FP64 else 1e-8, x0=B.RN_X0_ZERO)
    assert r0.converged and r0.iters > 0
    assert r0.K == pytest.approx(0.6, rel=1e-9 if precision == B.RN_FP64 else 1e-7)


@pytest.mark.timeout(240)
def test_budget_held_by_an_idle_slab_is_released():
    """Budget 1.5 GiB: a small solve leaves a 1 GiB slab behind; a request of
    about 1.2 GiB must still be admitted (synchronously and through the
    server), not wait for memory that nothing will return."""
    gib = 1 << 30
    budget = int(1.5 * gib)
    small = I.uniform_network(2, 64, 64, g0=1.0)
    side = 3400
    big = I.uniform_network(2, side, side, g0=2.0)
    fp = B.rn_footprint(B.problem(big), B.opts(B.RN_FP64))
    assert gib < fp < budget, fp
    for served in (False, True):
        c = B.Context(0, hbm_budget_bytes=budget)
        try:
            t0 = time.time()
            for net, g0 in ((small, 1.0), (big, 2.0)):
                say(f"budget test served={served}: {net.shape}")
                if served:
                    t = c.submit(B.problem(net), B.opts(B.RN_FP64, 1e-10))
                    while True:
                        st, r = c.poll(t)
                        if st != B.RN_EAGAIN:
                            break
                        assert time.time() - t0 < 120, "request never admitted"
                        time.sleep(0.002)
                    assert st == B.RN_OK
                else:
                    r = c.solve(B.problem(net), B.opts(B.RN_FP64, 1e-10))
                assert r.converged and r.K == pytest.approx(g0, rel=1e-12)
                assert c.stats()["bytes_in_use"] == 0
        finally:
            c.close()
