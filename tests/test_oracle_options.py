"""Pins of the oracle's solver options and of its stopping branches (CPU).

The initial guess (x = 0 or the linear profile along the flow axis) and the
preconditioner (Jacobi or none) change the path of the iteration but not the
solution of Eq. 3, which is unique on the live set (Sec. II). Each option is
pinned to something other than the oracle itself:

* the linear profile is the exact solution of a uniform network with no-flow
  sides (closed form), so the solve starts converged;
* every combination reaches the dense direct solve of the same system
  (numpy's LU on the assembled Kirchhoff matrix, tests/_pins.py);
* on a one-row network the matrix is irreducible tridiagonal, so its
  eigenvalues are distinct and CG ends in at most as many steps as there are
  unknowns (finite termination, Hestenes-Stiefel), with either option;
* the iteration counts with and without the Jacobi preconditioner are those
  of scipy's CG on the same system, assembled independently from the bonds;
* the stopping branch that continues from the recomputed true residual when
  the recurrence has drifted below it, and stops once that residual no longer
  halves, is driven at tolerances below the FP64 rounding floor.
"""
import numpy as np
import pytest

from paper_1908_03301_amd import inputs as I
from tests import _pins

COMBOS = [(x0, pc) for x0 in (0, 1) for pc in (0, 1)]   # (X0_LINEAR / X0_ZERO, JACOBI / NONE)


@pytest.mark.parametrize("dim,shape,axis", [(2, (17, 9, 1), 0), (2, (6, 23, 1), 1), (3, (7, 5, 9), 2),
                                            (3, (12, 4, 3), 0)])
def test_linear_guess_is_exact_on_uniform_networks(oracle_mod, dim, shape, axis):
    net = I.uniform_network(dim, *shape, g0=1.75, axis=axis)
    for pc in (oracle_mod.JACOBI, oracle_mod.NONE):
        r = oracle_mod.solve(net, tol=1e-12, x0=oracle_mod.X0_LINEAR, precond=pc)
        assert r.converged and r.status == 0 and r.iters == 0
        assert r.rel_resid <= 1e-14
        assert r.K == pytest.approx(1.75, rel=1e-14)
        # from x = 0 the same solve needs iterations
        r0 = oracle_mod.solve(net, tol=1e-12, x0=oracle_mod.X0_ZERO, precond=pc)
        assert r0.iters > 0 and r0.K == pytest.approx(1.75, rel=1e-11)


@pytest.mark.parametrize("case", range(5))
def test_every_option_reaches_the_dense_solution(oracle_mod, case):
    dim = 2 if case < 3 else 3
    nx, ny, nz = [(10, 9, 1), (8, 10, 1), (10, 6, 1), (5, 5, 4), (4, 5, 5)][case]
    occ = [1.0, 0.7, 0.62, 0.9, 0.5][case]
    base = I.fbm_network(dim, nx, ny, nz, H=0.7, sigma=2.0, occupancy=occ, index=140 + case)
    for axis in range(dim):
        net = base.with_axis(axis)
        P_ref, Q_ref = _pins.dense_solve(net)
        K_ref = Q_ref * (_pins.axis_len(net) - 1) / _pins.cross_section(net)
        for x0, pc in COMBOS:
            r = oracle_mod.solve(net, tol=1e-14, x0=x0, precond=pc)
            assert r.status in (0, -3), (x0, pc, r.status)
            assert r.rel_resid <= 1e-13
            np.testing.assert_allclose(r.pressure, P_ref, rtol=0, atol=1e-11)
            assert r.K == pytest.approx(K_ref, rel=1e-11, abs=1e-14)


@pytest.mark.parametrize("m,uniform", [(7, True), (12, True), (40, True), (25, False), (40, False)])
def test_cg_terminates_in_n_unknowns_steps_on_a_chain(oracle_mod, m, uniform):
    """One row of m + 2 nodes: A is an irreducible symmetric tridiagonal
    matrix, so its m eigenvalues are distinct, b has a component on each
    eigenvector, and CG (with or without the Jacobi scaling, which keeps the
    matrix tridiagonal and irreducible) needs exactly m steps in exact
    arithmetic. In FP64 the Jacobi-scaled chains and the uniform chain end at
    step m; the unscaled random chain is more ill-conditioned and shows the
    usual finite-precision delay of a few steps."""
    rng = np.random.default_rng(m)
    g = np.full((1, m + 2), 0.8) if uniform else np.exp(rng.normal(0.0, 0.5, (1, m + 2)))
    g[0, -1] = 0.0
    net = I.Network(2, m + 2, 1, 1, [g, np.zeros_like(g)], 0)
    K_ref = (m + 1) / np.sum(1.0 / g[0, : m + 1])
    for pc in (oracle_mod.JACOBI, oracle_mod.NONE):
        r = oracle_mod.solve(net, tol=1e-8, x0=oracle_mod.X0_ZERO, precond=pc)
        assert r.converged and r.K == pytest.approx(K_ref, rel=1e-12)
        if uniform or pc == oracle_mod.JACOBI:
            assert r.iters == m, (pc, r.iters)
        else:
            assert m <= r.iters <= m + m // 5, (pc, r.iters)


def _live_system(net):
    """The Kirchhoff system on the live set, assembled from the bond list
    (tests/_pins.py), as a scipy sparse matrix, its right-hand side and its
    diagonal."""
    import scipy.sparse as sp
    Ib, Jb, Gv = _pins.bond_list(net)
    f = _pins.faces(net)
    m = _pins.mask_scipy(net).ravel()
    live = np.nonzero(m == 3)[0]
    pos = -np.ones(net.n, dtype=np.int64)
    pos[live] = np.arange(live.size)
    rows, cols, vals = [], [], []
    diag = np.zeros(live.size)
    b = np.zeros(live.size)
    for a, c, g in zip(Ib, Jb, Gv):
        if g <= 0:
            continue
        for u, v in ((a, c), (c, a)):
            if pos[u] < 0:
                continue
            diag[pos[u]] += g
            if pos[v] >= 0:
                rows.append(pos[u])
                cols.append(pos[v])
                vals.append(-g)
            elif f[v] == 1:
                b[pos[u]] += g
    A = sp.csr_matrix((vals, (rows, cols)), shape=(live.size, live.size)) + sp.diags(diag)
    return A, b, diag


@pytest.mark.parametrize("case", range(3))
def test_iteration_counts_match_scipy_cg(oracle_mod, case):
    """From x = 0 with and without the Jacobi preconditioner, the oracle takes
    the iteration count of scipy.sparse.linalg.cg on the same system (stopping
    rules differ by the oracle's true-residual check, and rounding by 2%). The two
    preconditioners take visibly different counts on these networks, so the
    option really switches the preconditioner."""
    from scipy.sparse.linalg import cg
    nx, ny, occ, sigma = [(40, 30, 0.8, 2.0), (33, 41, 1.0, 3.0), (50, 20, 0.65, 1.5)][case]
    net = I.fbm_network(2, nx, ny, 1, H=0.6, sigma=sigma, occupancy=occ, index=160 + case)
    A, b, diag = _live_system(net)
    counts = {}
    for pc in (oracle_mod.JACOBI, oracle_mod.NONE):
        n_it = [0]

        def cb(_):
            n_it[0] += 1

        M = None if pc == oracle_mod.NONE else __import__("scipy.sparse", fromlist=["diags"]).diags(1.0 / diag)
        x, info = cg(A, b, rtol=1e-10, atol=0.0, M=M, maxiter=100_000, callback=cb)
        assert info == 0
        r = oracle_mod.solve(net, tol=1e-10, x0=oracle_mod.X0_ZERO, precond=pc)
        assert r.converged
        assert abs(r.iters - n_it[0]) <= 2 + 0.02 * n_it[0], (pc, r.iters, n_it[0])
        counts[pc] = r.iters
    assert abs(counts[oracle_mod.JACOBI] - counts[oracle_mod.NONE]) > 0.1 * counts[oracle_mod.JACOBI]


def test_options_are_validated(oracle_mod):
    net = I.uniform_network(2, 6, 5)
    for kw in ({"x0": 2}, {"precond": -1}, {"precond": 2}):
        with pytest.raises(oracle_mod.OracleError) as e:
            oracle_mod.solve(net, **kw)
        assert e.value.code == -1


def test_restart_from_true_residual_and_stagnation_stop(oracle_mod):
    """sigma = 3.5 on 40 x 30: conductances over about six orders of magnitude,
    so the recurrence residual drifts below the true one near 1e-12.

    At tol 3e-12 the first true-residual check fails and the next one does
    not halve it: the solve stops there (not converged) with the true
    residual reported. At tol 1e-12 the solve continues from the recomputed
    true residual with a fresh direction and converges: more iterations than
    the stagnating run, true residual (re-evaluated independently) below tol.
    Below the rounding floor (tol 1e-18) the solve stops by stagnation long
    before max_iter, and K is still that of the converged solve."""
    net = I.fbm_network(2, 40, 30, 1, H=0.5, sigma=3.5, occupancy=0.8, index=2)
    stag = oracle_mod.solve(net, tol=3e-12, max_iter=200_000)
    assert stag.status == -3 and not stag.converged
    c = oracle_mod.check_pressure(net, stag.pressure)
    assert c.rel_resid == pytest.approx(stag.rel_resid, rel=1e-6)
    assert stag.rel_resid > 3e-12

    conv = oracle_mod.solve(net, tol=1e-12, max_iter=200_000)
    assert conv.status == 0 and conv.converged
    assert conv.iters > stag.iters
    c = oracle_mod.check_pressure(net, conv.pressure)
    assert c.rel_resid <= 1e-12

    floor = oracle_mod.solve(net, tol=1e-18, max_iter=200_000)
    assert floor.status == -3 and not floor.converged
    assert floor.iters < 10 * conv.iters
    assert floor.rel_resid < 1e-10
    assert floor.K == pytest.approx(conv.K, rel=1e-10)
