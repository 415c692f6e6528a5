"""Pins of the oracle's periodic side boundaries (Sec. II: the pressure drop is
imposed along one direction, the other directions wrap around).

Each test checks the oracle against something other than itself: a
hand-solved network whose only conducting path crosses the wrap, closed forms
that periodicity leaves unchanged, a dense direct solve of Eq. 3 on the
periodic bond list, brute-force and scipy connectivity, invariance under a
translation along a periodic direction, and the reduction to no-flow sides
when every wrap bond is zero.
"""
import json
import os

import numpy as np
import pytest

from paper_1908_03301_amd import inputs as I
from tests import _pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rolled(net, k, shift):
    """The periodic network translated by `shift` planes along direction k."""
    ax = net.dim - 1 - k
    g = [np.ascontiguousarray(np.roll(a, shift, axis=ax)) for a in net.g]
    return I.Network(net.dim, net.nx, net.ny, net.nz, g, net.axis, {}, True)


def test_golden_wrap_path(oracle_mod):
    d = json.load(open(os.path.join(GOLDEN, "hand_periodic_3x3.json")))
    g = [np.array(d["g_x"]), np.array(d["g_y"])]
    for key, periodic in (("periodic", True), ("no_flow", False)):
        e = d[key]
        net = I.Network(2, d["nx"], d["ny"], 1, g, d["axis"], {}, periodic)
        r = oracle_mod.solve(net, tol=1e-14, want_mask=True)
        assert r.converged and r.n_live == e["n_live"]
        np.testing.assert_array_equal(r.mask, np.array(e["mask"], dtype=np.uint8))
        np.testing.assert_allclose(r.pressure, np.array(e["pressure"]), rtol=0, atol=1e-14)
        assert r.G == pytest.approx(e["G"], rel=1e-14, abs=1e-300)
        assert r.K == pytest.approx(e["K"], rel=1e-14, abs=1e-300)
        assert r.Q_in == pytest.approx(e["G"], rel=1e-14, abs=1e-300)


@pytest.mark.parametrize("dim,shape", [(2, (7, 5, 1)), (2, (4, 2, 1)), (2, (5, 1, 1)),
                                       (3, (5, 4, 3)), (3, (2, 3, 2)), (3, (4, 1, 5))])
def test_uniform_periodic_closed_form(oracle_mod, dim, shape):
    """Uniform g with wrapped sides: no transverse current, so K = g exactly."""
    nx, ny, nz = shape
    g0 = 1.75
    for axis in range(dim):
        net = I.uniform_network(dim, nx, ny, nz, g0=g0, axis=axis, periodic=True)
        na = _pins.axis_len(net)
        if na < 2:
            continue
        r = oracle_mod.solve(net, tol=1e-14)
        assert r.K == pytest.approx(g0, rel=1e-12)
        assert r.G == pytest.approx(g0 * _pins.cross_section(net) / (na - 1), rel=1e-12)


def test_stratified_periodic_unchanged(oracle_mod):
    """Rows of equal conductance: along x the rows stay parallel (arithmetic
    mean); along y every row is an equipotential, so the x wrap bonds carry no
    current and K_y stays the harmonic mean."""
    rng = np.random.default_rng(11)
    nx, ny = 8, 6
    c = np.exp(rng.normal(0, 1.5, ny))
    e = np.exp(rng.normal(0, 1.5, ny))
    gx = np.repeat(c[:, None], nx, axis=1)
    gy = np.repeat(e[:, None], nx, axis=1)
    net = I.Network(2, nx, ny, 1, [gx, gy], 0, {}, True)
    assert oracle_mod.solve(net, tol=1e-14).K == pytest.approx(c.mean(), rel=1e-12)
    ry = oracle_mod.solve(net.with_axis(1), tol=1e-14)
    assert ry.K == pytest.approx(1.0 / np.mean(1.0 / e[: ny - 1]), rel=1e-12)


CASES = [
    (2, 6, 5, 1, 0, 0.7), (2, 5, 6, 1, 1, 0.6), (2, 7, 2, 1, 0, 0.8), (2, 2, 7, 1, 1, 0.9),
    (3, 4, 3, 3, 0, 0.6), (3, 3, 4, 3, 1, 0.55), (3, 3, 3, 4, 2, 0.6), (3, 4, 2, 2, 0, 0.8),
]


@pytest.mark.parametrize("case", CASES)
def test_periodic_matches_dense(oracle_mod, case):
    dim, nx, ny, nz, axis, occ = case
    for idx in range(3):
        net = I.iid_network(dim, nx, ny, nz, sigma=1.0, occupancy=occ, index=300 + idx,
                            axis=axis, periodic=True)
        P, Qin = _pins.dense_solve(net)
        r = oracle_mod.solve(net, tol=1e-14)
        assert r.converged
        np.testing.assert_allclose(r.pressure, P, rtol=0, atol=1e-10)
        assert r.Q_in == pytest.approx(Qin, rel=1e-10, abs=1e-14)
        assert r.G == pytest.approx(Qin, rel=1e-10, abs=1e-14)


@pytest.mark.parametrize("case", CASES)
def test_periodic_masks_agree(oracle_mod, case):
    dim, nx, ny, nz, axis, _ = case
    for occ in (0.35, 0.5, 0.65):
        net = I.iid_network(dim, nx, ny, nz, occupancy=occ, index=400, axis=axis, periodic=True)
        mb, nb = oracle_mod.mask_bfs(net)
        mu, nu = oracle_mod.mask_uf(net)
        np.testing.assert_array_equal(mb, mu)
        np.testing.assert_array_equal(mb, _pins.mask_scipy(net))
        np.testing.assert_array_equal(mb, _pins.mask_bruteforce(net))
        assert nb == nu == int((mb == 3).sum())


def test_periodic_links_more_than_no_flow(oracle_mod):
    """The wrap can only join components: every node live without it stays live."""
    for idx in range(6):
        net = I.iid_network(2, 12, 9, 1, occupancy=0.55, index=500 + idx, periodic=True)
        mp, _ = oracle_mod.mask_bfs(net)
        mn, _ = oracle_mod.mask_bfs(net.with_periodic(False))
        assert np.all(mp[mn == 3] == 3)
        assert np.all((mp & mn) == mn)


@pytest.mark.parametrize("dim,shape,axis", [(2, (20, 17, 1), 0), (2, (15, 21, 1), 1),
                                            (3, (9, 8, 7), 0), (3, (7, 9, 8), 2)])
def test_translation_invariance(oracle_mod, dim, shape, axis):
    """Translating a periodic network along a wrapped direction moves the
    wrap to other bonds but leaves K unchanged and shifts the solution."""
    nx, ny, nz = shape
    net = I.fbm_network(dim, nx, ny, nz, H=0.7, sigma=1.5, occupancy=0.75, index=600, axis=axis,
                        periodic=True)
    r0 = oracle_mod.solve(net, tol=1e-13, want_mask=True)
    assert r0.converged and r0.n_live > 0
    for k in range(dim):
        if k == axis:
            continue
        for shift in (1, 3):
            rs = oracle_mod.solve(_rolled(net, k, shift), tol=1e-13, want_mask=True)
            ax = dim - 1 - k
            np.testing.assert_array_equal(rs.mask, np.roll(r0.mask, shift, axis=ax))
            assert rs.K == pytest.approx(r0.K, rel=1e-10)
            np.testing.assert_allclose(rs.pressure, np.roll(r0.pressure, shift, axis=ax), rtol=0, atol=1e-9)
    # the same translation without periodic sides generally changes K
    moved = _rolled(net, 1 if axis == 0 else 0, 3).with_periodic(False)
    assert oracle_mod.solve(moved, tol=1e-13).K != pytest.approx(r0.K, rel=1e-6)


def test_zero_wrap_bonds_reduce_to_no_flow(oracle_mod):
    for dim, shape, axis in ((2, (11, 9, 1), 1), (3, (6, 5, 4), 2)):
        net = I.fbm_network(dim, *shape, H=0.7, sigma=1.0, occupancy=0.8, index=700, axis=axis)
        per = net.with_periodic(True)      # generated without wrap bonds: their entries are 0
        a = oracle_mod.solve(net, tol=1e-13, want_mask=True)
        b = oracle_mod.solve(per, tol=1e-13, want_mask=True)
        np.testing.assert_array_equal(a.mask, b.mask)
        assert a.K == b.K and a.iters == b.iters


def test_periodic_validation(oracle_mod):
    net = I.iid_network(2, 6, 5, 1, index=800, periodic=True)
    gy = net.g[1].copy()
    gy[-1, 2] = np.nan                                   # a wrap bond along y
    bad = I.Network(2, 6, 5, 1, [net.g[0], gy], 0, {}, True)
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.solve(bad)
    assert e.value.code == -1                            # rejected as invalid input
    oracle_mod.solve(bad.with_periodic(False))           # ignored without wrap
    gx = net.g[0].copy()
    gx[1, -1] = np.nan                                   # last-plane entry along the flow axis
    oracle_mod.solve(I.Network(2, 6, 5, 1, [gx, net.g[1]], 0, {}, True))
