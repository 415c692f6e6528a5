"""Property-based pins of the oracle on random tiny lattices (hypothesis).

For any small 2D or 3D network with random dilution and conductances:
the BFS mask equals the union-find mask and scipy's connected components;
the pressures solve the dense Kirchhoff system; the energy conductance
equals the flux; reflecting the lattice along the flow axis leaves G
unchanged.
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from paper_1908_03301_amd import inputs as I
from tests import _pins


@st.composite
def networks(draw):
    dim = draw(st.sampled_from([2, 3]))
    nx = draw(st.integers(2, 7))
    ny = draw(st.integers(1, 6))
    nz = draw(st.integers(1, 4)) if dim == 3 else 1
    axis = draw(st.integers(0, dim - 1))
    if (nx, ny, nz)[axis] < 2:
        axis = 0
    seed = draw(st.integers(0, 2**31 - 1))
    occ = draw(st.floats(0.3, 1.0))
    rng = np.random.default_rng(seed)
    shape = I.node_shape(dim, nx, ny, nz)
    g = [np.exp(rng.normal(0.0, 1.5, shape)) * (rng.random(shape) < occ) for _ in range(dim)]
    return I.Network(dim, nx, ny, nz, I.clear_edge_bonds(g), axis)


SETTINGS = settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])


@SETTINGS
@given(networks())
def test_mask_agrees_everywhere(oracle_mod, net):
    mb, nb = oracle_mod.mask_bfs(net)
    mu, nu = oracle_mod.mask_uf(net)
    ms = _pins.mask_scipy(net)
    np.testing.assert_array_equal(mb, ms)
    np.testing.assert_array_equal(mu, ms)
    assert nb == nu == int((ms == 3).sum())


@SETTINGS
@given(networks())
def test_solution_matches_dense_and_energy(oracle_mod, net):
    P_ref, Q_ref = _pins.dense_solve(net)
    r = oracle_mod.solve(net, tol=1e-13)
    np.testing.assert_allclose(r.pressure, P_ref, atol=1e-9)
    assert r.G == pytest.approx(Q_ref, rel=1e-9, abs=1e-12)
    assert r.Q_out == pytest.approx(r.Q_in, rel=1e-8, abs=1e-12)
