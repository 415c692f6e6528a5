"""Pins of the oracle's backbone (Sec. VI: the spanning cluster near p_c).

The backbone is the set of interior nodes on some inlet-outlet path that
visits no node twice; dangling ends (branches and loops joined to the rest
through one node) carry no flow. The oracle finds it with Hopcroft and
Tarjan's biconnected components. It is held here to things other than itself:
  - a network built and worked out by hand, with a dangling loop (which a
    leaf-stripping "burning" method would keep) and a dangling branch;
  - a brute-force vertex-cut check (Menger's theorem) on tiny 2D and 3D
    lattices, diluted near and above the threshold, with periodic sides
    (also of extent 2, where two bonds join the same pair of nodes) and with
    3 planes on the flow axis, where a node touches both faces;
  - the physics, with a dense direct solve of Eq. 3: no bond of a live node
    off the backbone carries current, and removing those nodes leaves Q
    unchanged and makes the live set equal to the backbone;
  - special cases: an undiluted lattice is all backbone; nothing is backbone
    without a spanning cluster or without interior nodes.
"""
import json
import os

import numpy as np
import pytest

from paper_1908_03301_amd import inputs as I
from tests import _pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _net(d):
    g = [np.ascontiguousarray(np.array(d["g_x"], dtype=np.float64)),
         np.ascontiguousarray(np.array(d["g_y"], dtype=np.float64))]
    return I.Network(d["dim"], d["nx"], d["ny"], d["nz"], g, d["axis"])


def test_backbone_hand_built(oracle_mod):
    d = json.load(open(os.path.join(GOLDEN, "hand_backbone_7x4.json")))
    m, nl, nb = oracle_mod.backbone(_net(d))
    np.testing.assert_array_equal(m, np.array(d["mask"], dtype=np.uint8))
    assert (nl, nb) == (d["n_live"], d["n_backbone"])


def tiny_networks():
    out = []
    for seed in range(100):     # the sizes where a wrong low-point rule shows (a few % of these)
        out.append(I.iid_network(2, 9, 8, 1, occupancy=0.6, index=90000 + seed))
        out.append(I.iid_network(3, 6, 5, 4, occupancy=0.4, index=91000 + seed))
        out.append(I.iid_network(2, 8, 8, 1, occupancy=0.62, index=92000 + seed, periodic=True))
    for seed in range(6):
        out.append(I.iid_network(2, 7, 6, 1, occupancy=0.62, index=4100 + seed))
        out.append(I.iid_network(2, 6, 7, 1, occupancy=0.75, index=4110 + seed, axis=1))
        out.append(I.iid_network(3, 5, 4, 3, occupancy=0.45, index=4120 + seed))
        out.append(I.iid_network(2, 6, 6, 1, occupancy=0.65, index=4130 + seed, periodic=True))
        out.append(I.iid_network(2, 7, 2, 1, occupancy=0.8, index=4140 + seed, periodic=True))     # extent 2
        out.append(I.iid_network(3, 4, 2, 3, occupancy=0.6, index=4150 + seed, periodic=True))
        out.append(I.iid_network(2, 3, 8, 1, occupancy=0.7, index=4160 + seed))                   # 3 planes
        out.append(I.fbm_network(2, 7, 7, 1, H=0.7, sigma=1.5, occupancy=0.6, index=4170 + seed))
    return out


def test_backbone_bruteforce(oracle_mod):
    seen_dangling = 0
    for net in tiny_networks():
        m, nl, nb = oracle_mod.backbone(net)
        want = _pins.backbone_bruteforce(net)
        got = (m & 8) != 0
        np.testing.assert_array_equal(got, want)
        mref, nlref = oracle_mod.mask_bfs(net)
        np.testing.assert_array_equal(m & 7, mref)          # the mask bits are mask_bfs's
        assert nl == nlref and nb == int(want.sum())
        assert np.all(mref[got] == 3)                        # the backbone is live
        seen_dangling += int(nl - nb)
    assert seen_dangling > 20                                # the cases do have dangling ends


@pytest.mark.parametrize("dim,shape,occ,periodic", [(2, (22, 16, 1), 0.58, False), (2, (18, 14, 1), 0.6, True),
                                                    (3, (8, 7, 6), 0.38, False), (3, (7, 6, 6), 0.42, True)])
def test_backbone_carries_all_flow(oracle_mod, dim, shape, occ, periodic):
    for seed in range(3):
        net = I.iid_network(dim, *shape, occupancy=occ, index=4200 + 10 * seed + dim, periodic=periodic)
        m, nl, nb = oracle_mod.backbone(net)
        P, Q = _pins.dense_solve(net)
        bb = ((m & 8) != 0).ravel()
        dangling = (m.ravel() == 3)
        i, j, g, cur = _pins.bond_currents(net, P)
        touches = dangling[i] | dangling[j]
        if nl:
            assert Q > 0
            assert np.max(np.abs(cur[touches]), initial=0.0) <= 1e-12 * Q
        # remove every live node off the backbone: same flux, and the live set is the backbone
        pruned = _pins.prune_dangling(net, m)
        assert pruned.periodic == periodic and all(not np.shares_memory(a, b) for a, b in zip(pruned.g, net.g))
        P2, Q2 = _pins.dense_solve(pruned)
        assert Q2 == pytest.approx(Q, rel=1e-12, abs=1e-300)
        m2, nl2 = oracle_mod.mask_bfs(pruned)
        np.testing.assert_array_equal(m2.ravel() == 3, bb)
        assert nl2 == nb


def test_backbone_special_cases(oracle_mod):
    full = I.uniform_network(2, 9, 6, 1, g0=1.0)
    m, nl, nb = oracle_mod.backbone(full)
    assert nl == nb == 7 * 6 and np.all(m[:, 1:-1] == 11)
    full3 = I.uniform_network(3, 5, 4, 3, g0=2.0, axis=2)
    m, nl, nb = oracle_mod.backbone(full3)
    assert nl == nb == 5 * 4
    two = I.iid_network(2, 2, 6, 1, occupancy=1.0, index=4300)        # no interior nodes
    m, nl, nb = oracle_mod.backbone(two)
    assert nl == nb == 0
    empty = I.iid_network(2, 40, 30, 1, occupancy=0.2, index=4301)   # far below the threshold
    m, nl, nb = oracle_mod.backbone(empty)
    assert nl == nb == 0 and not np.any(m & 8)
