"""GPU parity of rn_build_backbone with the oracle (Sec. VI: the spanning cluster near p_c).

The device finds the backbone with a breadth-first spanning tree and Tarjan
and Vishkin's joins; the oracle with Hopcroft and Tarjan's depth-first
search. The masks must agree bit for bit (the backbone is unique, whatever
tree the device's races build), with the live and backbone counts:
  - diluted 2D and 3D networks near and above the threshold, i.i.d. and FBM,
    each flow axis, periodic sides (also of extent 2, with two bonds between
    the same nodes), 3 planes on the flow axis, host and device inputs, sizes
    from one workgroup to many;
  - the edge cases: an undiluted lattice (all backbone), nothing spanning,
    2 planes on the flow axis (no interior node);
  - the two single-network workloads at full size: the 2048^2 FBM network at
    occupancy 0.6 and the 256^3 layered network at occupancy 0.27.
The physics on the GPU: solving the network with its off-backbone live nodes
removed gives the same K (dangling ends carry no flow), and the GPU mask of
that pruned network has the backbone as its live set.
"""
import sys

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
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = B.Context(0)
    yield c
    c.close()


def cases():
    return [
        ("iid 2D 300x257 p0.55", I.iid_network(2, 300, 257, 1, occupancy=0.55, index=5100)),
        ("iid 2D 257x300 p0.53 axis y", I.iid_network(2, 257, 300, 1, occupancy=0.53, index=5101, axis=1)),
        ("fbm 2D 512x384 occ0.6", I.fbm_network(2, 512, 384, 1, H=0.7, sigma=1.5, occupancy=0.6, index=5102)),
        ("iid 3D 64x48x40 p0.3", I.iid_network(3, 64, 48, 40, occupancy=0.3, index=5103)),
        ("iid 3D 40x50x60 p0.28 axis z", I.iid_network(3, 40, 50, 60, occupancy=0.28, index=5104, axis=2)),
        ("fbm 3D 48^3 occ0.35", I.fbm_network(3, 48, 48, 48, H=0.7, sigma=1.0, occupancy=0.35, index=5105)),
        ("periodic 2D 200x150 p0.55", I.iid_network(2, 200, 150, 1, occupancy=0.55, index=5106, periodic=True)),
        ("periodic 2D 300x2 p0.8", I.iid_network(2, 300, 2, 1, occupancy=0.8, index=5107, periodic=True)),
        ("periodic 3D 30x2x20 p0.5", I.iid_network(3, 30, 2, 20, occupancy=0.5, index=5108, periodic=True)),
        ("periodic 3D 40^3 p0.3", I.iid_network(3, 40, 40, 40, occupancy=0.3, index=5109, periodic=True)),
        ("3 planes 3x500 p0.7", I.iid_network(2, 3, 500, 1, occupancy=0.7, index=5110)),
        ("tiny 7x6 p0.62", I.iid_network(2, 7, 6, 1, occupancy=0.62, index=4100)),
        ("uniform 2D 90x70", I.uniform_network(2, 90, 70, 1, g0=1.5)),
        ("uniform 3D 20x18x16", I.uniform_network(3, 20, 18, 16, g0=1.0, axis=1)),
        ("nothing spans 2D p0.3", I.iid_network(2, 200, 200, 1, occupancy=0.3, index=5111)),
        ("2 planes 2x50", I.iid_network(2, 2, 50, 1, occupancy=0.9, index=5112)),
    ]


@pytest.mark.parametrize("label,net", cases(), ids=[c[0] for c in cases()])
def test_backbone_against_oracle(ctx, oracle_mod, label, net):
    say(f"rn_build_backbone {label}")
    M, nl, nb = B.backbone_network(ctx, net)
    ref, nlr, nbr = oracle_mod.backbone(net)
    say(f"{label}: live {nl} backbone {nb} (oracle {nlr} {nbr})")
    np.testing.assert_array_equal(M, ref)
    assert (nl, nb) == (nlr, nbr)


def test_backbone_device_input_and_repeat(ctx, oracle_mod):
    import torch
    net = I.iid_network(2, 400, 300, 1, occupancy=0.54, index=5120)
    ref, nlr, nbr = oracle_mod.backbone(net)
    g = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in net.g]
    m = torch.zeros(net.shape, dtype=torch.uint8, device="cuda")
    for rep in range(3):
        m.zero_()
        nl, nb = ctx.build_backbone(B.problem(dim=2, nx=net.nx, ny=net.ny, g=g, mask_out=m))
        np.testing.assert_array_equal(m.cpu().numpy(), ref)
        assert (nl, nb) == (nlr, nbr)


def _prune(net, M):
    """The network with every live node off the backbone cut out (its bonds set to 0)."""
    dangling = M == 3
    gp = [np.array(a, copy=True) for a in net.g]
    for k in range(net.dim):
        ax = net.dim - 1 - k
        gp[k][dangling] = 0.0
        gp[k][np.roll(dangling, -1, axis=ax)] = 0.0
    return I.Network(net.dim, net.nx, net.ny, net.nz, gp, net.axis, periodic=net.periodic)


@pytest.mark.parametrize("net", [I.iid_network(2, 256, 256, 1, occupancy=0.55, index=5130),
                                 I.fbm_network(3, 48, 40, 36, H=0.7, sigma=1.0, occupancy=0.33, index=5131),
                                 I.iid_network(2, 200, 160, 1, occupancy=0.56, index=5132, periodic=True)])
def test_backbone_carries_the_flow(ctx, net):
    M, nl, nb = B.backbone_network(ctx, net)
    assert 0 < nb < nl
    pruned = _prune(net, M)
    r0, _, _ = B.solve_network(ctx, net, B.RN_FP64, 1e-11)
    r1, _, M1 = B.solve_network(ctx, pruned, B.RN_FP64, 1e-11, want_mask=True)
    say(f"live {nl} backbone {nb}: K {r0.K:.12g} pruned {r1.K:.12g} iters {r0.iters} -> {r1.iters}")
    assert r0.converged and r1.converged
    assert r1.K == pytest.approx(r0.K, rel=1e-9)
    np.testing.assert_array_equal(M1 == 3, (M & 8) != 0)
    assert r1.n_live == nb


@pytest.mark.parametrize("make", [I.workload_fbm_2d_2048, I.workload_strat_3d_256],
                         ids=["fbm2d_2048", "strat3d_256"])
def test_backbone_full_size(ctx, oracle_mod, make):
    net = make()
    say(f"full-size backbone: {net.meta.get('desc', '')} {net.shape}")
    M, nl, nb = B.backbone_network(ctx, net)
    ref, nlr, nbr = oracle_mod.backbone(net)
    say(f"live {nl} backbone {nb} (oracle {nlr} {nbr})")
    assert (nl, nb) == (nlr, nbr)
    np.testing.assert_array_equal(M, ref)


# ------------------------------------------------------------------ solves on the backbone (RN_OPT_BACKBONE)

TOL = {B.RN_FP64: 1e-10, B.RN_MIXED: 1e-8}
KBAR = {B.RN_FP64: 1e-9, B.RN_MIXED: 1e-7}


def bb_cases():
    return [
        ("iid 2D 300x257 p0.55 mixed", I.iid_network(2, 300, 257, 1, occupancy=0.55, index=5100), B.RN_MIXED),
        ("iid 2D 257x300 p0.53 axis y fp64", I.iid_network(2, 257, 300, 1, occupancy=0.53, index=5101, axis=1),
         B.RN_FP64),
        ("fbm 3D 48^3 occ0.35 mixed", I.fbm_network(3, 48, 48, 48, H=0.7, sigma=1.0, occupancy=0.35, index=5105),
         B.RN_MIXED),
        ("periodic 2D 200x150 p0.55 mixed", I.iid_network(2, 200, 150, 1, occupancy=0.55, index=5106,
                                                          periodic=True), B.RN_MIXED),
        ("periodic 3D 40^3 p0.3 fp64", I.iid_network(3, 40, 40, 40, occupancy=0.3, index=5109, periodic=True),
         B.RN_FP64),
        ("nothing spans 2D p0.3 mixed", I.iid_network(2, 200, 200, 1, occupancy=0.3, index=5111), B.RN_MIXED),
        ("2 planes 2x50 fp64", I.iid_network(2, 2, 50, 1, occupancy=0.9, index=5112), B.RN_FP64),
    ]


@pytest.mark.parametrize("label,net,prec", bb_cases(), ids=[c[0] for c in bb_cases()])
def test_backbone_option_against_oracle(ctx, oracle_mod, label, net, prec):
    """K, every pressure and the backbone mask of a solve on the backbone against the oracle's
    solve of the whole network."""
    from tests import _pins
    say(f"RN_OPT_BACKBONE {label}")
    r, P, M = B.solve_network(ctx, net, prec, TOL[prec], want_pressure=True, want_mask=True, backbone=True)
    r0, _, _ = B.solve_network(ctx, net, prec, TOL[prec])
    mref, nl, nb = oracle_mod.backbone(net)
    ref = oracle_mod.solve(net, tol=1e-13)
    say(f"{label}: live {r.n_live} backbone {r.n_backbone} K {r.K:.12g} oracle {ref.K:.12g} "
        f"iters {r0.iters} -> {r.iters}")
    np.testing.assert_array_equal(M, mref)
    assert (r.n_live, r.n_backbone) == (nl, nb)
    assert r.status == 0 and r.converged
    if nl == 0:
        assert r.K == pytest.approx(ref.K, rel=1e-12, abs=1e-300) and r.iters == 0
        return
    assert r.K == pytest.approx(ref.K, rel=KBAR[prec])
    # the filled field solves the whole network: its true residual, its energy, its pressures
    c = oracle_mod.check_pressure(net, P)
    assert c.rel_resid <= 1.01 * TOL[prec]
    assert r.G == pytest.approx(c.G_E, rel=1e-9)
    live = (mref.ravel() & 3) == 3                # live nodes: backbone (11) and dangling (3)
    R = _pins.face_path_resistance(net).ravel()[live]
    eps = _pins.pressure_error_bound(R, _pins.energy(net, P), ref.G)
    err = np.abs(P.ravel()[live] - ref.pressure.ravel()[live])
    assert np.all(err <= eps), float(np.max(err - eps))


def test_backbone_option_device_memory_and_batch(ctx):
    """Device buffers, and a batch mixing solves on the backbone with plain ones: each result and
    pressure field equals the same solve made alone."""
    import torch
    nets = [I.iid_network(2, 220, 180, 1, occupancy=0.55, index=5140),
            I.fbm_network(2, 300, 240, 1, H=0.7, sigma=1.5, occupancy=0.6, index=5141),
            I.iid_network(3, 40, 36, 30, occupancy=0.3, index=5142)]
    flags = [True, False, True]
    solo = []
    for net, bb in zip(nets, flags):
        solo.append(B.solve_network(ctx, net, B.RN_MIXED, 1e-8, want_pressure=True, want_mask=True, backbone=bb))
    gs = [[torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in n.g] for n in nets]
    Ps = [torch.zeros(n.shape, dtype=torch.float64, device="cuda") for n in nets]
    Ms = [torch.zeros(n.shape, dtype=torch.uint8, device="cuda") for n in nets]
    probs = [B.problem(dim=n.dim, nx=n.nx, ny=n.ny, nz=n.nz, axis=n.axis, g=g, p_out=P, mask_out=M)
             for n, g, P, M in zip(nets, gs, Ps, Ms)]
    res = ctx.solve_batch(probs, [B.opts(B.RN_MIXED, 1e-8, backbone=bb) for bb in flags])
    for (r0, P0, M0), r, P, M in zip(solo, res, Ps, Ms):
        for f in ("status", "converged", "K", "G", "Q_in", "Q_out", "iters", "n_live", "n_backbone"):
            assert getattr(r0, f) == getattr(r, f), f
        assert P0.tobytes() == P.cpu().numpy().tobytes()
        np.testing.assert_array_equal(M0, M.cpu().numpy())
    assert res[1].n_backbone == 0 and res[0].n_backbone > 0


def test_backbone_option_rejected_by_submit(ctx):
    net = I.iid_network(2, 64, 64, 1, occupancy=0.6, index=5150)
    with pytest.raises(B.RNError):
        ctx.submit(B.problem(net), B.opts(B.RN_MIXED, 1e-8, backbone=True))
