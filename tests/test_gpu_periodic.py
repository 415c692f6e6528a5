"""GPU parity with periodic side boundaries (RN_PERIODIC, Sec. II): librn
against the CPU oracle through the C ABI, on lattices whose extents put the
wrap at every position a tile can meet it (inside a wave, on a wave or
workgroup edge, on a tile of one column, across 2 planes).

Bars as for no-flow sides: mask bit-exact, K within 1e-9 (FP64) / 1e-7
(mixed) of the oracle solved to 1e-13, the returned field's true residual
(evaluated by the oracle) within tol.
"""
import json
import os

import numpy as np
import pytest

from paper_1908_03301_amd import binding as B
from paper_1908_03301_amd import inputs as I
from tests import _pins
from tests.test_gpu_parity import K_TOL, SOLVE_TOL, check_against_oracle, ctx, gpu_solve, say  # noqa: F401

pytestmark = pytest.mark.gpu

PRECS = [B.RN_FP64, B.RN_MIXED]


@pytest.mark.parametrize("precision", PRECS)
def test_golden_wrap_path(ctx, precision):
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_periodic_3x3.json")))
    g = [np.array(d["g_x"]), np.array(d["g_y"])]
    for key, periodic in (("periodic", True), ("no_flow", False)):
        e = d[key]
        net = I.Network(2, d["nx"], d["ny"], 1, g, d["axis"], {}, periodic)
        res, P, M = gpu_solve(ctx, net, precision, tol=1e-12)
        assert res.n_live == e["n_live"]
        np.testing.assert_array_equal(M, np.array(e["mask"], dtype=np.uint8))
        np.testing.assert_allclose(P, np.array(e["pressure"]), atol=1e-11)
        assert res.K == pytest.approx(e["K"], rel=1e-11, abs=1e-300)


# 2D extents: a wave holds 64 columns and 8 (FP32) or 4 (FP64) rows, a
# workgroup 4 waves stacked in y
SHAPES_2D = [(130, 70), (64, 32), (128, 16), (40, 33), (2, 50), (300, 2), (65, 9), (63, 8), (192, 31)]


@pytest.mark.parametrize("shape", SHAPES_2D)
@pytest.mark.parametrize("precision", PRECS)
def test_periodic_2d(ctx, oracle_mod, shape, precision):
    nx, ny = shape
    base = I.fbm_network(2, nx, ny, 1, H=0.7, sigma=1.5, occupancy=0.7, index=900 + nx + ny, periodic=True)
    for axis in range(2):
        net = base.with_axis(axis)
        if _pins.axis_len(net) < 2:
            continue
        res, P, M = gpu_solve(ctx, net, precision)
        check_against_oracle(oracle_mod, net, res, P, M, precision)


SHAPES_3D = [(67, 35, 20), (16, 16, 3), (5, 70, 18), (64, 16, 16), (33, 17, 2), (2, 40, 30), (65, 17, 33)]


@pytest.mark.parametrize("shape", SHAPES_3D)
@pytest.mark.parametrize("precision", PRECS)
def test_periodic_3d(ctx, oracle_mod, shape, precision):
    nx, ny, nz = shape
    base = I.fbm_network(3, nx, ny, nz, H=0.7, sigma=1.0, occupancy=0.6, index=950 + nx + ny + nz,
                         periodic=True)
    for axis in range(3):
        net = base.with_axis(axis)
        res, P, M = gpu_solve(ctx, net, precision)
        check_against_oracle(oracle_mod, net, res, P, M, precision)


@pytest.mark.parametrize("precision", PRECS)
def test_periodic_uniform_and_translation(ctx, precision):
    """K = g for uniform periodic lattices; a periodic network translated
    along a wrapped direction keeps its K."""
    for dim, shape in ((2, (70, 45, 1)), (3, (20, 18, 17))):
        for axis in range(dim):
            net = I.uniform_network(dim, *shape, g0=1.75, axis=axis, periodic=True)
            res, _, _ = gpu_solve(ctx, net, precision)
            assert res.K == pytest.approx(1.75, rel=K_TOL[precision])
    net = I.fbm_network(2, 150, 90, 1, H=0.7, sigma=1.5, occupancy=0.7, index=990, periodic=True)
    r0, _, M0 = gpu_solve(ctx, net, precision)
    g = [np.ascontiguousarray(np.roll(a, 37, axis=0)) for a in net.g]       # shift along y
    moved = I.Network(2, 150, 90, 1, g, 0, {}, True)
    r1, _, M1 = gpu_solve(ctx, moved, precision)
    np.testing.assert_array_equal(M1, np.roll(M0, 37, axis=0))
    assert r1.K == pytest.approx(r0.K, rel=2 * K_TOL[precision])


def test_periodic_device_memory_and_build_mask(ctx, oracle_mod):
    import torch
    net = I.fbm_network(3, 40, 30, 20, H=0.7, sigma=1.0, occupancy=0.45, index=995, axis=2, periodic=True)
    gd = [torch.from_numpy(a).cuda() for a in net.g]
    Md = torch.zeros(net.shape, dtype=torch.uint8, device="cuda")
    say("rn_build_mask, periodic, device memory")
    n_live = ctx.build_mask(B.problem(dim=3, nx=40, ny=30, nz=20, axis=2, g=gd, mask_out=Md, periodic=True))
    ref, nl = oracle_mod.mask_bfs(net)
    np.testing.assert_array_equal(Md.cpu().numpy(), ref)
    assert n_live == nl
    res = ctx.solve(B.problem(dim=3, nx=40, ny=30, nz=20, axis=2, g=gd, periodic=True), B.opts(B.RN_MIXED, 1e-8))
    r = oracle_mod.solve(net, tol=1e-13)
    assert res.K == pytest.approx(r.K, rel=1e-7)
