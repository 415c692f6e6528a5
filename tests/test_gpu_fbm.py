"""GPU generation of correlated networks (rn_fbm_field, rn_fbm_bonds) against
the numpy generator on the same random numbers: the Fourier filter of Eqs.
1-2 (numpy's FFT as the CPU reference), the bond construction and the
dilution; then a network generated on the GPU gives the K of the numpy one."""
import numpy as np
import pytest

from paper_1908_03301_amd import binding as B
from paper_1908_03301_amd import inputs as I
from tests.test_gpu_parity import ctx, say  # noqa: F401

pytestmark = pytest.mark.gpu

FIELDS = [  # dim, nx, ny, nz, H, beta per lattice direction (x, y, z)
    (2, 256, 192, 1, 0.7, (1.0, 1.0)),
    (2, 201, 150, 1, 0.75, (4.0, 1.0)),
    (2, 64, 7, 1, 0.35, (1.0, 2.5)),
    (3, 40, 30, 20, 0.35, (1.0, 2.0, 1.0)),
    (3, 33, 17, 9, 0.8, (1.0, 1.0, 1.0)),
]


def _numpy_beta(dim, beta):
    return list(beta[:dim])[::-1]        # numpy axes are (y, x) or (z, y, x)


@pytest.mark.parametrize("case", range(len(FIELDS)))
@pytest.mark.parametrize("device", [False, True])
def test_field_matches_numpy_filter(ctx, case, device):
    import torch
    dim, nx, ny, nz, H, beta = FIELDS[case]
    shape = (ny, nx) if dim == 2 else (nz, ny, nx)
    noise = I.rng_for(700 + case).standard_normal(shape)
    ref = I.fbm_filter(noise, H, _numpy_beta(dim, beta))
    say(f"fbm field dim={dim} shape={shape} H={H} beta={beta} device={device}")
    if device:
        nd = torch.from_numpy(noise).cuda()
        out = torch.empty_like(nd)
        ctx.fbm_field(dim, nx, ny, nz, H, nd, out, beta=beta)
        got = out.cpu().numpy()
    else:
        got = np.empty_like(noise)
        ctx.fbm_field(dim, nx, ny, nz, H, noise, got, beta=beta)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-11)
    assert abs(got.mean()) < 1e-12 and got.std() == pytest.approx(1.0, rel=1e-12)


@pytest.mark.parametrize("periodic", [False, True])
def test_bonds_and_dilution_match_numpy(ctx, periodic):
    import torch
    for dim, nx, ny, nz in ((2, 130, 97, 1), (3, 21, 18, 15)):
        shape = (ny, nx) if dim == 2 else (nz, ny, nx)
        rng = I.rng_for(800 + dim)
        phi = rng.standard_normal(shape)
        u = [rng.random(shape) for _ in range(dim)]
        ref = I.bonds_from_node_field(phi, 1.5, periodic=periodic)
        ref = [np.where(uk < 0.6, g, 0.0) for uk, g in zip(u, ref)]
        say(f"fbm bonds dim={dim} periodic={periodic}")
        g = [np.empty(shape) for _ in range(dim)]
        ctx.fbm_bonds(dim, nx, ny, nz, phi, 1.5, periodic, g, u=u, occupancy=0.6)
        gd = [torch.empty(shape, dtype=torch.float64, device="cuda") for _ in range(dim)]
        ctx.fbm_bonds(dim, nx, ny, nz, torch.from_numpy(phi).cuda(), 1.5, periodic, gd,
                      u=[torch.from_numpy(a).cuda() for a in u], occupancy=0.6)
        for a, b, r in zip(g, gd, ref):
            np.testing.assert_array_equal(a == 0.0, r == 0.0)
            np.testing.assert_allclose(a, r, rtol=1e-14, atol=0)
            np.testing.assert_array_equal(b.cpu().numpy(), a)
        # no dilution: every in-lattice bond present
        g2 = [np.empty(shape) for _ in range(dim)]
        ctx.fbm_bonds(dim, nx, ny, nz, phi, 1.5, periodic, g2)
        for a, r in zip(g2, I.bonds_from_node_field(phi, 1.5, periodic=periodic)):
            np.testing.assert_allclose(a, r, rtol=1e-14, atol=0)


def test_gpu_generated_network_solves_like_numpy(ctx):
    """A 512^2 network built on the GPU from the numpy generator's own random
    draws (normals, then dilution uniforms) has the numpy network's K."""
    import torch
    nx = ny = 512
    rng = I.rng_for(901)
    noise = rng.standard_normal((ny, nx))
    ref = I.fbm_network(2, nx, ny, 1, H=0.7, sigma=1.5, occupancy=0.65, index=901)
    u = [rng.random((ny, nx)) for _ in range(2)]           # dilute_iid's draws, in its order
    phi = torch.empty((ny, nx), dtype=torch.float64, device="cuda")
    ctx.fbm_field(2, nx, ny, 1, 0.7, torch.from_numpy(noise).cuda(), phi)
    g = [torch.empty((ny, nx), dtype=torch.float64, device="cuda") for _ in range(2)]
    ctx.fbm_bonds(2, nx, ny, 1, phi, 1.5, False, g, u=[torch.from_numpy(a).cuda() for a in u], occupancy=0.65)
    for a, r in zip(g, ref.g):
        np.testing.assert_array_equal(a.cpu().numpy() == 0.0, r == 0.0)
        np.testing.assert_allclose(a.cpu().numpy(), r, rtol=1e-9)
    for axis in (0, 1):
        r_gpu = ctx.solve(B.problem(dim=2, nx=nx, ny=ny, nz=1, axis=axis, g=g), B.opts(B.RN_FP64, 1e-10))
        r_np = ctx.solve(B.problem(ref.with_axis(axis)), B.opts(B.RN_FP64, 1e-10))
        assert r_gpu.converged and r_np.converged
        assert r_gpu.n_live == r_np.n_live
        assert r_gpu.K == pytest.approx(r_np.K, rel=1e-8)
