"""The seeded generator: determinism, conventions and the statistics the paper's workloads assume."""
import numpy as np
import pytest

from paper_1908_03301_amd import inputs as I


def test_determinism_and_independence():
    a = I.fbm_network(2, 64, 48, 1, H=0.7, sigma=1.5, occupancy=0.6, index=3)
    b = I.fbm_network(2, 64, 48, 1, H=0.7, sigma=1.5, occupancy=0.6, index=3)
    c = I.fbm_network(2, 64, 48, 1, H=0.7, sigma=1.5, occupancy=0.6, index=4)
    for k in range(2):
        assert a.g[k].tobytes() == b.g[k].tobytes()
    assert a.g[0].tobytes() != c.g[0].tobytes()


@pytest.mark.parametrize("dim", [2, 3])
def test_edge_entries_cleared_and_layout(dim):
    net = I.iid_network(dim, 7, 6, 5 if dim == 3 else 1, sigma=1.0, index=1)
    assert net.g[0].shape == net.shape and net.g[0].flags["C_CONTIGUOUS"]
    assert np.all(net.g[0][..., -1] == 0)
    assert np.all(net.g[1][..., -1, :] == 0)
    if dim == 3:
        assert np.all(net.g[2][-1] == 0)
    assert np.all(net.g[0][..., :-1] > 0)


def _radial_slope(field):
    F = np.abs(np.fft.fftn(field)) ** 2
    ks = [np.fft.fftfreq(n) for n in field.shape]
    K = np.sqrt(sum(np.meshgrid(*[k ** 2 for k in ks], indexing="ij")))
    sel = (K > 0.02) & (K < 0.2)
    return np.polyfit(np.log(K[sel]), np.log(F[sel]), 1)[0]


@pytest.mark.parametrize("H", [0.35, 0.7])
def test_fbm_spectrum_slope_2d(H):
    """Eq. 1: the power spectrum falls off as |k|^-(2H+2) in 2D."""
    slopes = [_radial_slope(I.fbm_field((256, 256), H, I.rng_for(50 + s))) for s in range(3)]
    assert np.mean(slopes) == pytest.approx(-(2 * H + 2), abs=0.15)


def test_fbm_spectrum_slope_1d():
    slopes = [_radial_slope(I.fbm_field((4096,), 0.8, I.rng_for(60 + s))) for s in range(6)]
    assert np.mean(slopes) == pytest.approx(-(2 * 0.8 + 1), abs=0.2)


def test_fbm_standardised_and_anisotropic():
    f = I.fbm_field((128, 128), 0.7, I.rng_for(7))
    assert abs(f.mean()) < 1e-12 and f.std() == pytest.approx(1.0, rel=1e-12)
    # Eq. 2 with a large weight on numpy axis 1 (x): the field varies slowly along x (layers along x)
    fa = I.fbm_field((128, 128), 0.7, I.rng_for(7), beta=[1.0, 25.0])
    dx = np.mean(np.diff(fa, axis=1) ** 2)
    dy = np.mean(np.diff(fa, axis=0) ** 2)
    assert dx < dy


def test_iid_dilution_fraction():
    net = I.iid_network(2, 300, 300, 1, sigma=1.0, occupancy=0.6, index=9)
    valid = I.edge_valid(2, net.shape, 0)
    frac = (net.g[0][valid] > 0).mean()
    assert frac == pytest.approx(0.6, abs=0.01)


def test_rank_dilution_removes_smallest():
    net = I.fbm_network(2, 40, 30, 1, H=0.7, sigma=1.5, index=2)
    q = 0.37
    d = I.dilute_rank(net.g, q)
    vals_before, vals_after = [], []
    for k in range(2):
        v = I.edge_valid(2, net.shape, k)
        vals_before.append(net.g[k][v])
        vals_after.append(d[k][v])
    b = np.concatenate(vals_before)
    a = np.concatenate(vals_after)
    n_cut = int(np.floor(q * b.size))
    assert int((a == 0).sum()) == n_cut
    assert b[a == 0].max() <= b[a > 0].min()


def test_stratified_layers():
    net = I.stratified_network(12, H=0.8, sigma=2.0, occupancy=1.0, index=0)
    gx = net.g[0][:, :, :-1]
    assert np.all(gx == gx[:, :1, :1])          # constant within a z-layer
    phi = net.meta["phi"]
    np.testing.assert_allclose(net.g[2][:-1, 0, 0], np.exp(phi[:-1] + phi[1:]), rtol=1e-14)


def test_batch_and_stream_specs():
    specs = I.batch_specs(512)
    assert len(specs) == 512
    s2 = [s for s in specs if s.dim == 2]
    s3 = [s for s in specs if s.dim == 3]
    assert len(s2) == len(s3) == 256
    assert all(64 <= s.side <= 1024 and 0.55 <= s.occupancy <= 1.0 for s in s2)
    assert all(32 <= s.side <= 128 and 0.3 <= s.occupancy <= 1.0 for s in s3)
    assert all(0.5 <= s.H <= 0.9 for s in specs)
    reqs = I.stream_requests(400, rate_per_s=10.0)
    ns = np.array([r.side ** r.dim for r in reqs])
    assert ns.min() >= 5e3 and ns.max() <= 4e7
    assert 0.35 < np.mean([r.dim == 2 for r in reqs]) < 0.65
    t = np.array([r.t_arrival for r in reqs])
    assert np.all(np.diff(t) > 0)


def test_aniso_spectrum_layers_along_x(oracle_mod):
    """Eq. 2 with beta_x / beta_y > 1 stretches the correlations along x:
    the field varies less from column to column than from row to row, and
    flow along the strata (K_x) is easier than across them (K_y)."""
    import numpy as np
    specs = [s for s in I.aniso_specs(H_values=(0.75,), ratios=(1, 16), seeds=4)]
    ratios = {1.0: [], 16.0: []}
    for sp in specs:
        net = I.aniso_network(sp, n=64)
        lg = np.log(net.g[1][:-1, :])                     # y-bonds: ln g = sigma * mean of two node values
        vx = np.var(np.diff(lg, axis=1))
        vy = np.var(np.diff(lg, axis=0))
        if sp.ratio == 16.0:
            assert vx < 0.5 * vy
        kx = oracle_mod.solve(net, tol=1e-12).K
        ky = oracle_mod.solve(net.with_axis(1), tol=1e-12).K
        ratios[sp.ratio].append(kx / ky)
    assert np.mean(ratios[16.0]) > 1.0
    assert np.mean(ratios[16.0]) > np.mean(ratios[1.0])
