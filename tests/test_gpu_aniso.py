"""GPU parity on anisotropic and rank-diluted FBM networks (Sec. II Eq. 2; Sec. VI.B).

The conductance field follows the anisotropic spectrum of Eq. 2 with
beta_x / beta_y in {1, 4, 16}; some networks are also diluted by the
rank-threshold rule of Sec. VI.B (the fraction q of bonds with the smallest
conductance removed), near the correlated-percolation threshold, where strata
parallel to x leave no path along y. Every network is solved along x and y
in one rn_solve_batch (mixed precision to 1e-8 and FP64 to 1e-10) and held to
the CPU oracle: mask bit for bit, K within 1e-7 / 1e-9 of the oracle solved
to 1e-13, the true residual of the returned field re-evaluated by the oracle,
the energy conductance against the oracle's evaluation of that field, and the
maximum principle to within the field's energy bound (tests/_pins).

A second test checks the direction of the Fig. 10 study on the GPU: on
seeded 128 x 128 networks the median of K_x / K_y grows from near 1 at
beta_x / beta_y = 1 to several times that at 16, for H = 0.75 and 0.35.
"""
import sys

import numpy as np
import pytest

from paper_1908_03301_amd import binding as B
from paper_1908_03301_amd import inputs as I
from tests import _pins

pytestmark = pytest.mark.gpu

TOL = {B.RN_FP64: 1e-10, B.RN_MIXED: 1e-8}
KBAR = {B.RN_FP64: 1e-9, B.RN_MIXED: 1e-7}


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
    """(label, network, precision) for both flow axes of each network."""
    nets = [
        ("H0.75 b1", I.fbm_network(2, 320, 256, 1, H=0.75, sigma=1.5, index=31600, beta=[1.0, 1.0]), (B.RN_MIXED,)),
        ("H0.75 b16", I.fbm_network(2, 320, 256, 1, H=0.75, sigma=1.5, index=31601, beta=[1.0, 16.0]),
         (B.RN_MIXED, B.RN_FP64)),
        ("H0.35 b16 q0.40", I.fbm_network(2, 320, 256, 1, H=0.35, sigma=1.5, index=31500, beta=[1.0, 16.0],
                                          rank_q=0.40), (B.RN_MIXED,)),
        ("H0.75 b4 q0.45", I.fbm_network(2, 256, 300, 1, H=0.75, sigma=1.5, index=31602, beta=[1.0, 4.0],
                                         rank_q=0.45), (B.RN_FP64,)),
        ("H0.35 b1 q0.45", I.fbm_network(2, 300, 300, 1, H=0.35, sigma=1.5, index=31603, beta=[1.0, 1.0],
                                         rank_q=0.45), (B.RN_MIXED,)),
    ]
    out = []
    for label, net, precs in nets:
        for axis in (0, 1):
            for prec in precs:
                out.append((f"{label} axis {axis}", net.with_axis(axis), prec))
    return out


def test_aniso_and_rank_diluted_against_oracle(ctx, oracle_mod):
    cs = cases()
    Ps = [np.zeros(net.shape) for _, net, _ in cs]
    Ms = [np.zeros(net.shape, dtype=np.uint8) for _, net, _ in cs]
    probs = [B.problem(net, p_out=P, mask_out=M) for (_, net, _), P, M in zip(cs, Ps, Ms)]
    say(f"rn_solve_batch of {len(probs)} anisotropic / rank-diluted solves")
    res = ctx.solve_batch(probs, [B.opts(prec, TOL[prec]) for _, _, prec in cs])
    no_path = 0
    for (label, net, prec), r, P, M in zip(cs, res, Ps, Ms):
        mref, nl = oracle_mod.mask_bfs(net)
        np.testing.assert_array_equal(M, mref)
        assert r.n_live == nl
        assert r.status == 0 and r.converged
        ref = oracle_mod.solve(net, tol=1e-13)
        say(f"{label} {'fp64' if prec == B.RN_FP64 else 'mixed'}: n_live {nl} K {r.K:.12g} oracle {ref.K:.12g} "
            f"iters {r.iters}")
        if nl == 0:
            no_path += 1
            assert r.K == 0.0 and ref.K == 0.0
            continue
        assert r.K == pytest.approx(ref.K, rel=KBAR[prec])
        c = oracle_mod.check_pressure(net, P)
        assert c.rel_resid <= 1.01 * TOL[prec]
        assert r.G == pytest.approx(c.G_E, rel=1e-9)
        # maximum principle: the exact pressures lie in [0, 1]; the returned
        # field is within the energy bound of them at every live node
        E = _pins.energy(net, P)
        live = mref.ravel() == 3
        R = _pins.face_path_resistance(net).ravel()[live]
        eps = float(np.max(_pins.pressure_error_bound(R, E, ref.G)))
        assert -eps <= c.p_min and c.p_max <= 1.0 + eps, (c.p_min, c.p_max, eps)
    # strata parallel to x and rank dilution near the threshold: no path along y
    assert no_path >= 1


def test_fig10_trend_on_gpu(ctx):
    """Median K_x / K_y over seeded 128^2 networks rises steeply with beta_x / beta_y."""
    med = {}
    for H in (0.75, 0.35):
        for ratio in (1, 16):
            nets = [I.fbm_network(2, 128, 128, 1, H=H, sigma=1.5, beta=[1.0, float(ratio)],
                                  index=31000 + seed + 100 * ratio + 1000 * int(H * 100)) for seed in range(6)]
            probs = [B.problem(n.with_axis(ax)) for n in nets for ax in (0, 1)]
            res = ctx.solve_batch(probs, B.opts(B.RN_MIXED, 1e-8))
            assert all(r.status == 0 and r.converged for r in res)
            ratios = [res[2 * k].K / res[2 * k + 1].K for k in range(len(nets))]
            med[(H, ratio)] = float(np.median(ratios))
            say(f"H={H} beta_x/beta_y={ratio}: K_x/K_y {np.round(sorted(ratios), 3)}")
    for H in (0.75, 0.35):
        assert 0.5 < med[(H, 1)] < 2.0
        assert med[(H, 16)] > 3.0 * med[(H, 1)]
