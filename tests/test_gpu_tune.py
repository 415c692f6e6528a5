"""GPU test of the launch-shape search (rn_autotune) and its disk cache.

The paper's kernels used one fixed launch grid (Sec. IV); here each size
class gets the shape that measured fastest on the device. The quick search
must write a cache file with one line per searched class, install the table
process-wide (rn_plan follows it), and leave every result bit-identical
between a network alone and in a batch, with K still within the bars against
the oracle (Sec. II, Eqs. 3-4). The built-in rules are restored afterwards.
"""
import sys

import numpy as np
import pytest

from paper_1908_03301_amd import binding as B
from paper_1908_03301_amd import inputs as I

pytestmark = pytest.mark.gpu

FIELDS = ("status", "converged", "Q_in", "Q_out", "G", "K", "rel_resid", "iters", "refreshes", "n_live")


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def test_quick_autotune_cache_and_bits(tmp_path, oracle_mod):
    import time
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cache = tmp_path / "shapes.txt"
    c = B.Context(0)
    try:
        t0 = time.time()
        c.autotune(str(cache), quick=True)
        say(f"quick search: {time.time() - t0:.1f}s")
        lines = [l for l in cache.read_text().splitlines() if l and not l.startswith("#")]
        say("\n" + "\n".join(lines))
        # 2D classes 12..18 and 3D classes 15..17, both precisions
        assert len(lines) == 2 * 7 + 2 * 3
        rows = [l.split() for l in lines]
        assert all(float(r[6]) > 0.0 for r in rows)
        # the installed table is the cached one
        B.rn_tune_reset()
        B.rn_tune_load(str(cache))
        nets = [
            (I.fbm_network(2, 300, 280, 1, H=0.7, sigma=1.5, occupancy=0.7, index=4200), B.RN_MIXED, 1e-8),
            (I.fbm_network(2, 90, 200, 1, H=0.7, sigma=1.5, occupancy=0.65, index=4201), B.RN_FP64, 1e-10),
            (I.fbm_network(3, 45, 40, 38, H=0.7, sigma=1.0, occupancy=0.5, index=4202), B.RN_MIXED, 1e-8),
            (I.fbm_network(3, 50, 50, 50, H=0.7, sigma=1.0, occupancy=0.7, index=4203).with_axis(1), B.RN_FP64,
             1e-10),
        ]
        for net, prec, _ in nets:
            cls = int(np.floor(np.log2(net.n)))
            row = [r for r in rows if int(r[0]) == net.dim and r[1] == ("fp32" if prec == B.RN_MIXED else "fp64")
                   and int(r[2]) == cls]
            assert len(row) == 1
            plan = B.rn_plan(B.problem(net), B.opts(prec))
            if net.dim == 2:
                assert plan["path"] == (B.RN_PATH_2D_FULL if int(row[0][3]) == 0 else B.RN_PATH_2D_SMALL)
                assert plan["tiles_per_wg"] == min(int(row[0][4]), plan["tiles"])
            else:
                assert plan["tile_z"] == int(row[0][5])
            say(f"{net.dim}D n={net.n} class {cls}: {plan}")
        solos = []
        for net, prec, tol in nets:
            P = np.zeros(net.shape)
            solos.append((c.solve(B.problem(net, p_out=P), B.opts(prec, tol)), P))
        Ps = [np.zeros(net.shape) for net, _, _ in nets]
        res = c.solve_batch([B.problem(net, p_out=P) for (net, _, _), P in zip(nets, Ps)],
                            [B.opts(p, t) for _, p, t in nets])
        for (rs, Psolo), r, P, (net, prec, tol) in zip(solos, res, Ps, nets):
            for f in FIELDS:
                assert getattr(rs, f) == getattr(r, f), f
            assert P.tobytes() == Psolo.tobytes()
            ref = oracle_mod.solve(net, tol=1e-13)
            assert r.K == pytest.approx(ref.K, rel=1e-9 if prec == B.RN_FP64 else 1e-7)
    finally:
        B.rn_tune_reset()
        c.close()
