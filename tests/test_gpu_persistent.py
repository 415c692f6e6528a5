"""GPU tests of the persistent pass kernels against the one-round-per-launch kernels.

By default a context runs one pass kernel launch per round and kind. A
context created with RN_PERSIST=1 in the environment runs every chunk of
rounds of a kind in one persistent launch, where a network's passes read
each other's state through device-scope loads and stores and wait on the
network's published pass count; with RN_PERSIST=2 every network small enough
is placed on one XCD and its items are claimed only by workgroups there (the
XCC_ID register), so its state stays coherent in that XCD's L2 (larger
networks keep one launch per round). All run the same tile code and the same
fixed-order reduction, so every result field and every pressure must be
bit-identical: alone, in a batch of uneven networks (2D full / small tiles,
two tiles per workgroup, 3D tiles of several depths, both precisions, both
side conditions, a network with no live node) and in the served stream. The
mixed results are also held to the oracle's K (Sec. II, Eqs. 3-4).
"""
import os
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


def networks():
    return [
        (I.fbm_network(2, 200, 150, 1, H=0.7, sigma=1.5, occupancy=0.6, index=900), B.RN_MIXED, 1e-8),
        (I.fbm_network(2, 640, 512, 1, H=0.7, sigma=1.0, occupancy=0.85, index=901), B.RN_MIXED, 1e-8),
        (I.fbm_network(2, 1100, 1030, 1, H=0.7, sigma=1.0, occupancy=0.9, index=902), B.RN_FP64, 1e-10),
        (I.fbm_network(3, 70, 40, 37, H=0.7, sigma=1.0, occupancy=0.35, index=903), B.RN_MIXED, 1e-8),
        (I.fbm_network(3, 96, 64, 80, H=0.7, sigma=1.0, occupancy=0.5, index=904).with_axis(2), B.RN_FP64, 1e-10),
        (I.iid_network(2, 64, 64, 1, occupancy=0.3, index=905), B.RN_MIXED, 1e-8),        # no live node
        (I.workload_iid_2d_128(), B.RN_FP64, 1e-10),
        (I.fbm_network(2, 130, 70, 1, H=0.7, sigma=1.5, occupancy=0.7, index=906, periodic=True).with_axis(1),
         B.RN_MIXED, 1e-8),
        (I.fbm_network(3, 40, 33, 17, H=0.7, sigma=1.0, occupancy=0.6, index=907, periodic=True), B.RN_MIXED, 1e-8),
    ]


def make_ctx(mode: int):
    """A context created with RN_PERSIST=mode (0: one launch per round)."""
    old = os.environ.get("RN_PERSIST")
    os.environ["RN_PERSIST"] = str(int(mode))
    try:
        return B.Context(0)
    finally:
        if old is None:
            del os.environ["RN_PERSIST"]
        else:
            os.environ["RN_PERSIST"] = old


def solve_all(mode: int, batched: bool):
    """Results and pressures of every network, from a context created with
    RN_PERSIST=mode."""
    c = make_ctx(mode)
    try:
        sets = networks()
        Ps = [np.zeros(net.shape) for net, _, _ in sets]
        probs = [B.problem(net, p_out=P) for (net, _, _), P in zip(sets, Ps)]
        if batched:
            res = c.solve_batch(probs, [B.opts(p, t) for _, p, t in sets])
        else:
            res = [c.solve(pr, B.opts(p, t)) for pr, (_, p, t) in zip(probs, sets)]
        launches = c.stats()["launches"]
        return res, Ps, launches
    finally:
        c.close()


@pytest.fixture(scope="module")
def reference():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    say("one launch per round: solo solves")
    return solve_all(mode=0, batched=False)


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("batched", [False, True])
def test_persistent_bit_identical(reference, batched, mode):
    ref_res, ref_P, ref_launches = reference
    say(f"persistent launches (RN_PERSIST={mode}): {'batch' if batched else 'solo solves'}")
    res, Ps, launches = solve_all(mode=mode, batched=batched)
    for k, (a, b, Pa, Pb) in enumerate(zip(ref_res, res, ref_P, Ps)):
        for f in FIELDS:
            assert getattr(a, f) == getattr(b, f), (k, f, getattr(a, f), getattr(b, f))
        assert Pa.tobytes() == Pb.tobytes(), k
    if not batched and mode == 1:
        # one persistent launch per chunk and kind instead of one per round (with
        # mode 2 the large FP64 network keeps one launch per round)
        assert launches < ref_launches / 4, (launches, ref_launches)
    say(f"persistent {'batch' if batched else 'solo'}: {launches} launches against {ref_launches}")


@pytest.mark.parametrize("mode", [1, 2])
def test_persistent_served_and_oracle(reference, oracle_mod, mode):
    """Served stream on persistent launches: solo bits, and K against the oracle."""
    import time
    ref_res, ref_P, _ = reference
    sets = networks()
    c = make_ctx(mode)
    try:
        Ps = [np.zeros(net.shape) for net, _, _ in sets]
        probs = [B.problem(net, p_out=P) for (net, _, _), P in zip(sets, Ps)]
        tickets = [c.submit(pr, B.opts(p, t)) for pr, (_, p, t) in zip(probs, sets)]
        done, t0 = {}, time.time()
        while len(done) < len(tickets):
            assert time.time() - t0 < 300, "served stream did not finish"
            for t in tickets:
                if t not in done:
                    st, r = c.poll(t)
                    if st != B.RN_EAGAIN:
                        done[t] = (st, r)
            time.sleep(0.001)
        errmsg = c.last_error()
    finally:
        c.close()
    for k, (t, a, Pa) in enumerate(zip(tickets, ref_res, ref_P)):
        st, r = done[t]
        assert st == a.status, (k, st, errmsg)
        for f in FIELDS:
            assert getattr(a, f) == getattr(r, f), (k, f)
        assert Pa.tobytes() == Ps[k].tobytes(), k
    for k, ((net, prec, tol), r) in enumerate(zip(sets, ref_res)):
        if net.n > 300_000:
            continue
        ref = oracle_mod.solve(net, tol=1e-13)
        assert r.n_live == ref.n_live
        bar = 1e-9 if prec == B.RN_FP64 else 1e-7
        assert r.K == pytest.approx(ref.K, rel=bar, abs=1e-300), k
