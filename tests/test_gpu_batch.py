"""GPU tests of batched and served solves (rn_solve_batch, rn_submit / rn_poll).

Every network in a batch or in the served stream must give exactly the bits
it gives when solved alone (same tiles, same reduction order, its own
control block), and the served stream must overlap networks on the device
while admitting them against the HBM budget.
"""
import sys
import time

import numpy as np
import pytest

from paper_1908_03301_amd import binding as B
from paper_1908_03301_amd import inputs as I

pytestmark = pytest.mark.gpu

FIELDS = ("status", "converged", "Q_in", "Q_out", "G", "K", "rel_resid", "iters", "refreshes", "n_live")


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def mixed_set():
    """Uneven networks: 2D and 3D, both precisions, ragged shapes, all axes, both side conditions."""
    nets = [
        (I.fbm_network(2, 200, 150, 1, H=0.7, sigma=1.5, occupancy=0.6, index=700), B.RN_FP64, 1e-10),
        (I.fbm_network(2, 129, 257, 1, H=0.35, sigma=1.5, occupancy=0.55, index=701).with_axis(1), B.RN_MIXED, 1e-8),
        (I.fbm_network(3, 70, 40, 37, H=0.7, sigma=1.0, occupancy=0.35, index=702), B.RN_MIXED, 1e-8),
        (I.fbm_network(3, 33, 33, 33, H=0.7, sigma=1.0, occupancy=0.6, index=703).with_axis(2), B.RN_FP64, 1e-10),
        (I.iid_network(2, 64, 64, 1, occupancy=0.3, index=704), B.RN_FP64, 1e-10),       # non-percolating
        (I.uniform_network(2, 2, 40, 1, g0=1.5), B.RN_MIXED, 1e-8),                         # two planes
        (I.workload_iid_2d_128(), B.RN_MIXED, 1e-8),
        (I.stratified_network(24, H=0.8, sigma=2.0, occupancy=0.4, index=705).with_axis(2), B.RN_MIXED, 1e-8),
        (I.fbm_network(2, 300, 5, 1, H=0.7, sigma=1.5, occupancy=0.9, index=706), B.RN_FP64, 1e-10),
        (I.fbm_network(3, 5, 70, 18, H=0.7, sigma=1.0, occupancy=0.7, index=707).with_axis(1), B.RN_MIXED, 1e-8),
        # periodic sides (each network carries its own flag through the batch)
        (I.fbm_network(2, 130, 70, 1, H=0.7, sigma=1.5, occupancy=0.7, index=708, periodic=True).with_axis(1),
         B.RN_MIXED, 1e-8),
        (I.fbm_network(3, 40, 33, 17, H=0.7, sigma=1.0, occupancy=0.6, index=709, periodic=True), B.RN_FP64, 1e-10),
    ]
    return nets


def solo(ctx, net, prec, tol):
    P = np.zeros(net.shape)
    r = ctx.solve(B.problem(net, p_out=P), B.opts(prec, tol))
    return r, P


def same(a, b):
    for f in FIELDS:
        assert getattr(a, f) == getattr(b, f), (f, getattr(a, f), getattr(b, f))


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = B.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def solos(ctx):
    out = []
    for net, prec, tol in mixed_set():
        say(f"solo dim={net.dim} shape={net.shape} axis={net.axis} prec={prec}")
        out.append(solo(ctx, net, prec, tol))
    return out


def test_batch_bit_identical_to_solo(ctx, solos):
    sets = mixed_set()
    Ps = [np.zeros(net.shape) for net, _, _ in sets]
    probs = [B.problem(net, p_out=P) for (net, _, _), P in zip(sets, Ps)]
    say(f"rn_solve_batch of {len(probs)} networks")
    res = ctx.solve_batch(probs, [B.opts(p, t) for _, p, t in sets])
    for (r_solo, P_solo), r, P in zip(solos, res, Ps):
        same(r_solo, r)
        assert P.tobytes() == P_solo.tobytes()
    # the batch really ran networks side by side: fewer rounds than the sum of solos
    assert max(r.passes for r in res) < sum(r.passes for r, _ in solos)


def test_batch_members_against_oracle(ctx, oracle_mod):
    sets = mixed_set()
    probs = [B.problem(net) for net, _, _ in sets]
    res = ctx.solve_batch(probs, [B.opts(p, t) for _, p, t in sets])
    for (net, prec, tol), r in zip(sets, res):
        ref = oracle_mod.solve(net, tol=1e-13)
        assert r.n_live == ref.n_live
        assert r.converged and r.status == 0
        bar = 1e-9 if prec == B.RN_FP64 else 1e-7
        assert r.K == pytest.approx(ref.K, rel=bar, abs=1e-300)


def test_served_stream_matches_solo_and_overlaps(ctx, solos):
    sets = mixed_set()
    Ps = [np.zeros(net.shape) for net, _, _ in sets]
    probs = [B.problem(net, p_out=P) for (net, _, _), P in zip(sets, Ps)]
    c = B.Context(0)
    try:
        say("server: submitting")
        tickets = []
        peak_active = 0
        for pr, (_, prec, tol) in zip(probs, sets):
            tickets.append(c.submit(pr, B.opts(prec, tol)))
            peak_active = max(peak_active, c.stats()["active"])
        done = {}
        t0 = time.time()
        while len(done) < len(tickets):
            assert time.time() - t0 < 120, "served stream did not finish"
            for t in tickets:
                if t in done:
                    continue
                st, r = c.poll(t)
                if st != B.RN_EAGAIN:
                    done[t] = (st, r)
            peak_active = max(peak_active, c.stats()["active"])
            time.sleep(0.001)
        for t, (r_solo, P_solo), P in zip(tickets, solos, Ps):
            st, r = done[t]
            assert st == r_solo.status
            same(r_solo, r)
            assert P.tobytes() == P_solo.tobytes()
            assert r.t_total_s > 0
        # networks shared pass launches on the device (continuous batching)
        assert c.stats()["peak_active"] >= 2, "networks never overlapped on the device"
        # collected tickets are forgotten
        st, _ = c.poll(tickets[0])
        assert st == B.RN_ENOTFOUND
        st, _ = c.poll(123456789)
        assert st == B.RN_ENOTFOUND
        # synchronous calls go through the running server and give the same bits
        r = c.solve(B.problem(sets[0][0]), B.opts(sets[0][1], sets[0][2]))
        same(solos[0][0], r)
    finally:
        c.close()


def test_admission_under_a_small_budget(ctx):
    nets = [I.fbm_network(2, 256, 256, 1, H=0.7, sigma=1.5, occupancy=0.7, index=800 + i) for i in range(8)]
    o = B.opts(B.RN_MIXED, 1e-8)
    fp = max(B.rn_footprint(B.problem(n), o) for n in nets)
    budget = int(2.5 * fp)
    say(f"server with budget {budget} bytes (2.5 networks)")
    c = B.Context(0, hbm_budget_bytes=budget)
    try:
        big = I.uniform_network(2, 1024, 1024)
        with pytest.raises(B.RNError) as e:
            c.submit(B.problem(big), o)
        assert e.value.code == B.RN_ENOMEM
        probs = [B.problem(n) for n in nets]
        tickets = [c.submit(pr, o) for pr in probs]
        saw_waiting = False
        done = {}
        t0 = time.time()
        while len(done) < len(tickets):
            assert time.time() - t0 < 120
            s = c.stats()
            assert s["bytes_in_use"] <= budget
            saw_waiting |= s["waiting"] > 0
            for t in tickets:
                if t not in done:
                    st, r = c.poll(t)
                    if st != B.RN_EAGAIN:
                        done[t] = (st, r)
            time.sleep(0.0005)
        assert saw_waiting, "no request ever waited for memory"
        for t in tickets:
            st, r = done[t]
            assert st == B.RN_OK and r.converged
        # each result equals the unconstrained solo solve
        for n, t in zip(nets[:3], tickets[:3]):
            r_solo = ctx.solve(B.problem(n), o)
            same(r_solo, done[t][1])
    finally:
        c.close()


def test_eagain_then_ok(ctx):
    net = I.fbm_network(2, 1024, 1024, 1, H=0.7, sigma=1.5, occupancy=0.65, index=900)
    c = B.Context(0)
    try:
        t = c.submit(B.problem(net), B.opts(B.RN_MIXED, 1e-8))
        st, _ = c.poll(t)
        assert st == B.RN_EAGAIN
        t0 = time.time()
        while st == B.RN_EAGAIN:
            assert time.time() - t0 < 60
            time.sleep(0.002)
            st, r = c.poll(t)
        assert st == B.RN_OK and r.converged and r.iters > 0
    finally:
        c.close()


def test_graph_replay_bit_identical(solos):
    """With RN_GRAPHS=1 the pass rounds of each chunk are replayed from a
    captured hipGraph; every network must give the bits of direct launches."""
    import os
    sets = mixed_set()
    old = os.environ.get("RN_GRAPHS")
    os.environ["RN_GRAPHS"] = "1"
    try:
        c = B.Context(0)
    finally:
        if old is None:
            del os.environ["RN_GRAPHS"]
        else:
            os.environ["RN_GRAPHS"] = old
    try:
        for i in (0, 2, 6):   # 2D FP64, 3D mixed, the 128^2 workload
            net, prec, tol = sets[i]
            say(f"graph replay: solo {i} dim={net.dim} shape={net.shape}")
            r, P = solo(c, net, prec, tol)
            same(solos[i][0], r)
            assert P.tobytes() == solos[i][1].tobytes()
        Ps = [np.zeros(net.shape) for net, _, _ in sets]
        probs = [B.problem(net, p_out=P) for (net, _, _), P in zip(sets, Ps)]
        say("graph replay: batch")
        res = c.solve_batch(probs, [B.opts(p, t) for _, p, t in sets])
        for (r_solo, P_solo), r, P in zip(solos, res, Ps):
            same(r_solo, r)
            assert P.tobytes() == P_solo.tobytes()
    finally:
        c.close()


def test_host_input_admitted_mid_run(ctx):
    """A request with host buffers, submitted while a large device-resident network
    iterates, is uploaded and prepared on the context's side stream, overlaps the
    running passes, finishes first, and gives the bits of its solo solve."""
    import torch
    big = I.fbm_network(2, 1536, 1536, 1, H=0.7, sigma=1.5, occupancy=0.62, index=810)
    small = I.fbm_network(3, 60, 50, 40, H=0.7, sigma=1.0, occupancy=0.6, index=811)
    o = B.opts(B.RN_MIXED, 1e-8)
    gd = [torch.from_numpy(a).to("cuda") for a in big.g]
    torch.cuda.synchronize()
    P_small_solo = np.zeros(small.shape)
    r_small_solo = ctx.solve(B.problem(small, p_out=P_small_solo), o)
    r_big_solo = ctx.solve(B.problem(dim=2, nx=big.nx, ny=big.ny, nz=1, axis=0, g=gd), o)
    c = B.Context(0)
    try:
        tb = c.submit(B.problem(dim=2, nx=big.nx, ny=big.ny, nz=1, axis=0, g=gd), o)
        t0 = time.time()
        while c.stats()["active"] < 1:
            assert time.time() - t0 < 60
            time.sleep(0.001)
        time.sleep(0.05)                  # the big network is iterating
        P_small = np.zeros(small.shape)
        ts = c.submit(B.problem(small, p_out=P_small), o)
        done = {}
        while len(done) < 2:
            assert time.time() - t0 < 300, "served requests did not finish"
            for t in (tb, ts):
                if t not in done:
                    st, r = c.poll(t)
                    if st != B.RN_EAGAIN:
                        done[t] = (st, r, time.time())
            time.sleep(0.0005)
    finally:
        c.close()
    st_s, r_s, t_s = done[ts]
    st_b, r_b, t_b = done[tb]
    assert st_s == B.RN_OK and st_b == B.RN_OK
    same(r_small_solo, r_s)
    same(r_big_solo, r_b)
    assert P_small.tobytes() == P_small_solo.tobytes()
    assert t_s < t_b, "the host-input request waited for the running network"
    say(f"host-input request done in {r_s.t_total_s:.3f}s while the 1536^2 network took {r_b.t_total_s:.3f}s")


def test_smaller_request_goes_ahead_of_one_that_does_not_fit(ctx):
    """First-fit admission: with one large network running and a second large one
    waiting for its memory, a small request submitted after the second is
    admitted beside the first and finishes before the second, with its solo bits."""
    o = B.opts(B.RN_MIXED, 1e-8)
    big1 = I.fbm_network(2, 1024, 1024, 1, H=0.7, sigma=1.5, occupancy=0.65, index=820)
    big2 = I.fbm_network(2, 1024, 1024, 1, H=0.7, sigma=1.5, occupancy=0.65, index=821)
    small = I.fbm_network(2, 200, 200, 1, H=0.7, sigma=1.5, occupancy=0.7, index=822)
    fb = B.rn_footprint(B.problem(big1), o)
    fs = B.rn_footprint(B.problem(small), o)
    budget = fb + 2 * fs          # room for one large network and the small one, not two large
    r_small_solo = ctx.solve(B.problem(small), o)
    c = B.Context(0, hbm_budget_bytes=budget)
    try:
        t1 = c.submit(B.problem(big1), o)
        t2 = c.submit(B.problem(big2), o)
        t3 = c.submit(B.problem(small), o)
        done, order, t0 = {}, [], time.time()
        while len(done) < 3:
            assert time.time() - t0 < 300
            assert c.stats()["bytes_in_use"] <= budget
            for t in (t1, t2, t3):
                if t not in done:
                    st, r = c.poll(t)
                    if st != B.RN_EAGAIN:
                        done[t] = (st, r)
                        order.append(t)
            time.sleep(0.0005)
    finally:
        c.close()
    assert all(done[t][0] == B.RN_OK for t in (t1, t2, t3))
    assert order.index(t3) < order.index(t2), order
    same(r_small_solo, done[t3][1])
    say(f"completion order {order} (big1={t1}, big2={t2}, small={t3})")
