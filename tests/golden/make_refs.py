#!/usr/bin/env python3
"""Write the oracle reference values that the full-size GPU parity tests read.

Every number written here comes from the CPU oracle (oracle/, FP64 conjugate
gradients to a relative residual of 1e-13) or from test-side post-processing
of its output (tests/_pins.py); nothing comes from the GPU library. The
networks are regenerated from their seeded recipes (paper_1908_03301_amd/inputs.py),
so a file holds only the recipe and the results:

  fullsize_refs.json  networks large enough to reach the pass kernels' big
                      tile paths: K, G, fluxes, n_live, the energy of the
                      oracle field, and its pressures at seeded live nodes
  batch_refs.json     a seeded sample of 32 members of the 512-network batch
                      (which members, and the oracle's K for those whose
                      solve is affordable here)
  stream_refs.json    the same for 32 requests of the served stream
  layered_refs.json   the 256^3 layered network at occupancy 0.27 (K_x and
                      K_z), solved by the oracle with its dangling ends cut
                      out (tests/_pins.prune_dangling on the oracle's
                      backbone): the same K and, on the backbone, the same
                      pressures, for 2.2 M unknowns instead of 8.5 M

Usage: python3 tests/golden/make_refs.py [fullsize|batch|stream|layered ...] [--jobs N]
(several hours of CPU in total, spread over N processes).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1908_03301_amd import inputs as I  # noqa: E402
from tests import _pins  # noqa: E402

REF_TOL = 1e-13
SAMPLES = 512            # live nodes whose oracle pressure is stored per full-size network
MASTER_SAMPLE_SEED = 77  # seed of the member / request / node samples

# network recipes: generator of paper_1908_03301_amd.inputs and its arguments
FULLSIZE = {
    # FP64 tiles of 128 x 8 nodes: 32 x 33 = 1,056 tiles (two per workgroup); FP32 tiles of
    # 128 x 16: 32 x 17 = 544 (full tiles, one per workgroup)
    "fbm2d_4096x264": ("fbm_network", dict(dim=2, nx=4096, ny=264, nz=1, H=0.7, sigma=1.0, occupancy=0.8,
                                           index=1301, axis=1)),
    # FP64: 32 x 67 = 2,144 tiles, FP32: 32 x 34 = 1,088 tiles: two per workgroup in both
    "fbm2d_4096x530": ("fbm_network", dict(dim=2, nx=4096, ny=530, nz=1, H=0.7, sigma=1.0, occupancy=0.8,
                                           index=1302, axis=1)),
    # 3D tiles of 64 x 16 x tile_z: 8 x 16 column tiles; 16-plane tiles (3 x 128 = 384 workgroups,
    # one round) win over 8-plane ones (640, two rounds)
    "fbm3d_500x250x40": ("fbm_network", dict(dim=3, nx=500, ny=250, nz=40, H=0.7, sigma=1.0, occupancy=0.6,
                                             index=1303, axis=2)),
    # 11 x 16 column tiles: 32-plane tiles (352 workgroups, one round) against 16-plane (528, two)
    "fbm3d_700x250x33": ("fbm_network", dict(dim=3, nx=700, ny=250, nz=33, H=0.7, sigma=1.0, occupancy=0.6,
                                             index=1304, axis=2)),
}

# the 256^3 layered network of the single-network workloads, flow along x and z
LAYERED = {
    "layered3d_256_x": ("stratified_network", dict(n=256, H=0.8, sigma=2.0, occupancy=0.27, index=0, axis=0)),
    "layered3d_256_z": ("stratified_network", dict(n=256, H=0.8, sigma=2.0, occupancy=0.27, index=0, axis=2)),
}

BATCH_COUNT, STREAM_COUNT = 512, 512
SAMPLE_MEMBERS = 32
ORACLE_NODE_CAP = 1_100_000     # members above this many nodes get mask / residual checks only


def make_network(recipe):
    fn, kw = recipe
    return getattr(I, fn)(**kw)


def _fullsize_one(name):
    t = time.time()
    net = make_network(FULLSIZE[name])
    r = oracle.solve(net, tol=REF_TOL, want_mask=True)
    live = np.flatnonzero(r.mask.ravel() == 3)
    rng = np.random.default_rng([MASTER_SAMPLE_SEED, len(name)])
    pick = np.sort(rng.choice(live, size=min(SAMPLES, live.size), replace=False))
    out = {"recipe": list(FULLSIZE[name]), "status": r.status, "converged": bool(r.converged), "K": r.K, "G": r.G,
           "Q_in": r.Q_in, "Q_out": r.Q_out, "rel_resid": r.rel_resid, "iters": r.iters, "n_live": r.n_live,
           "energy": _pins.energy(net, r.pressure), "sample_index": [int(i) for i in pick],
           "sample_pressure": [float(v) for v in r.pressure.ravel()[pick]], "oracle_s": round(time.time() - t, 1)}
    print(f"{name}: K={r.K!r} iters={r.iters} live={r.n_live} in {out['oracle_s']}s", flush=True)
    return name, out


def _layered_one(name):
    t = time.time()
    net = make_network(LAYERED[name])
    mask, n_live, n_bb = oracle.backbone(net)
    pruned = _pins.prune_dangling(net, mask)
    r = oracle.solve(pruned, tol=REF_TOL, want_mask=True)
    bb = np.flatnonzero(r.mask.ravel() == 3)            # the pruned network's live set: the backbone
    assert bb.size == n_bb
    rng = np.random.default_rng([MASTER_SAMPLE_SEED, len(name)])
    pick = np.sort(rng.choice(bb, size=min(SAMPLES, bb.size), replace=False))
    R = _pins.face_path_resistance(net).ravel()[pick]     # on the whole network, as the GPU solves see it
    out = {"recipe": list(LAYERED[name]), "status": r.status, "converged": bool(r.converged), "K": r.K, "G": r.G,
           "Q_in": r.Q_in, "Q_out": r.Q_out, "rel_resid": r.rel_resid, "iters": r.iters, "n_live": n_live,
           "n_backbone": n_bb, "backbone_mask_sha256": hashlib.sha256(np.ascontiguousarray(mask).tobytes()).hexdigest(),
           "energy": _pins.energy(pruned, r.pressure), "sample_index": [int(i) for i in pick],
           "sample_pressure": [float(v) for v in r.pressure.ravel()[pick]], "sample_R": [float(v) for v in R],
           "oracle_s": round(time.time() - t, 1)}
    print(f"{name}: K={r.K!r} iters={r.iters} live={n_live} backbone={n_bb} in {out['oracle_s']}s", flush=True)
    return name, out


def _member_one(args):
    kind, k = args
    if kind == "batch":
        spec = I.batch_specs(BATCH_COUNT)[k]
        net = I.batch_network(spec)
        desc = {"dim": spec.dim, "side": spec.side, "H": spec.H, "occupancy": spec.occupancy, "index": spec.index}
    else:
        req = I.stream_requests(STREAM_COUNT, rate_per_s=1.0)[k]
        net = I.stream_network(req)
        desc = {"dim": req.dim, "side": req.side, "occupancy": req.occupancy, "index": req.index}
    out = {"member": k, "spec": desc, "nodes": net.n}
    if net.n <= ORACLE_NODE_CAP:
        t = time.time()
        r = oracle.solve(net, tol=REF_TOL, want_pressure=False)
        out.update({"K": r.K, "G": r.G, "n_live": r.n_live, "iters": r.iters, "status": r.status,
                    "oracle_s": round(time.time() - t, 1)})
        print(f"{kind} {k}: n={net.n} K={r.K!r} iters={r.iters} in {out['oracle_s']}s", flush=True)
    else:
        print(f"{kind} {k}: n={net.n} above the oracle cap: mask and residual checks only", flush=True)
    return out


def sample_members(kind):
    rng = np.random.default_rng([MASTER_SAMPLE_SEED, 4 if kind == "batch" else 5])
    count = BATCH_COUNT if kind == "batch" else STREAM_COUNT
    return sorted(int(v) for v in rng.choice(count, size=SAMPLE_MEMBERS, replace=False))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", nargs="*", default=["fullsize", "batch", "stream", "layered"])
    ap.add_argument("--jobs", type=int, default=4)
    args = ap.parse_args()
    oracle.build(force=False)
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        if "fullsize" in args.what:
            res = dict(ex.map(_fullsize_one, sorted(FULLSIZE)))
            doc = {"ref_tol": REF_TOL, "cases": res}
            json.dump(doc, open(os.path.join(HERE, "fullsize_refs.json"), "w"), indent=1)
        if "layered" in args.what:
            res = dict(ex.map(_layered_one, sorted(LAYERED)))
            doc = {"ref_tol": REF_TOL, "cases": res}
            json.dump(doc, open(os.path.join(HERE, "layered_refs.json"), "w"), indent=1)
        for kind in ("batch", "stream"):
            if kind not in args.what:
                continue
            members = sample_members(kind)
            res = list(ex.map(_member_one, [(kind, k) for k in members]))
            doc = {"ref_tol": REF_TOL, "count": BATCH_COUNT if kind == "batch" else STREAM_COUNT,
                   "oracle_node_cap": ORACLE_NODE_CAP, "members": res}
            json.dump(doc, open(os.path.join(HERE, f"{kind}_refs.json"), "w"), indent=1)


if __name__ == "__main__":
    main()
