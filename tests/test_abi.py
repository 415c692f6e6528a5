"""The C-ABI library on the CPU: it loads, exports what include/rn.h declares,
and validates arguments before any device call (no GPU needed here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1908_03301_amd import binding as B
from paper_1908_03301_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_1908_03301_amd import build
        build.build()
    return B.lib()


def declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "rn.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(rn_[a-z_]+)\s*\(", hdr)))


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert "rn_solve" in names and "rn_build_mask" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(B.EXPORTED)


def test_strerror_and_defaults(lib):
    assert B.strerror(0) == "ok"
    assert B.strerror(-3) == "not converged"
    assert B.strerror(-99) == "unknown status"
    o = B.opts()
    assert o.precision == B.RN_FP64 and o.tol == 1e-8 and o.max_iter == 10_000_000
    assert B.rn_version() >= 100


def test_struct_layout_matches_header(lib):
    # sizes of the three ABI structs, compiled from rn.h by the host compiler
    src = '#include "rn.h"\n#include <stdio.h>\n#include <stddef.h>\nint main(){printf("%zu %zu %zu %zu %zu",' \
          'sizeof(rn_problem),sizeof(rn_opts),sizeof(rn_result),sizeof(rn_stats_t),' \
          'offsetof(rn_stats_t,pass_timed_launches));return 0;}\n'
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        open(os.path.join(d, "t.c"), "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), os.path.join(d, "t.c"), "-o",
                               os.path.join(d, "t")])
        out = subprocess.check_output([os.path.join(d, "t")]).decode().split()
    assert [int(v) for v in out] == [C.sizeof(B.rn_problem), C.sizeof(B.rn_opts), C.sizeof(B.rn_result),
                                     C.sizeof(B.rn_stats_t), B.rn_stats_t.pass_timed_launches.offset]


def test_plan_struct_and_paths(lib):
    """rn_plan: layout of rn_plan_t as the host compiler sees rn.h, and the
    path each lattice takes (no device call)."""
    src = '#include "rn.h"\n#include <stdio.h>\n#include <stddef.h>\nint main(){printf("%zu %zu %zu",' \
          'sizeof(rn_plan_t),offsetof(rn_plan_t,groups),offsetof(rn_plan_t,footprint));return 0;}\n'
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        open(os.path.join(d, "t.c"), "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), os.path.join(d, "t.c"), "-o",
                               os.path.join(d, "t")])
        out = [int(v) for v in subprocess.check_output([os.path.join(d, "t")]).decode().split()]
    assert out == [C.sizeof(B.rn_plan_t), B.rn_plan_t.groups.offset, B.rn_plan_t.footprint.offset]
    small = B.problem(dim=2, nx=128, ny=128, g=[np.ones(128 * 128)] * 2)
    p = B.rn_plan(small, B.opts(B.RN_MIXED))
    assert p["path"] == B.RN_PATH_2D_SMALL and p["tile_z"] == 1 and p["tiles"] >= 1
    assert p["workgroups"] % 8 == 0 and p["footprint"] == B.rn_footprint(small, B.opts(B.RN_MIXED))
    n = 1024 * 1024
    full = B.problem(dim=2, nx=1024, ny=1024, g=[np.ones(n), np.ones(n)])
    p = B.rn_plan(full, B.opts(B.RN_FP64))
    assert p["path"] == B.RN_PATH_2D_FULL and p["tiles"] * p["tile_x"] * p["tile_y"] >= n
    n3 = 64 ** 3
    cube = B.problem(dim=3, nx=64, ny=64, nz=64, g=[np.ones(n3)] * 3)
    p = B.rn_plan(cube, B.opts(B.RN_MIXED))
    assert p["path"] == B.RN_PATH_3D and p["tile_x"] == 64 and p["tile_z"] >= 2
    bad = B.rn_problem()
    assert lib.rn_plan(C.byref(bad), None, C.byref(B.rn_plan_t())) == B.RN_EINVAL
    assert lib.rn_plan(C.byref(small.c), None, None) == B.RN_EINVAL


def test_opts_field_offsets_match_header(lib):
    fields = [f for f, _ in B.rn_opts._fields_]
    src = '#include "rn.h"\n#include <stdio.h>\n#include <stddef.h>\nint main(){' + "".join(
        f'printf("%zu ", offsetof(rn_opts, {f}));' for f in fields) + 'return 0;}\n'
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        open(os.path.join(d, "t.c"), "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), os.path.join(d, "t.c"), "-o",
                               os.path.join(d, "t")])
        out = subprocess.check_output([os.path.join(d, "t")]).decode().split()
    assert [int(v) for v in out] == [getattr(B.rn_opts, f).offset for f in fields]


def test_opts_precond_and_initial_guess(lib):
    o = B.rn_opts()
    assert lib.rn_opts_default(C.byref(o)) == B.RN_OK
    assert o.precond == B.RN_JACOBI and o.x0 == B.RN_X0_LINEAR and o.flags == 0
    p = _prob()
    for prec in (B.RN_JACOBI, B.RN_NONE):
        for x0 in (B.RN_X0_LINEAR, B.RN_X0_ZERO):
            assert B.rn_validate(p, B.opts(precond=prec, x0=x0)) == B.RN_OK
    for bb in (False, True):
        for cp in (False, True):
            assert B.rn_validate(p, B.opts(backbone=bb, compact=cp)) == B.RN_OK
    for field, bad in (("precond", 2), ("precond", -1), ("x0", 2), ("x0", -1), ("flags", 4), ("flags", -1)):
        o = B.opts()
        setattr(o, field, bad)
        assert B.rn_validate(p, o) == B.RN_EINVAL, field
        assert B.rn_footprint(p, o) > 0                # the footprint does not depend on them


def test_binding_rejects_mismatched_buffers(lib):
    """The binding checks every buffer's element count, dtype, layout and
    memory space before a pointer reaches the library."""
    import torch
    net = I.uniform_network(2, 8, 6)
    with pytest.raises(ValueError, match="elements"):
        B.problem(dim=2, nx=8, ny=6, nz=1, g=[net.g[0], net.g[1][:5]])
    with pytest.raises(ValueError, match="elements"):
        B.problem(net, p_out=np.zeros((6, 7)))
    with pytest.raises(ValueError, match="float64"):
        B.problem(net, p_out=np.zeros((6, 8), dtype=np.float32))
    with pytest.raises(ValueError, match="uint8"):
        B.problem(net, mask_out=np.zeros((6, 8), dtype=np.int8))
    with pytest.raises(ValueError, match="contiguous"):
        B.problem(net, p_out=np.zeros((8, 6)).T)
    # device problems take CUDA tensors only (here: CPU tensors are rejected)
    gt = [torch.from_numpy(a) for a in net.g]
    with pytest.raises(ValueError, match="CUDA"):
        B.problem(dim=2, nx=8, ny=6, nz=1, g=gt)
    ok = B.problem(net, p_out=np.zeros((6, 8)), mask_out=np.zeros((6, 8), dtype=np.uint8))
    assert ok.device is None and ok.c.mem == B.RN_MEM_HOST


def _prob(**kw):
    net = I.uniform_network(2, 8, 6)
    p = B.problem(net)
    for k, v in kw.items():
        setattr(p.c, k, v)
    return p


def test_validate_rejects_bad_arguments(lib):
    assert B.rn_validate(_prob()) == B.RN_OK
    assert B.rn_validate(_prob(dim=4)) == B.RN_EINVAL
    assert B.rn_validate(_prob(nz=2)) == B.RN_EINVAL          # 2D needs nz == 1
    assert B.rn_validate(_prob(axis=2)) == B.RN_EINVAL
    assert B.rn_validate(_prob(nx=0)) == B.RN_EINVAL
    assert B.rn_validate(_prob(mem=7)) == B.RN_EINVAL
    assert B.rn_validate(_prob(flags=2)) == B.RN_EINVAL
    assert B.rn_validate(_prob(flags=B.RN_PERIODIC)) == B.RN_OK
    p = _prob()
    p.c.g[1] = None
    assert B.rn_validate(p) == B.RN_EINVAL
    # flow axis with a single plane
    net = I.uniform_network(2, 1, 6)
    assert B.rn_validate(B.problem(net)) == B.RN_EINVAL
    # option checks
    assert B.rn_validate(_prob(), B.opts(tol=0.0)) == B.RN_EINVAL
    assert B.rn_validate(_prob(), B.opts(precision=5)) == B.RN_EINVAL
    assert B.rn_validate(_prob(), B.opts(max_iter=-1)) == B.RN_EINVAL
    assert B.rn_validate(_prob(), B.opts(delta=1.5)) == B.RN_EINVAL


@pytest.mark.parametrize("bad", [-1.0, np.nan, np.inf])
def test_validate_rejects_bad_conductance(lib, bad):
    net = I.uniform_network(3, 5, 4, 3)
    g = [a.copy() for a in net.g]
    g[2][1, 2, 3] = bad
    assert B.rn_validate(B.problem(I.Network(3, 5, 4, 3, g, 0))) == B.RN_EINVAL
    # the same value past the lattice edge is ignored
    g = [a.copy() for a in net.g]
    g[2][-1, 2, 3] = bad
    g[0][1, 1, -1] = bad
    assert B.rn_validate(B.problem(I.Network(3, 5, 4, 3, g, 0))) == B.RN_OK
    # with periodic sides the last-plane entries of the directions other than
    # the flow axis are wrap bonds and are checked; along the flow axis they
    # stay ignored
    assert B.rn_validate(B.problem(I.Network(3, 5, 4, 3, g, 0), periodic=True)) == B.RN_EINVAL
    assert B.rn_validate(B.problem(I.Network(3, 5, 4, 3, g, 1), periodic=True)) == B.RN_EINVAL
    g = [a.copy() for a in net.g]
    g[0][1, 1, -1] = bad
    assert B.rn_validate(B.problem(I.Network(3, 5, 4, 3, g, 0), periodic=True)) == B.RN_OK
    assert B.rn_validate(B.problem(I.Network(3, 5, 4, 3, g, 1), periodic=True)) == B.RN_EINVAL


def test_footprint(lib):
    net = I.uniform_network(2, 2048, 2048)
    n = 2048 * 2048
    f64 = B.rn_footprint(B.problem(net), B.opts(B.RN_FP64))
    f32 = B.rn_footprint(B.problem(net), B.opts(B.RN_MIXED))
    # host input: FP64 copy of g (16) + P x2 (16) + mask (1), then in the inner
    # precision s: dim conductance arrays, two sets of z, u and three of p
    assert f64 >= n * (16 + 16 + 1 + 8 * (2 + 7))
    assert f32 >= n * (16 + 16 + 1 + 4 * (2 + 7))
    assert f32 < f64 < n * (16 + 16 + 1 + 8 * (2 + 7) + 2)
    assert B.rn_footprint(_prob(dim=5)) == 0


def test_null_context_is_rejected(lib):
    res = B.rn_result()
    assert lib.rn_solve(None, C.byref(_prob().c), None, C.byref(res)) == B.RN_EINVAL
    assert lib.rn_build_mask(None, C.byref(_prob().c), None) == B.RN_EINVAL
    assert lib.rn_build_backbone(None, C.byref(_prob().c), None, None) == B.RN_EINVAL
    assert lib.rn_build_backbone(None, None, None, None) == B.RN_EINVAL
    assert lib.rn_destroy(None) == B.RN_OK


def test_batch_and_serve_argument_checks(lib):
    """rn_solve_batch / rn_submit / rn_poll / rn_stats reject bad arguments before any device call."""
    res = (B.rn_result * 2)()
    probs = (B.rn_problem * 2)(_prob().c, _prob().c)
    assert lib.rn_solve_batch(None, 2, probs, None, 0, res) == B.RN_EINVAL
    t = C.c_uint64(0)
    assert lib.rn_submit(None, C.byref(_prob().c), None, C.byref(t)) == B.RN_EINVAL
    assert lib.rn_poll(None, 1, C.byref(B.rn_result())) == B.RN_EINVAL
    assert lib.rn_stats(None, C.byref(B.rn_stats_t())) == B.RN_EINVAL
    assert lib.rn_set_timing(None, 1) == B.RN_EINVAL
    assert lib.rn_build_mask_noalloc(None, None, None) == B.RN_EINVAL


def test_fbm_entry_points_reject_bad_arguments(lib):
    import ctypes as C
    L = B.lib()
    x = np.zeros(16)
    p = C.c_void_p(x.ctypes.data)
    assert L.rn_fbm_field(None, 2, 4, 4, 1, 0.7, None, p, p, B.RN_MEM_HOST) == B.RN_EINVAL
    DA3 = C.c_void_p * 3
    g = DA3(x.ctypes.data, x.ctypes.data, None)
    assert L.rn_fbm_bonds(None, 2, 4, 4, 1, p, 1.0, 0, None, 1.0, C.byref(g), B.RN_MEM_HOST) == B.RN_EINVAL


def test_launch_shape_table_load_and_reset(lib, tmp_path):
    """rn_tune_load installs a launch-shape table that rn_plan follows for the
    classes it sets (and only those); malformed files are refused whole;
    rn_tune_reset restores the built-in rules."""
    n512 = B.problem(dim=2, nx=512, ny=512, nz=1, axis=0, g=[np.ones((512, 512)), np.ones((512, 512))])
    n800 = B.problem(dim=2, nx=800, ny=800, nz=1, axis=0, g=[np.ones((800, 800)), np.ones((800, 800))])
    n64c = B.problem(dim=3, nx=64, ny=64, nz=64, axis=0, g=[np.ones((64, 64, 64))] * 3)
    mixed = B.opts(B.RN_MIXED)
    base512 = B.rn_plan(n512, mixed)
    base512d = B.rn_plan(n512, B.opts(B.RN_FP64))
    base800 = B.rn_plan(n800, mixed)
    base3d = B.rn_plan(n64c, mixed)
    assert base512["path"] == B.RN_PATH_2D_FULL and base512["tiles_per_wg"] == 1
    f = tmp_path / "shapes.txt"
    # 512^2 = 2^18 nodes: class 18; 64^3 = 2^18: class 18
    f.write_text("# comment\n2 fp32 18 1 2 0 0.125\n3 fp32 18 0 0 8 0.5\n")
    try:
        B.rn_tune_load(str(f))
        p = B.rn_plan(n512, mixed)
        assert p["path"] == B.RN_PATH_2D_SMALL and p["tiles_per_wg"] == 2
        assert p["workgroups"] >= p["tiles"] // 2
        assert B.rn_plan(n800, mixed) == base800          # 800^2 is in class 19: untouched
        assert B.rn_plan(n512, B.opts(B.RN_FP64)) == base512d     # FP64 entries untouched
        assert B.rn_plan(n64c, mixed)["tile_z"] == 8
        for bad in ("2 fp32 18 1 9 0 0.1\n", "4 fp32 18 1 1 0 0.1\n", "2 fp16 18 1 1 0 0.1\n",
                    "2 fp32 40 1 1 0 0.1\n", "3 fp32 18 0 0 0 0.1\n", "2 fp32 18 1 1 0\n", "2 fp32 18 1 1 0 0.1 x\n"):
            f.write_text(bad)
            with pytest.raises(B.RNError):
                B.rn_tune_load(str(f))
            # a refused file leaves the installed table alone
            assert B.rn_plan(n512, mixed)["path"] == B.RN_PATH_2D_SMALL
        with pytest.raises(B.RNError):
            B.rn_tune_load(str(tmp_path / "missing.txt"))
    finally:
        B.rn_tune_reset()
    assert B.rn_plan(n512, mixed) == base512
    assert B.rn_plan(n64c, mixed) == base3d
    assert lib.rn_autotune(None, None, 0) == B.RN_EINVAL
