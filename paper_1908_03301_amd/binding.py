"""ctypes binding of librn (include/rn.h): argument marshalling only.

Every step of the solve runs in librn's HIP kernels; this module converts
numpy arrays (host memory) or torch CUDA tensors (device memory) into the C
structures and calls the entry points of the same names. It raises
``RuntimeError`` when librn.so has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librn.so")

RN_OK, RN_EINVAL, RN_ENOMEM, RN_ENOCONV, RN_ENUMERIC, RN_EDEVICE, RN_EAGAIN, RN_ENOTFOUND = 0, -1, -2, -3, -4, -5, -6, -7
RN_FP64, RN_MIXED = 0, 1
RN_JACOBI, RN_NONE = 0, 1
RN_X0_LINEAR, RN_X0_ZERO = 0, 1
RN_MEM_HOST, RN_MEM_DEVICE = 0, 1
RN_PERIODIC = 1
RN_OPT_BACKBONE = 1
RN_OPT_COMPACT = 2
RN_PATH_2D_FULL, RN_PATH_2D_SMALL, RN_PATH_3D = 0, 1, 2

EXPORTED = ["rn_version", "rn_strerror", "rn_opts_default", "rn_create", "rn_destroy", "rn_set_stream",
            "rn_last_error", "rn_validate", "rn_footprint", "rn_build_mask", "rn_solve", "rn_solve_batch",
            "rn_submit", "rn_poll", "rn_stats", "rn_plan", "rn_fbm_field", "rn_fbm_bonds",
            "rn_build_mask_noalloc", "rn_set_timing", "rn_autotune", "rn_tune_load", "rn_tune_reset",
            "rn_build_backbone"]
RN_TUNE_QUICK = 1
RN_NOALLOC_MAX_NODES = 1 << 22


class rn_problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("axis", C.c_int32),
                ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
                ("g", C.c_void_p * 3), ("p_out", C.c_void_p), ("mask_out", C.c_void_p),
                ("mem", C.c_int32), ("flags", C.c_int32)]


class rn_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("precond", C.c_int32), ("tol", C.c_double),
                ("max_iter", C.c_int64), ("delta", C.c_double), ("x0", C.c_int32), ("flags", C.c_int32)]


class rn_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("converged", C.c_int32),
                ("Q_in", C.c_double), ("Q_out", C.c_double), ("G", C.c_double), ("K", C.c_double),
                ("rel_resid", C.c_double), ("iters", C.c_int64), ("refreshes", C.c_int64),
                ("n_live", C.c_int64), ("passes", C.c_int64),
                ("t_mask_s", C.c_double), ("t_loop_s", C.c_double), ("t_total_s", C.c_double),
                ("n_backbone", C.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class rn_stats_t(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("waiting", "preparing", "active", "finishing", "bytes_in_use", "budget",
                                          "launches", "peak_active")] + \
               [("pass_device_s", (C.c_double * 2) * 3), ("pass_timed_launches", (C.c_int64 * 2) * 3)]

    def as_dict(self) -> dict:
        out = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            out[k] = [[v[a][b] for b in range(2)] for a in range(3)] if k.startswith("pass_") else v
        return out


class rn_plan_t(C.Structure):
    _fields_ = [("path", C.c_int32), ("tiles_per_wg", C.c_int32), ("tile_x", C.c_int32), ("tile_y", C.c_int32),
                ("tile_z", C.c_int32), ("tiles", C.c_int32), ("workgroups", C.c_int32), ("groups", C.c_int32),
                ("footprint", C.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class RNError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"librn status {code} ({strerror(code)}){': ' + msg if msg else ''}")
        self.code = code


_lib = None


def lib():
    """Load librn.so (built in-tree by ``__graft_entry__.build()``); no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P, I64 = C.POINTER, C.c_int64
        L.rn_version.restype = C.c_int
        L.rn_strerror.argtypes = [C.c_int]
        L.rn_strerror.restype = C.c_char_p
        L.rn_opts_default.argtypes = [P(rn_opts)]
        L.rn_create.argtypes = [C.c_int, C.c_size_t, P(C.c_void_p)]
        L.rn_destroy.argtypes = [C.c_void_p]
        L.rn_set_stream.argtypes = [C.c_void_p, C.c_void_p]
        L.rn_last_error.argtypes = [C.c_void_p]
        L.rn_last_error.restype = C.c_char_p
        L.rn_validate.argtypes = [P(rn_problem), P(rn_opts)]
        L.rn_validate.restype = C.c_int
        L.rn_footprint.argtypes = [P(rn_problem), P(rn_opts)]
        L.rn_footprint.restype = C.c_size_t
        L.rn_build_mask.argtypes = [C.c_void_p, P(rn_problem), P(I64)]
        L.rn_build_mask_noalloc.argtypes = [C.c_void_p, P(rn_problem), P(I64)]
        L.rn_build_backbone.argtypes = [C.c_void_p, P(rn_problem), P(I64), P(I64)]
        L.rn_solve.argtypes = [C.c_void_p, P(rn_problem), P(rn_opts), P(rn_result)]
        L.rn_solve_batch.argtypes = [C.c_void_p, C.c_int32, P(rn_problem), P(rn_opts), C.c_int32, P(rn_result)]
        L.rn_submit.argtypes = [C.c_void_p, P(rn_problem), P(rn_opts), P(C.c_uint64)]
        L.rn_poll.argtypes = [C.c_void_p, C.c_uint64, P(rn_result)]
        L.rn_stats.argtypes = [C.c_void_p, P(rn_stats_t)]
        L.rn_set_timing.argtypes = [C.c_void_p, C.c_int]
        L.rn_autotune.argtypes = [C.c_void_p, C.c_char_p, C.c_int32]
        L.rn_tune_load.argtypes = [C.c_char_p]
        L.rn_tune_reset.argtypes = []
        L.rn_plan.argtypes = [P(rn_problem), P(rn_opts), P(rn_plan_t)]
        D, DA3 = P(C.c_double), C.c_void_p * 3
        L.rn_fbm_field.argtypes = [C.c_void_p, C.c_int32, I64, I64, I64, C.c_double, D, C.c_void_p, C.c_void_p,
                                   C.c_int32]
        L.rn_fbm_bonds.argtypes = [C.c_void_p, C.c_int32, I64, I64, I64, C.c_void_p, C.c_double, C.c_int32,
                                   P(DA3), C.c_double, P(DA3), C.c_int32]
        for f in ("rn_opts_default", "rn_create", "rn_destroy", "rn_set_stream", "rn_build_mask",
                  "rn_build_mask_noalloc", "rn_set_timing", "rn_autotune", "rn_tune_load", "rn_tune_reset",
                  "rn_build_backbone", "rn_solve",
                  "rn_solve_batch", "rn_submit", "rn_poll", "rn_stats", "rn_plan", "rn_fbm_field", "rn_fbm_bonds"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().rn_strerror(int(code)).decode()
    except RuntimeError:
        return str(code)


def opts(precision: int = RN_FP64, tol: float = 1e-8, max_iter: int = 10_000_000, delta: float = 0.0,
         precond: int = RN_JACOBI, x0: int = RN_X0_LINEAR, backbone: bool = False, compact: bool = False) -> rn_opts:
    o = rn_opts()
    lib().rn_opts_default(C.byref(o))
    o.precision, o.tol, o.max_iter, o.delta = int(precision), float(tol), int(max_iter), float(delta)
    o.precond, o.x0 = int(precond), int(x0)
    o.flags = (RN_OPT_BACKBONE if backbone else 0) | (RN_OPT_COMPACT if compact else 0)
    return o


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


@dataclass
class Problem:
    """An rn_problem plus references that keep its buffers alive.

    ``device`` is the CUDA device index of its buffers (None: host memory)."""
    c: rn_problem
    keep: list
    device: Optional[int] = None


def _check_device_buffer(name: str, a, n: int, dtype: str, device: Optional[int]) -> int:
    """Raise ValueError unless `a` is a contiguous CUDA tensor of n elements of
    `dtype` on `device`; returns its device index."""
    if not _is_torch(a):
        raise ValueError(f"{name}: device problems take CUDA tensors for every buffer")
    if not a.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if str(a.dtype) != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, not {a.dtype}")
    if not a.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if a.numel() != n:
        raise ValueError(f"{name} has {a.numel()} elements; the lattice has {n} nodes")
    if device is not None and a.device.index != device:
        raise ValueError(f"{name} is on cuda:{a.device.index}, the other buffers on cuda:{device}")
    return a.device.index


def _check_host_buffer(name: str, a, n: int, dtype) -> None:
    if not (isinstance(a, np.ndarray) and a.dtype == dtype and a.flags["C_CONTIGUOUS"]):
        raise ValueError(f"{name} must be a C-contiguous {np.dtype(dtype).name} numpy array")
    if a.size != n:
        raise ValueError(f"{name} has {a.size} elements; the lattice has {n} nodes")


def problem(net=None, *, dim=None, nx=None, ny=None, nz=1, axis=0, g: Optional[Sequence] = None,
            p_out=None, mask_out=None, periodic: Optional[bool] = None) -> Problem:
    """Build an rn_problem from a Network (inputs.Network) or explicit fields.

    ``g`` entries are float64 numpy arrays (host) or float64 CUDA tensors
    (device); ``p_out`` / ``mask_out`` must be in the same memory space.
    ``periodic`` (default: the Network's own setting, else False) sets
    RN_PERIODIC: the directions other than the flow axis wrap around.
    """
    if net is not None:
        dim, nx, ny, nz, axis, g = net.dim, net.nx, net.ny, net.nz, net.axis, net.g
        if periodic is None:
            periodic = bool(getattr(net, "periodic", False))
    keep: List = []
    pr = rn_problem()
    pr.dim, pr.axis, pr.nx, pr.ny, pr.nz = int(dim), int(axis), int(nx), int(ny), int(nz)
    pr.flags = RN_PERIODIC if periodic else 0
    n = int(nx) * int(ny) * int(nz)
    device = any(_is_torch(a) for a in g if a is not None)
    pr.mem = RN_MEM_DEVICE if device else RN_MEM_HOST
    dev_index: Optional[int] = None
    for k in range(3):
        a = g[k] if k < len(g) else None
        if a is None:
            pr.g[k] = None
            continue
        if device:
            dev_index = _check_device_buffer(f"g[{k}]", a, n, "torch.float64", dev_index)
            pr.g[k] = a.data_ptr()
        else:
            a = np.ascontiguousarray(a, dtype=np.float64)
            if a.size != n:
                raise ValueError(f"g[{k}] has {a.size} elements; the lattice has {n} nodes")
            pr.g[k] = a.ctypes.data
        keep.append(a)
    for name, arr, dt in (("p_out", p_out, np.float64), ("mask_out", mask_out, np.uint8)):
        if arr is None:
            setattr(pr, name, None)
            continue
        if device:
            _check_device_buffer(name, arr, n, "torch.float64" if dt is np.float64 else "torch.uint8", dev_index)
            setattr(pr, name, arr.data_ptr())
        else:
            _check_host_buffer(name, arr, n, dt)
            setattr(pr, name, arr.ctypes.data)
        keep.append(arr)
    return Problem(pr, keep, dev_index)


class Context:
    """An rn_ctx on one device (rn_create / rn_destroy)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = C.c_void_p()
        st = lib().rn_create(int(device), C.c_size_t(hbm_budget_bytes), C.byref(h))
        if st:
            raise RNError(st)
        self.h = h
        self.device = int(device)

    def _own(self, prob: "Problem") -> "Problem":
        """Raise ValueError when a device problem's buffers are on another GPU."""
        if prob.device is not None and prob.device != self.device:
            raise ValueError(f"problem buffers are on cuda:{prob.device}, the context on cuda:{self.device}")
        return prob

    def close(self):
        if getattr(self, "h", None):
            lib().rn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def last_error(self) -> str:
        return lib().rn_last_error(self.h).decode()

    def set_stream(self, stream_handle: Optional[int]):
        st = lib().rn_set_stream(self.h, C.c_void_p(stream_handle or 0))
        if st:
            raise RNError(st)

    def footprint(self, prob: Problem, o: Optional[rn_opts] = None) -> int:
        return int(lib().rn_footprint(C.byref(prob.c), C.byref(o) if o is not None else None))

    def fbm_field(self, dim: int, nx: int, ny: int, nz: int, H: float, noise, out, beta=None):
        """rn_fbm_field: `noise` and `out` are float64 numpy arrays (host) or
        contiguous float64 CUDA tensors (device) of nx*ny*nz nodes; `beta` per
        lattice direction (x, y, z) or None."""
        dev = _is_torch(noise)
        ptr = (lambda a: a.data_ptr()) if dev else (lambda a: a.ctypes.data)
        n = int(nx) * int(ny) * int(nz)
        for name, a in (("noise", noise), ("out", out)):
            if dev:
                if _check_device_buffer(name, a, n, "torch.float64", None) != self.device:
                    raise ValueError(f"{name} is not on the context's device cuda:{self.device}")
            else:
                _check_host_buffer(name, a, n, np.float64)
        b = (C.c_double * 3)(*([float(v) for v in beta] + [1.0] * (3 - len(beta)))) if beta is not None else None
        st = lib().rn_fbm_field(self.h, int(dim), int(nx), int(ny), int(nz), float(H), b, C.c_void_p(ptr(noise)),
                                C.c_void_p(ptr(out)), RN_MEM_DEVICE if dev else RN_MEM_HOST)
        if st:
            raise RNError(st, self.last_error())

    def fbm_bonds(self, dim: int, nx: int, ny: int, nz: int, field, sigma: float, periodic: bool, g_out,
                  u=None, occupancy: float = 1.0):
        """rn_fbm_bonds: `g_out` (and `u` when given) hold dim arrays like `field`."""
        dev = _is_torch(field)
        ptr = (lambda a: a.data_ptr()) if dev else (lambda a: a.ctypes.data)
        n = int(nx) * int(ny) * int(nz)
        if len(g_out) != int(dim) or (u is not None and len(u) != int(dim)):
            raise ValueError("g_out (and u) need one array per lattice direction")
        arrs = [field] + list(g_out) + (list(u) if u is not None else [])
        for k, a in enumerate(arrs):
            if dev:
                if _check_device_buffer(f"array {k}", a, n, "torch.float64", None) != self.device:
                    raise ValueError(f"array {k} is not on the context's device cuda:{self.device}")
            else:
                _check_host_buffer(f"array {k}", a, n, np.float64)
        DA3 = C.c_void_p * 3
        g3 = DA3(*([ptr(a) for a in g_out] + [None] * (3 - len(g_out))))
        u3 = DA3(*([ptr(a) for a in u] + [None] * (3 - len(u)))) if u is not None else None
        st = lib().rn_fbm_bonds(self.h, int(dim), int(nx), int(ny), int(nz), C.c_void_p(ptr(field)), float(sigma),
                                int(bool(periodic)), C.byref(u3) if u3 is not None else None, float(occupancy),
                                C.byref(g3), RN_MEM_DEVICE if dev else RN_MEM_HOST)
        if st:
            raise RNError(st, self.last_error())

    def build_mask(self, prob: Problem) -> int:
        nl = C.c_int64(0)
        st = lib().rn_build_mask(self.h, C.byref(self._own(prob).c), C.byref(nl))
        if st:
            raise RNError(st, self.last_error())
        return int(nl.value)

    def build_mask_noalloc(self, prob: Problem) -> int:
        """rn_build_mask_noalloc: device buffers only, nothing allocated by the library."""
        nl = C.c_int64(0)
        st = lib().rn_build_mask_noalloc(self.h, C.byref(self._own(prob).c), C.byref(nl))
        if st:
            raise RNError(st, self.last_error())
        return int(nl.value)

    def build_backbone(self, prob: Problem):
        """rn_build_backbone: (n_live, n_backbone); prob's mask gets bit 3 on backbone nodes."""
        nl, nb = C.c_int64(0), C.c_int64(0)
        st = lib().rn_build_backbone(self.h, C.byref(self._own(prob).c), C.byref(nl), C.byref(nb))
        if st:
            raise RNError(st, self.last_error())
        return int(nl.value), int(nb.value)

    def solve(self, prob: Problem, o: Optional[rn_opts] = None, check: bool = True) -> rn_result:
        res = rn_result()
        st = lib().rn_solve(self.h, C.byref(self._own(prob).c), C.byref(o) if o is not None else None, C.byref(res))
        if check and st not in (RN_OK, RN_ENOCONV):
            raise RNError(st, self.last_error())
        return res


    def solve_batch(self, probs: Sequence[Problem], o=None, check: bool = True) -> List[rn_result]:
        """rn_solve_batch: o is None (defaults), one rn_opts, or a list with one per problem."""
        n = len(probs)
        arr = (rn_problem * n)(*[self._own(pb).c for pb in probs])
        res = (rn_result * n)()
        if o is None:
            opt_arr, n_opts = None, 0
        elif isinstance(o, rn_opts):
            opt_arr, n_opts = (rn_opts * 1)(o), 1
        else:
            opt_arr, n_opts = (rn_opts * n)(*o), n
        st = lib().rn_solve_batch(self.h, n, arr, opt_arr, n_opts, res)
        if check and st not in (RN_OK, RN_ENOCONV, RN_ENUMERIC):
            raise RNError(st, self.last_error())
        return [res[i] for i in range(n)]

    def submit(self, prob: Problem, o: Optional[rn_opts] = None) -> int:
        """rn_submit: queue a solve; prob's buffers must outlive the ticket."""
        t = C.c_uint64(0)
        st = lib().rn_submit(self.h, C.byref(self._own(prob).c), C.byref(o) if o is not None else None, C.byref(t))
        if st:
            raise RNError(st, self.last_error())
        return int(t.value)

    def poll(self, ticket: int):
        """rn_poll: (status, rn_result) with status RN_EAGAIN while running."""
        res = rn_result()
        st = lib().rn_poll(self.h, C.c_uint64(ticket), C.byref(res))
        return st, res

    def set_timing(self, enable: bool) -> None:
        """rn_set_timing: per-launch device timing of the pass kernels into stats()."""
        st = lib().rn_set_timing(self.h, int(bool(enable)))
        if st:
            raise RNError(st)

    def autotune(self, cache_path: Optional[str] = None, quick: bool = False) -> None:
        """rn_autotune: measure the launch shapes on this device and install them process-wide."""
        st = lib().rn_autotune(self.h, cache_path.encode() if cache_path else None, RN_TUNE_QUICK if quick else 0)
        if st:
            raise RNError(st, self.last_error())

    def stats(self) -> dict:
        s = rn_stats_t()
        st = lib().rn_stats(self.h, C.byref(s))
        if st:
            raise RNError(st)
        return s.as_dict()


# module-level names matching the C ABI
def rn_validate(prob: Problem, o: Optional[rn_opts] = None) -> int:
    return int(lib().rn_validate(C.byref(prob.c), C.byref(o) if o is not None else None))


def rn_footprint(prob: Problem, o: Optional[rn_opts] = None) -> int:
    return int(lib().rn_footprint(C.byref(prob.c), C.byref(o) if o is not None else None))


def rn_plan(prob: Problem, o: Optional[rn_opts] = None) -> dict:
    """rn_plan: the launch plan of a network as a dict (RNError if invalid)."""
    out = rn_plan_t()
    st = lib().rn_plan(C.byref(prob.c), C.byref(o) if o is not None else None, C.byref(out))
    if st:
        raise RNError(st)
    return out.as_dict()


def rn_tune_load(path: str) -> None:
    """rn_tune_load: install a launch-shape table file (host only)."""
    st = lib().rn_tune_load(path.encode())
    if st:
        raise RNError(st)


def rn_tune_reset() -> None:
    lib().rn_tune_reset()


def rn_version() -> int:
    return int(lib().rn_version())


def rn_create(device: int = 0, hbm_budget_bytes: int = 0) -> Context:
    return Context(device, hbm_budget_bytes)


def rn_build_mask(ctx: Context, prob: Problem) -> int:
    return ctx.build_mask(prob)


def rn_build_mask_noalloc(ctx: Context, prob: Problem) -> int:
    return ctx.build_mask_noalloc(prob)


def rn_build_backbone(ctx: Context, prob: Problem):
    return ctx.build_backbone(prob)


def backbone_network(ctx: Context, net):
    """Host-memory convenience: (mask with bit 3 on the backbone, n_live, n_backbone)."""
    M = np.zeros(net.shape, dtype=np.uint8)
    nl, nb = ctx.build_backbone(problem(net, mask_out=M))
    return M, nl, nb


def rn_solve(ctx: Context, prob: Problem, o: Optional[rn_opts] = None) -> rn_result:
    return ctx.solve(prob, o)


def solve_network(ctx: Context, net, precision: int = RN_FP64, tol: float = 1e-8, max_iter: int = 10_000_000,
                  want_pressure: bool = False, want_mask: bool = False, delta: float = 0.0,
                  precond: int = RN_JACOBI, x0: int = RN_X0_LINEAR, backbone: bool = False, compact: bool = False):
    """Host-memory convenience: returns (rn_result, pressure or None, mask or None)."""
    P = np.zeros(net.shape, dtype=np.float64) if want_pressure else None
    M = np.zeros(net.shape, dtype=np.uint8) if want_mask else None
    pr = problem(net, p_out=P, mask_out=M)
    res = ctx.solve(pr, opts(precision, tol, max_iter, delta, precond, x0, backbone, compact))
    return res, P, M
