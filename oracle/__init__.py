"""CPU FP64 oracle for the random-network flow problem -- test infrastructure only.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It wraps ``rn_oracle.c`` (plain C,
single-threaded, FP64) through ctypes; see that file for what each routine
computes and which passage of the paper it follows (Sec. II, Eqs. 3-4).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rn_oracle.c")
_LIB = os.path.join(_HERE, "librn_oracle.so")

STATUS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "not converged", -4: "numerical breakdown"}


def build(force: bool = True) -> str:
    """Compile rn_oracle.c into librn_oracle.so with gcc (-O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("converged", C.c_int32),
                ("Q_in", C.c_double), ("Q_out", C.c_double), ("G", C.c_double), ("K", C.c_double),
                ("rel_resid", C.c_double), ("iters", C.c_int64), ("n_live", C.c_int64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        u8p = C.POINTER(C.c_uint8)
        i64 = C.c_int64
        common = [C.c_int, i64, i64, i64, C.c_int, C.c_int, dp, dp, dp]
        lib.rno_mask_bfs.argtypes = common + [u8p, C.POINTER(i64)]
        lib.rno_mask_uf.argtypes = common + [u8p, C.POINTER(i64)]
        lib.rno_solve.argtypes = common + [C.c_double, i64, C.c_int, C.c_int, dp, u8p, C.POINTER(_Result)]
        lib.rno_check_pressure.argtypes = common + [dp, dp]
        lib.rno_backbone.argtypes = common + [u8p, C.POINTER(i64), C.POINTER(i64)]
        for f in (lib.rno_mask_bfs, lib.rno_mask_uf, lib.rno_solve, lib.rno_check_pressure, lib.rno_backbone):
            f.restype = C.c_int
        _lib = lib
    return _lib


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return C.POINTER(C.c_double)()
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _args(dim: int, nx: int, ny: int, nz: int, axis: int, periodic: bool, g: Sequence[np.ndarray]):
    gs = [np.ascontiguousarray(a, dtype=np.float64) for a in g]
    while len(gs) < 3:
        gs.append(None)
    return gs, [int(dim), int(nx), int(ny), int(nz), int(axis), int(bool(periodic)),
                _dptr(gs[0]), _dptr(gs[1]), _dptr(gs[2])]


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle status {code}: {STATUS.get(code, '?')}")
        self.code = code


@dataclass
class OracleResult:
    status: int
    converged: bool
    Q_in: float
    Q_out: float
    G: float
    K: float
    rel_resid: float
    iters: int
    n_live: int
    pressure: Optional[np.ndarray] = None
    mask: Optional[np.ndarray] = None


def _net_args(net):
    """(dim, nx, ny, nz, axis, periodic, g) of a Network; `periodic` wraps the
    directions other than the flow axis (the side condition of Sec. II)."""
    return net.dim, net.nx, net.ny, net.nz, net.axis, bool(getattr(net, "periodic", False)), net.g


def mask_bfs(net) -> tuple:
    """(mask uint8 array of the node shape, n_live) by two breadth-first searches."""
    keep, a = _args(*_net_args(net))
    out = np.zeros(net.shape, dtype=np.uint8)
    nl = C.c_int64(0)
    st = _load().rno_mask_bfs(*a, out.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(nl))
    if st:
        raise OracleError(st)
    return out, int(nl.value)


def mask_uf(net) -> tuple:
    """Same mask by an independent sequential union-find."""
    keep, a = _args(*_net_args(net))
    out = np.zeros(net.shape, dtype=np.uint8)
    nl = C.c_int64(0)
    st = _load().rno_mask_uf(*a, out.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(nl))
    if st:
        raise OracleError(st)
    return out, int(nl.value)


def backbone(net) -> tuple:
    """(mask, n_live, n_backbone): the mask of mask_bfs with bit3 (8) set on
    the interior nodes of the backbone (nodes on a simple inlet-outlet path),
    by Hopcroft and Tarjan's biconnected components."""
    keep, a = _args(*_net_args(net))
    out = np.zeros(net.shape, dtype=np.uint8)
    nl, nb = C.c_int64(0), C.c_int64(0)
    st = _load().rno_backbone(*a, out.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(nl), C.byref(nb))
    if st:
        raise OracleError(st)
    return out, int(nl.value), int(nb.value)


X0_LINEAR, X0_ZERO = 0, 1
JACOBI, NONE = 0, 1


def solve(net, tol: float = 1e-12, max_iter: int = 1_000_000, want_pressure: bool = True,
          want_mask: bool = False, raise_on_error: bool = True, x0: int = X0_ZERO,
          precond: int = JACOBI) -> OracleResult:
    """Preconditioned CG to ||b - A x|| <= tol ||b|| (FP64), then fluxes, energy G and K.

    ``x0``: X0_ZERO (x = 0) or X0_LINEAR (the linear profile along the flow
    axis); ``precond``: JACOBI (M = diag d) or NONE (M = I)."""
    keep, a = _args(*_net_args(net))
    P = np.zeros(net.shape, dtype=np.float64) if want_pressure else None
    M = np.zeros(net.shape, dtype=np.uint8) if want_mask else None
    res = _Result()
    st = _load().rno_solve(*a, float(tol), int(max_iter), int(x0), int(precond), _dptr(P),
                           M.ctypes.data_as(C.POINTER(C.c_uint8)) if M is not None else C.POINTER(C.c_uint8)(),
                           C.byref(res))
    if st and st != -3 and raise_on_error:
        raise OracleError(st)
    return OracleResult(int(res.status), bool(res.converged), res.Q_in, res.Q_out, res.G, res.K,
                        res.rel_resid, int(res.iters), int(res.n_live), P, M)


@dataclass
class PressureCheck:
    resid: float
    bnorm: float
    Q_in: float
    Q_out: float
    G_E: float
    K_E: float
    p_min: float
    p_max: float
    sum_Ax_minus_b: float
    n_live: int

    @property
    def rel_resid(self) -> float:
        return self.resid / self.bnorm if self.bnorm > 0 else 0.0


def check_pressure(net, P: np.ndarray) -> PressureCheck:
    """Evaluate, with the oracle's own mask and operator, a given full pressure field."""
    keep, a = _args(*_net_args(net))
    Pc = np.ascontiguousarray(P, dtype=np.float64).reshape(net.shape)
    out = np.zeros(10, dtype=np.float64)
    st = _load().rno_check_pressure(*a, _dptr(Pc), _dptr(out))
    if st:
        raise OracleError(st)
    return PressureCheck(*[float(v) for v in out[:9]], int(out[9]))
