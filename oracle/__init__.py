"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over ``galsat_oracle.c``.  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import this package; the
product library never loads it.  See ``galsat_oracle.c`` for the paper
passages each function follows and the readings it takes.

Conventions: ``x`` is restart-major float64 ``[R, n]``; losses and counts are
``[F, R]``.  A CNF is anything with the attributes ``clause_ptr``,
``clause_lits``, ``formula_clause_begin`` and ``n`` (int32 numpy arrays); the
oracle reads the clause-major orientation only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "galsat_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libgalsat_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC,
                               "-lm", "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P, i32, i64, f64, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                 ctypes.c_uint64)
        lib.oracle_clause_U.argtypes = [i32, P, P]
        lib.oracle_clause_U.restype = f64
        lib.oracle_loss.argtypes = [i32, i32, P, P, P, i32, P, P]
        lib.oracle_grad.argtypes = [i32, i32, P, P, P, i32, P, P, P, P]
        lib.oracle_grad_def.argtypes = [i32, i32, P, P, P, i32, P, P]
        lib.oracle_fd_grad.argtypes = [i32, i32, P, P, i32, P, i32, P, f64, P]
        lib.oracle_step_sgd.argtypes = [i64, f64, P, P]
        lib.oracle_step_adam.argtypes = [i64, f64, f64, f64, f64, i32, P, P, P, P]
        lib.oracle_unsat.argtypes = [i32, i32, P, P, P, i32, P, P]
        lib.oracle_best.argtypes = [i32, i32, P, P]
        lib.oracle_full_step.argtypes = [i32, i32, P, P, P, i32, f64, P, P, P, P]
        lib.oracle_init_state.argtypes = [u64, i32, i32, P]
        lib.oracle_splitmix64.argtypes = [u64, i32, P]
        lib.oracle_gumbel_noise.argtypes = [u64, i32, i32, i32, P]
        lib.oracle_gumbel_step.argtypes = [i32, i32, P, P, P, i32, P, P, f64, f64, f64, f64, f64,
                                           i32, i32, P, P, P, P, P]
        for fn in ("oracle_loss", "oracle_grad", "oracle_grad_def", "oracle_fd_grad",
                   "oracle_step_sgd", "oracle_step_adam", "oracle_unsat", "oracle_best",
                   "oracle_full_step", "oracle_init_state", "oracle_splitmix64",
                   "oracle_gumbel_noise", "oracle_gumbel_step"):
            getattr(lib, fn).restype = None
        _lib = lib
    return _lib


class use_library:
    """Context manager that points the wrapper at another build of the
    oracle source (the mutation tests compile deliberately broken copies to
    show that the pins catch them)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib, _LIB_PATH
        self._saved = (_lib, _LIB_PATH)
        _lib, _LIB_PATH = None, self.path
        return self

    def __exit__(self, *exc):
        global _lib, _LIB_PATH
        _lib, _LIB_PATH = self._saved
        return False


def build_variant(source_text: str, out_path: str) -> str:
    """Compile an edited copy of the oracle source to out_path."""
    src = out_path + ".c"
    with open(src, "w") as fh:
        fh.write(source_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", src, "-lm",
                           "-o", out_path])
    return out_path


def source() -> str:
    with open(_SRC) as fh:
        return fh.read()


def _p(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be contiguous"
    return a.ctypes.data


def _csr(cnf):
    fcb = np.ascontiguousarray(cnf.formula_clause_begin, dtype=np.int32)
    cp = np.ascontiguousarray(cnf.clause_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(cnf.clause_lits, dtype=np.int32)
    return int(cnf.n), int(fcb.shape[0] - 1), fcb, cp, cl


def _x(x, n):
    x = np.ascontiguousarray(x, dtype=np.float64)
    assert x.ndim == 2 and x.shape[1] == n, "x must be [R, n]"
    return x


def clause_U(codes, xr) -> float:
    codes = np.ascontiguousarray(codes, dtype=np.int32)
    xr = np.ascontiguousarray(xr, dtype=np.float64)
    return _L().oracle_clause_U(len(codes), _p(codes), _p(xr))


def loss(cnf, x) -> np.ndarray:
    n, F, fcb, cp, cl = _csr(cnf)
    x = _x(x, n)
    R = x.shape[0]
    out = np.empty((F, R), dtype=np.float64)
    _L().oracle_loss(n, F, _p(fcb), _p(cp), _p(cl), R, _p(x), _p(out))
    return out


def grad(cnf, x, with_abs: bool = False):
    """(loss [F,R], grad [R,n]) or (loss, grad, absg) with absg the sum of
    |per-occurrence contributions|."""
    n, F, fcb, cp, cl = _csr(cnf)
    x = _x(x, n)
    R = x.shape[0]
    lo = np.empty((F, R), dtype=np.float64)
    g = np.empty((R, n), dtype=np.float64)
    a = np.empty((R, n), dtype=np.float64) if with_abs else None
    _L().oracle_grad(n, F, _p(fcb), _p(cp), _p(cl), R, _p(x), _p(lo), _p(g), _p(a))
    return (lo, g, a) if with_abs else (lo, g)


def grad_def(cnf, x) -> np.ndarray:
    n, F, fcb, cp, cl = _csr(cnf)
    x = _x(x, n)
    R = x.shape[0]
    g = np.empty((R, n), dtype=np.float64)
    _L().oracle_grad_def(n, F, _p(fcb), _p(cp), _p(cl), R, _p(x), _p(g))
    return g


def fd_grad(cnf, x, vars_, h: float = 1e-3) -> np.ndarray:
    """Central differences [R, len(vars_)] over the clauses containing each var."""
    n, F, fcb, cp, cl = _csr(cnf)
    x = _x(x, n)
    R = x.shape[0]
    vs = np.ascontiguousarray(vars_, dtype=np.int32)
    out = np.empty((R, vs.shape[0]), dtype=np.float64)
    _L().oracle_fd_grad(n, int(fcb[-1]), _p(cp), _p(cl), R, _p(x), vs.shape[0], _p(vs), h, _p(out))
    return out


def step_sgd(x, g, lr: float) -> np.ndarray:
    x = np.array(x, dtype=np.float64, order="C", copy=True)
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert x.shape == g.shape
    _L().oracle_step_sgd(x.size, lr, _p(x), _p(g))
    return x


def step_adam(x, mom, vel, g, t: int, lr: float = 0.5, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """Returns (x, mom, vel) after one Adam step at 1-based step t."""
    x = np.array(x, dtype=np.float64, order="C", copy=True)
    mom = np.array(mom, dtype=np.float64, order="C", copy=True)
    vel = np.array(vel, dtype=np.float64, order="C", copy=True)
    g = np.ascontiguousarray(g, dtype=np.float64)
    _L().oracle_step_adam(x.size, lr, b1, b2, eps, t, _p(x), _p(mom), _p(vel), _p(g))
    return x, mom, vel


def unsat(cnf, x) -> np.ndarray:
    n, F, fcb, cp, cl = _csr(cnf)
    x = _x(x, n)
    R = x.shape[0]
    out = np.empty((F, R), dtype=np.int32)
    _L().oracle_unsat(n, F, _p(fcb), _p(cp), _p(cl), R, _p(x), _p(out))
    return out


def best(unsat_fr) -> np.ndarray:
    u = np.ascontiguousarray(unsat_fr, dtype=np.int32)
    F, R = u.shape
    out = np.empty(F, dtype=np.int32)
    _L().oracle_best(F, R, _p(u), _p(out))
    return out


def full_step(cnf, x, lr: float):
    """One iteration at x: returns (loss [F,R], unsat [F,R], grad [R,n], x_next)."""
    n, F, fcb, cp, cl = _csr(cnf)
    x = np.array(_x(x, n), copy=True)
    R = x.shape[0]
    g = np.empty((R, n), dtype=np.float64)
    lo = np.empty((F, R), dtype=np.float64)
    us = np.empty((F, R), dtype=np.int32)
    _L().oracle_full_step(n, F, _p(fcb), _p(cp), _p(cl), R, lr, _p(x), _p(g), _p(lo), _p(us))
    return lo, us, g, x


def init_state(seed: int, n: int, R: int) -> np.ndarray:
    out = np.empty((R, n), dtype=np.float64)
    _L().oracle_init_state(ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), n, R, _p(out))
    return out


def splitmix64(state: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _L().oracle_splitmix64(ctypes.c_uint64(state), count, _p(out))
    return out


def gumbel_noise(seed: int, t: int, n: int, R: int) -> np.ndarray:
    """Noise differences l (= g1 - g0 in law: standard logistic) of step t,
    [R, n], FP64."""
    out = np.empty((R, n), dtype=np.float64)
    _L().oracle_gumbel_noise(ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), t, n, R, _p(out))
    return out


def gumbel_step(cnf, d, noise, tau: float = 1.0, lr: float = 0.5, b1: float = 0.9,
                b2: float = 0.999, eps: float = 1e-8, t: int = 1, adam: bool = True, mom=None,
                vel=None):
    """One straight-through Gumbel step.  d, noise: [R, n] (noise is used as
    FP32).  Returns dict(d, mom, vel, xh, loss [F,R], unsat [F,R])."""
    n, F, fcb, cp, cl = _csr(cnf)
    d = np.array(_x(d, n), copy=True)
    R = d.shape[0]
    l32 = np.ascontiguousarray(noise, dtype=np.float32)
    assert l32.shape == d.shape
    mom = np.zeros_like(d) if mom is None else np.array(mom, dtype=np.float64, copy=True)
    vel = np.zeros_like(d) if vel is None else np.array(vel, dtype=np.float64, copy=True)
    xh = np.empty_like(d)
    lo = np.empty((F, R), dtype=np.float64)
    us = np.empty((F, R), dtype=np.int32)
    _L().oracle_gumbel_step(n, F, _p(fcb), _p(cp), _p(cl), R, _p(d), _p(l32), tau, lr, b1, b2, eps,
                            t, 1 if adam else 0, _p(mom), _p(vel), _p(xh), _p(lo), _p(us))
    return {"d": d, "mom": mom, "vel": vel, "xh": xh, "loss": lo, "unsat": us}
