"""Seeded synthetic CNF workloads and CSR construction.

This module only BUILDS inputs.  It contains none of the method's arithmetic
(no clause polynomial, gradient, update or rounding), so the CPU oracle and
the HIP path can both draw the same instances from it without sharing any
code that computes a result.

The paper evaluates on the SAT Competition 2024 instances (Section 4 and the
appendix's experiment setup); those are not available here, so seeded
synthetic families of matching structure stand in for them:

* planted random k-SAT (clause/variable ratio 4.26, uniform variables);
* mixed-length clauses (2 + geometric, mean 4) with Zipf-popular variables
  inside 1,000 communities and 90 % intra-community literals;
* an uneven batch of thousands of small planted formulas;
* one large formula with 5 % long clauses (50-200 literals) and global
  Zipf(1.2) variable popularity.

Every generator plants a hidden assignment: a clause that the hidden
assignment falsifies gets one uniformly chosen literal flipped, so the
formula is satisfiable and the planted assignment satisfies every clause.

Literal code convention: ``code = 2 * var + neg`` with 0-based variable ids
(``neg = 1`` for a negated literal).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Iterable, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.cpp")
_LIB_PATH = os.path.join(_HERE, "libgalsat_inputs.so")
_lib = None


def build_lib(force: bool = True) -> str:
    """Compile the generator library with g++ (host code only)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["g++", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared", "-std=c++17",
               _SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class GenSpec(ctypes.Structure):
    _fields_ = [
        ("len_kind", ctypes.c_int32),
        ("k0", ctypes.c_int32), ("ka", ctypes.c_int32), ("kb", ctypes.c_int32),
        ("kmax", ctypes.c_int32),
        ("p0", ctypes.c_double), ("geom_p", ctypes.c_double),
        ("var_kind", ctypes.c_int32),
        ("n_comm", ctypes.c_int32),
        ("zipf_s", ctypes.c_double),
        ("p_intra", ctypes.c_double),
        ("plant", ctypes.c_int32),
        ("distinct", ctypes.c_int32),
    ]


def _get_lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_lib(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.gen_batch_sizes.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_double, ctypes.c_double, P, P]
        lib.gen_batch_sizes.restype = None
        lib.gen_lengths.argtypes = [ctypes.POINTER(GenSpec), ctypes.c_uint64, ctypes.c_int32, P, P]
        lib.gen_lengths.restype = ctypes.c_int
        lib.gen_literals.argtypes = [ctypes.POINTER(GenSpec), ctypes.c_uint64, ctypes.c_int32,
                                     P, P, P, P, P]
        lib.gen_literals.restype = ctypes.c_int
        lib.gen_transpose.argtypes = [ctypes.c_int32, P, P, P, P, P, P]
        lib.gen_transpose.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


@dataclass
class CNF:
    """A batch of F CNF formulas in both CSR orientations.

    clause_ptr[m+1], clause_lits[L]   clause-major: literal codes of clause t
                                      at clause_lits[clause_ptr[t]:clause_ptr[t+1]]
    var_ptr[n+1], var_occ[L]          variable-major: positions p into
                                      clause_lits with clause_lits[p] >> 1 == v,
                                      increasing p within a variable
    formula_var_begin[F+1], formula_clause_begin[F+1]
                                      contiguous variable and clause ranges of
                                      each formula (global ids)
    planted[n]                        hidden satisfying assignment (or None)
    """

    clause_ptr: np.ndarray
    clause_lits: np.ndarray
    var_ptr: np.ndarray
    var_occ: np.ndarray
    formula_var_begin: np.ndarray
    formula_clause_begin: np.ndarray
    planted: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.var_ptr.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.clause_ptr.shape[0] - 1)

    @property
    def L(self) -> int:
        return int(self.clause_lits.shape[0])

    @property
    def F(self) -> int:
        return int(self.formula_var_begin.shape[0] - 1)

    def clause_lengths(self) -> np.ndarray:
        return np.diff(self.clause_ptr)

    def clauses(self) -> List[List[int]]:
        """Clause list of literal codes (small formulas only)."""
        cp, cl = self.clause_ptr, self.clause_lits
        return [cl[cp[t]:cp[t + 1]].tolist() for t in range(self.m)]

    def formula_of_var(self) -> np.ndarray:
        return np.repeat(np.arange(self.F, dtype=np.int32), np.diff(self.formula_var_begin))

    def formula_of_clause(self) -> np.ndarray:
        return np.repeat(np.arange(self.F, dtype=np.int32), np.diff(self.formula_clause_begin))

    def sub(self, f: int) -> "CNF":
        """Formula f alone, with variables renumbered from 0."""
        v0, v1 = int(self.formula_var_begin[f]), int(self.formula_var_begin[f + 1])
        c0, c1 = int(self.formula_clause_begin[f]), int(self.formula_clause_begin[f + 1])
        p0, p1 = int(self.clause_ptr[c0]), int(self.clause_ptr[c1])
        cp = (self.clause_ptr[c0:c1 + 1] - p0).astype(np.int32)
        cl = (self.clause_lits[p0:p1] - 2 * v0).astype(np.int32)
        pl = None if self.planted is None else self.planted[v0:v1].copy()
        return csr_from_clause_major(v1 - v0, cp, cl, planted=pl, name=f"{self.name}[{f}]")


def transpose(F: int, var_begin: np.ndarray, clause_begin: np.ndarray, clause_ptr: np.ndarray,
              clause_lits: np.ndarray):
    """Variable-major CSR (var_ptr, var_occ) of a clause-major CSR."""
    lib = _get_lib()
    n = int(var_begin[F])
    vb = np.ascontiguousarray(var_begin, dtype=np.int64)
    cb = np.ascontiguousarray(clause_begin, dtype=np.int64)
    cp = np.ascontiguousarray(clause_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(clause_lits, dtype=np.int32)
    var_ptr = np.empty(n + 1, dtype=np.int32)
    var_occ = np.empty(cl.shape[0], dtype=np.int32)
    rc = lib.gen_transpose(F, _ptr(vb), _ptr(cb), _ptr(cp), _ptr(cl), _ptr(var_ptr), _ptr(var_occ))
    if rc != 0:
        raise ValueError("transpose: a literal refers to a variable outside [0, n)")
    return var_ptr, var_occ


def csr_from_clause_major(n: int, clause_ptr, clause_lits, planted=None, name: str = "") -> CNF:
    clause_ptr = np.ascontiguousarray(clause_ptr, dtype=np.int32)
    clause_lits = np.ascontiguousarray(clause_lits, dtype=np.int32)
    if clause_lits.size and (clause_lits.min() < 0 or (clause_lits >> 1).max() >= n):
        raise ValueError("literal code out of range")
    vb = np.array([0, n], dtype=np.int64)
    cb = np.array([0, clause_ptr.shape[0] - 1], dtype=np.int64)
    var_ptr, var_occ = transpose(1, vb, cb, clause_ptr, clause_lits)
    return CNF(clause_ptr, clause_lits, var_ptr, var_occ,
               np.array([0, n], dtype=np.int32), np.array([0, clause_ptr.shape[0] - 1], dtype=np.int32),
               planted, name)


def from_clauses(clauses: Sequence[Sequence[int]], n: Optional[int] = None, dimacs: bool = True,
                 name: str = "") -> CNF:
    """Build a CNF from a clause list.

    With ``dimacs=True`` literals are DIMACS integers (+v / -v, 1-based);
    otherwise they are literal codes 2*v+neg.
    """
    codes: List[int] = []
    ptr = [0]
    maxv = -1
    for c in clauses:
        for lit in c:
            if dimacs:
                if lit == 0:
                    raise ValueError("0 is not a DIMACS literal")
                v, neg = abs(lit) - 1, 1 if lit < 0 else 0
                code = 2 * v + neg
            else:
                code = int(lit)
            codes.append(code)
            maxv = max(maxv, code >> 1)
        ptr.append(len(codes))
    if n is None:
        n = maxv + 1
    return csr_from_clause_major(n, np.array(ptr, dtype=np.int32),
                                 np.array(codes, dtype=np.int32), name=name)


def concat(formulas: Sequence[CNF], name: str = "") -> CNF:
    """Stack independent formulas into one batch with global ids."""
    vb, cb = [0], [0]
    cps, cls, pls = [], [], []
    lit_off = 0
    for g in formulas:
        cps.append(g.clause_ptr[:-1] + lit_off)
        cls.append(g.clause_lits + 2 * vb[-1])
        pls.append(g.planted if g.planted is not None else np.zeros(g.n, np.uint8))
        lit_off += g.L
        vb.append(vb[-1] + g.n)
        cb.append(cb[-1] + g.m)
    cp = np.concatenate(cps + [np.array([lit_off])]).astype(np.int32)
    cl = np.concatenate(cls).astype(np.int32) if cls else np.zeros(0, np.int32)
    vb_a, cb_a = np.array(vb, dtype=np.int64), np.array(cb, dtype=np.int64)
    var_ptr, var_occ = transpose(len(formulas), vb_a, cb_a, cp, cl)
    return CNF(cp, cl, var_ptr, var_occ, vb_a.astype(np.int32), cb_a.astype(np.int32),
               np.concatenate(pls).astype(np.uint8), name)


def read_dimacs(path: str) -> CNF:
    clauses, cur, n = [], [], None
    with open(path) as fh:
        for line in fh:
            s = line.strip()
            if not s or s[0] in "c%":
                continue
            if s[0] == "p":
                n = int(s.split()[2])
                continue
            for tok in s.split():
                v = int(tok)
                if v == 0:
                    clauses.append(cur)
                    cur = []
                else:
                    cur.append(v)
    if cur:
        clauses.append(cur)
    return from_clauses(clauses, n=n, name=os.path.basename(path))


def write_dimacs(cnf: CNF, path: str) -> None:
    with open(path, "w") as fh:
        fh.write(f"p cnf {cnf.n} {cnf.m}\n")
        for c in cnf.clauses():
            fh.write(" ".join(str((x >> 1) + 1 if not (x & 1) else -((x >> 1) + 1)) for x in c))
            fh.write(" 0\n")


def generate(spec: GenSpec, seed: int, n_f: Sequence[int], m_f: Sequence[int], name: str = "") -> CNF:
    """Generate F formulas with the given sizes (global variable ids)."""
    lib = _get_lib()
    F = len(n_f)
    vb = np.zeros(F + 1, dtype=np.int64)
    vb[1:] = np.cumsum(np.asarray(n_f, dtype=np.int64))
    cb = np.zeros(F + 1, dtype=np.int64)
    cb[1:] = np.cumsum(np.asarray(m_f, dtype=np.int64))
    m = int(cb[-1])
    lens = np.empty(m, dtype=np.int32)
    lib.gen_lengths(ctypes.byref(spec), ctypes.c_uint64(seed), F, _ptr(cb), _ptr(lens))
    cp64 = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lens, out=cp64[1:])
    if cp64[-1] >= 2 ** 31:
        raise OverflowError("literal count exceeds int32 CSR range")
    cp = cp64.astype(np.int32)
    del cp64, lens
    lits = np.empty(int(cp[-1]), dtype=np.int32)
    planted = np.empty(int(vb[-1]), dtype=np.uint8)
    rc = lib.gen_literals(ctypes.byref(spec), ctypes.c_uint64(seed), F, _ptr(vb), _ptr(cb), _ptr(cp),
                          _ptr(lits), _ptr(planted))
    if rc != 0:
        raise ValueError("generator: clause longer than its formula's variable count, "
                         "or communities do not divide n")
    var_ptr, var_occ = transpose(F, vb, cb, cp, lits)
    return CNF(cp, lits, var_ptr, var_occ, vb.astype(np.int32), cb.astype(np.int32), planted, name)


def spec(len_kind=0, k0=3, ka=0, kb=0, kmax=0, p0=1.0, geom_p=0.0, var_kind=0, n_comm=0,
         zipf_s=0.0, p_intra=1.0, plant=1, distinct=1) -> GenSpec:
    return GenSpec(len_kind, k0, ka, kb, kmax, p0, geom_p, var_kind, n_comm, zipf_s, p_intra, plant,
                   distinct)


SEED_BASE = 0x6A150000


# --- the five workloads ----------------------------------------------------

def planted_ksat(n: int, m: int, k: int = 3, seed: int = SEED_BASE + 1, name: str = "") -> CNF:
    """Planted random k-SAT, variables uniform, k distinct variables per clause."""
    return generate(spec(0, k0=k), seed, [n], [m], name or f"planted{k}sat_n{n}_m{m}")


def structured_mixed(n: int = 1_000_000, m: int = 4_000_000, n_comm: int = 1000,
                     seed: int = SEED_BASE + 3, name: str = "") -> CNF:
    """Mixed clause lengths 2 + Geometric(1/3) (redrawn above 30; mean 4),
    n_comm contiguous communities, 90 % intra-community literals, Zipf(1.5)
    popularity within a community over a seeded permutation of its members."""
    sp = spec(1, k0=3, kmax=30, geom_p=1.0 / 3.0, var_kind=2, n_comm=n_comm, zipf_s=1.5,
              p_intra=0.9)
    return generate(sp, seed, [n], [m], name or f"mixed_n{n}_m{m}")


def uneven_batch(F: int = 4096, nmin: int = 50, nmax: int = 20000, rmin: float = 3.5,
                 rmax: float = 4.3, seed: int = SEED_BASE + 4, name: str = "") -> CNF:
    """F independent planted formulas; n_f uniform in [nmin, nmax], ratio
    uniform in [rmin, rmax), clause length 3 w.p. 0.8 else uniform in 4..8."""
    lib = _get_lib()
    n_f = np.empty(F, dtype=np.int64)
    m_f = np.empty(F, dtype=np.int64)
    lib.gen_batch_sizes(ctypes.c_uint64(seed), F, nmin, nmax, rmin, rmax, _ptr(n_f), _ptr(m_f))
    sp = spec(2, k0=3, ka=4, kb=8, p0=0.8)
    return generate(sp, seed, n_f.tolist(), m_f.tolist(), name or f"batch_F{F}")


def large_zipf(n: int = 10_000_000, m: int = 42_000_000, seed: int = SEED_BASE + 5,
               name: str = "") -> CNF:
    """95 % 3-literal clauses and 5 % long clauses (uniform 50..200 literals),
    variables by global Zipf(1.2) over a seeded permutation of ids."""
    sp = spec(2, k0=3, ka=50, kb=200, p0=0.95, var_kind=1, zipf_s=1.2)
    return generate(sp, seed, [n], [m], name or f"large_n{n}_m{m}")


@dataclass(frozen=True)
class Workload:
    """A run configuration: instance family and sizes, restarts R, steps, lr."""
    key: str
    description: str
    restarts: int
    steps: int
    lr: float
    make: object  # callable() -> CNF
    recompute: int = 0  # 0 auto, 1 store partials, 2 recompute


WORKLOADS = {
    "planted3sat_n200": Workload(
        "planted3sat_n200", "planted random 3-SAT n=200 m=852, R=64, 500 steps, lr 0.1",
        64, 500, 0.1, lambda: planted_ksat(200, 852, 3, SEED_BASE + 1)),
    "planted3sat_n1e5": Workload(
        "planted3sat_n1e5", "planted random 3-SAT n=100000 m=426000, R=1024, 1000 steps, lr 0.1",
        1024, 1000, 0.1, lambda: planted_ksat(100_000, 426_000, 3, SEED_BASE + 2)),
    "mixed_n1e6": Workload(
        "mixed_n1e6", "mixed k 2-30 (mean 4), Zipf 1.5, 1000 communities, n=1e6 m=4e6, R=256, "
        "100 steps, lr 0.1, recompute", 256, 100, 0.1, lambda: structured_mixed(), recompute=2),
    "batch4096": Workload(
        "batch4096", "uneven batch of 4096 planted formulas n in [50,20000], R=32, 200 steps, lr 0.1",
        32, 200, 0.1, lambda: uneven_batch()),
    "large_n1e7": Workload(
        "large_n1e7", "n=1e7 m=4.2e7, 5% clauses of 50-200 literals, Zipf 1.2, R=16, 100 steps, lr 0.1",
        16, 100, 0.1, lambda: large_zipf()),
}
