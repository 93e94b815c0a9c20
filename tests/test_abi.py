"""The C ABI library loads and exports every symbol include/galsat.h declares;
host-side validation rejects malformed problems before touching the device
(these run without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2603_28796_amd import galsat as G
from paper_2603_28796_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "galsat.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(galsat_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared() == sorted(G.EXPORTS)


def test_kernel_kinds_and_info_layout_match_header():
    text = open(HEADER).read()
    kinds = int(re.search(r"GALSAT_K_KINDS\s*=\s*(\d+)", text).group(1))
    assert kinds == len(G.KERNEL_KINDS)
    body = text[:text.index("} galsat_info;")]
    body = body[body.rindex("typedef struct {") + len("typedef struct {"):]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:
            names += [w.strip() for w in decl.split(None, 1)[1].split(",")]
    assert names == [k for k, _ in G._Info._fields_]


def test_library_exports_every_declared_symbol():
    lib = G.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings_and_defaults():
    lib = G.load_library()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.galsat_status_string(code)
    opt = G._Options()
    lib.galsat_default_options(ctypes.byref(opt))
    assert opt.optimizer == 0 and abs(opt.lr - 0.1) < 1e-7
    assert abs(opt.beta1 - 0.9) < 1e-7 and abs(opt.beta2 - 0.999) < 1e-7
    assert opt.validate == 1 and opt.partials == 0 and opt.schedule == 0


def _create(cnf, R=4, **over):
    lib = G.load_library()
    arrs = {k: np.ascontiguousarray(getattr(cnf, k), dtype=np.int32) for k in
            ("formula_var_begin", "formula_clause_begin", "clause_ptr", "clause_lits", "var_ptr",
             "var_occ")}
    arrs.update({k: np.ascontiguousarray(v, dtype=np.int32) for k, v in over.items()
                 if isinstance(v, np.ndarray)})
    F = over.get("F", cnf.F)
    n = over.get("n", cnf.n)
    m = over.get("m", cnf.m)
    L = over.get("L", cnf.L)
    nul = over.get("null", ())
    prob = G._Problem(F, None if "fvb" in nul else arrs["formula_var_begin"].ctypes.data,
                      None if "fcb" in nul else arrs["formula_clause_begin"].ctypes.data, n, m, L,
                      arrs["clause_ptr"].ctypes.data, arrs["clause_lits"].ctypes.data,
                      arrs["var_ptr"].ctypes.data, arrs["var_occ"].ctypes.data, R, 0)
    h = ctypes.c_void_p()
    st = lib.galsat_create(ctypes.byref(prob), None, None, ctypes.byref(h))
    return st, lib.galsat_last_error(None).decode(), h


@pytest.fixture
def small():
    return I.from_clauses([[1, -2, 3], [-1, 2], [2, 3, -4], [4]], n=4)


def test_rejects_bad_clause_ptr(small):
    cp = small.clause_ptr.copy()
    cp[2] = cp[1] - 1
    st, msg, h = _create(small, clause_ptr=cp)
    assert st == -1 and "clause_ptr" in msg and not h.value


def test_rejects_literal_out_of_range(small):
    cl = small.clause_lits.copy()
    cl[0] = 2 * small.n + 1
    st, msg, _ = _create(small, clause_lits=cl)
    assert st == -1 and "out of range" in msg


def test_rejects_non_transpose(small):
    vo = small.var_occ.copy()
    vo[0], vo[-1] = vo[-1], vo[0]
    st, msg, _ = _create(small, var_occ=vo)
    assert st == -1 and "transpose" in msg


def test_rejects_duplicate_occurrence():
    cnf = I.from_clauses([[1, 2], [1, 3]], n=3)
    vo = cnf.var_occ.copy()
    # variable 0 occurs at positions 0 and 2; list position 0 twice
    assert vo[0] == 0 and vo[1] == 2
    vo[1] = 0
    st, msg, _ = _create(cnf, var_occ=vo)
    assert st == -1 and ("twice" in msg or "transpose" in msg)


def test_rejects_cross_formula_literal():
    a = I.from_clauses([[1, 2]], n=2)
    b = I.from_clauses([[1, -2]], n=2)
    batch = I.concat([a, b])
    cl = batch.clause_lits.copy()
    cl[0] = 2 * 3  # variable 3 belongs to formula 1
    vp, vo = I.transpose(2, batch.formula_var_begin.astype(np.int64),
                         batch.formula_clause_begin.astype(np.int64), batch.clause_ptr, cl)
    st, msg, _ = _create(batch, clause_lits=cl, var_ptr=vp, var_occ=vo)
    assert st == -1 and "another formula" in msg


def test_rejects_missing_formula_ranges():
    batch = I.concat([I.from_clauses([[1]], n=1), I.from_clauses([[-1]], n=1)])
    st, msg, _ = _create(batch, null=("fvb", "fcb"))
    assert st == -1 and "formula" in msg


def test_rejects_bad_sizes(small):
    st, _, _ = _create(small, R=0)
    assert st == -1
    st, _, _ = _create(small, F=0)
    assert st == -1
    st, msg, _ = _create(small, L=small.L - 1)
    assert st == -1


def test_python_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(RuntimeError, match="not found"):
        G.load_library(str(tmp_path / "missing.so"))


@pytest.mark.parametrize("plan", ["", "two=1", "two=0", "two=1,short=0", "two=1,wave=0",
                                  "lpi=4,rpl=4", "lpi=16,rpl=1,two=1", "stream=1", "two=1,krec=4",
                                  "flat=1", "flat=1,lpi=4,rpl=1", "flat=0"])
@pytest.mark.parametrize("partials", [0, 1, 2])
def test_planning_completes_for_every_plan(plan, partials):
    """galsat_create's host planning (records, chunk tables, partial-sum row
    layout) for uneven batches with empty and long clauses: without a GPU it
    must get as far as the first upload (GALSAT_EDEVICE); with one, succeed."""
    fs = [I.planted_ksat(30 + 7 * i, 4 * (30 + 7 * i), 3, seed=500 + i) for i in range(5)]
    fs.append(I.from_clauses([[]], n=1))
    fs.append(I.generate(I.spec(2, k0=3, ka=20, kb=80, p0=0.8, var_kind=1, zipf_s=1.2),
                         21, [400], [500], "long"))
    cnf = I.concat(fs, name="plan")
    lib = G.load_library()
    arrs = {k: np.ascontiguousarray(getattr(cnf, k), dtype=np.int32) for k in
            ("formula_var_begin", "formula_clause_begin", "clause_ptr", "clause_lits", "var_ptr",
             "var_occ")}
    for R in (1, 16, 40):
        prob = G._Problem(cnf.F, arrs["formula_var_begin"].ctypes.data,
                          arrs["formula_clause_begin"].ctypes.data, cnf.n, cnf.m, cnf.L,
                          arrs["clause_ptr"].ctypes.data, arrs["clause_lits"].ctypes.data,
                          arrs["var_ptr"].ctypes.data, arrs["var_occ"].ctypes.data, R, 0)
        opt = G._Options()
        lib.galsat_default_options(ctypes.byref(opt))
        opt.partials = partials
        keep = plan.encode() if plan else None
        opt.plan_override = keep
        h = ctypes.c_void_p()
        st = lib.galsat_create(ctypes.byref(prob), ctypes.byref(opt), None, ctypes.byref(h))
        if st == 0:
            lib.galsat_destroy(h)
        else:
            assert st == -3, (R, lib.galsat_last_error(None))


def test_rejects_restarts_beyond_index_range(small):
    st, msg, h = _create(small, R=65537)
    assert st == -4 and not h.value


@pytest.mark.parametrize("clauses,n", [([], 3), ([[]], 2), ([], 0), ([[1]], 1), ([[], []], 1),
                                       ([[1, -1], [2, 2, 2]], 2)])
def test_planning_degenerate_formulas(clauses, n):
    """No clauses, only empty clauses, no variables, a tautology and a
    repeated literal: planning completes (up to the first upload without a
    GPU)."""
    cnf = I.from_clauses(clauses, n=n)
    for R in (1, 16, 100):
        st, msg, h = _create(cnf, R=R)
        if st == 0:
            G.load_library().galsat_destroy(h)
        else:
            assert st == -3, (R, msg)


def _create_with(cnf, R, plan=None, **fields):
    """galsat_create with option fields set; returns (status, message)."""
    lib = G.load_library()
    arrs = {k: np.ascontiguousarray(getattr(cnf, k), dtype=np.int32) for k in
            ("formula_var_begin", "formula_clause_begin", "clause_ptr", "clause_lits", "var_ptr",
             "var_occ")}
    prob = G._Problem(cnf.F, arrs["formula_var_begin"].ctypes.data,
                      arrs["formula_clause_begin"].ctypes.data, cnf.n, cnf.m, cnf.L,
                      arrs["clause_ptr"].ctypes.data, arrs["clause_lits"].ctypes.data,
                      arrs["var_ptr"].ctypes.data, arrs["var_occ"].ctypes.data, R, 0)
    opt = G._Options()
    lib.galsat_default_options(ctypes.byref(opt))
    for k, v in fields.items():
        setattr(opt, k, v)
    keep = plan.encode() if plan else None
    opt.plan_override = keep
    h = ctypes.c_void_p()
    st = lib.galsat_create(ctypes.byref(prob), ctypes.byref(opt), None, ctypes.byref(h))
    msg = lib.galsat_last_error(None).decode()
    if st == 0:
        lib.galsat_destroy(h)
    return st, msg


@pytest.mark.parametrize("plan", ["", "ldsrg=1", "ldsrg=32", "ldsstage=0", "ldsrg=8,ldsstage=0"])
def test_lds_schedule_planning(plan):
    """The persistent LDS schedule plans uneven batches with empty clauses
    and clauses of up to 80 literals (records that name their clause) for
    every restart group and with the records staged or not: planning gets
    as far as the first upload without a GPU."""
    fs = [I.planted_ksat(30 + 7 * i, 4 * (30 + 7 * i), 3, seed=500 + i) for i in range(5)]
    fs.append(I.from_clauses([[]], n=1))
    fs.append(I.generate(I.spec(2, k0=3, ka=20, kb=80, p0=0.8, var_kind=1, zipf_s=1.2),
                         21, [400], [500], "long"))
    cnf = I.concat(fs, name="plan")
    for R in (1, 16, 40):
        for partials in (0, 2):
            st, msg = _create_with(cnf, R, plan, schedule=G.SCHEDULE["lds"], partials=partials)
            assert st in (0, -3), (R, partials, msg)


def test_lds_schedule_rejections():
    """Adam, stored partials and a formula whose state does not fit LDS
    (12 bytes per variable of one restart within 64 KB: about 5,400
    variables) are refused as unsupported, before any device call."""
    lds = G.SCHEDULE["lds"]
    small = I.planted_ksat(100, 400, 3, seed=7)
    assert _create_with(small, 16, schedule=lds, optimizer=1)[0] == -5
    assert _create_with(small, 16, schedule=lds, partials=G.PARTIALS["store"])[0] == -5
    assert _create_with(I.planted_ksat(5400, 21600, 3, seed=8), 4, schedule=lds)[0] in (0, -3)
    st, msg = _create_with(I.planted_ksat(5500, 22000, 3, seed=9), 4, schedule=lds)
    assert st == -5 and "too large" in msg


def test_lds_schedule_dispatch_limit():
    """A dispatch holds fewer than 2^32 work-items: 200 formulas at 65,536
    restarts still plan (two restarts per workgroup); 5,000 one-variable
    formulas at 65,536 restarts need more than 32 per workgroup and are
    refused."""
    lds = G.SCHEDULE["lds"]
    mid = I.concat([I.planted_ksat(300, 1200, 3, seed=900 + i) for i in range(200)], name="mid")
    assert _create_with(mid, 65536, schedule=lds)[0] in (0, -3)
    tiny = I.concat([I.from_clauses([[1]], n=1)] * 5000, name="tiny")
    st, msg = _create_with(tiny, 65536, schedule=lds)
    assert st == -5 and "too many" in msg
