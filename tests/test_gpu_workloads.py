"""GPU parity at the full sizes of the five workloads, in the launch
configuration the benchmark uses.  The oracle evaluates a sample of restarts
(or of formulas) one by one at exactly the GPU's state; counts of given 0/1
assignments are compared everywhere."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_28796_amd import inputs as I
from paper_2603_28796_amd.galsat import GalsatLoss, Problem
from tests.gpu_util import (check_counts, check_grad, check_loss, check_update_oracle, from_oracle,
                            say, to_oracle)

pytestmark = pytest.mark.gpu

_cache = {}


def workload(key):
    if key not in _cache:
        say(f"[gen] {key}")
        _cache[key] = I.WORKLOADS[key].make()
    return _cache[key]


def sampled_parity(prob, cnf, x, rows, what, grad=True):
    """GPU loss/grad/unsat at x for all restarts; oracle on restarts `rows`."""
    R = prob.R
    loss, g = prob.loss_grad(x) if grad else (prob.loss(x), None)
    unsat, best, _ = prob.round_check(x, want_assign=False)
    torch.cuda.synchronize()
    xs = to_oracle(x, R)[rows]
    lo_ref, g_ref, A = oracle.grad(cnf, xs, with_abs=True)
    check_loss(loss[:, rows], lo_ref, cnf, what)
    if grad:
        check_grad(g, g_ref, A, R, what, rows=rows)
    check_counts(unsat[:, rows], oracle.unsat(cnf, xs), what)
    return loss, unsat


def flip_counts(cnf, assign, vs):
    """Unsat count after flipping each variable of vs in a satisfying
    assignment: the clauses whose only true literal is that variable's."""
    lits = cnf.clause_lits
    val = assign[lits >> 1].astype(bool) ^ (lits & 1).astype(bool)
    ntrue = np.add.reduceat(val.astype(np.int64), cnf.clause_ptr[:-1]) if cnf.m else np.zeros(0)
    ntrue = np.where(np.diff(cnf.clause_ptr) == 0, 0, ntrue)
    out = []
    for v in vs:
        cnt = 0
        for q in range(cnf.var_ptr[v], cnf.var_ptr[v + 1]):
            p = cnf.var_occ[q]
            t = np.searchsorted(cnf.clause_ptr, p, side="right") - 1
            if val[p] and ntrue[t] == 1:
                cnt += 1
        out.append(cnt)
    return out


@pytest.mark.timeout(300)
def test_planted3sat_n1e5_autograd_and_fd():
    """Planted 3-SAT n=1e5, m=426,000, R=1024: autograd gradient at steps
    0, 1, 100 and 999 of the fused SGD trajectory against the oracle on 32
    restarts, and against FP64 central differences (h = 1e-3) on 64 sampled
    variables."""
    w = I.WORKLOADS["planted3sat_n1e5"]
    cnf = workload(w.key)
    R = w.restarts
    prob = Problem(cnf, R, lr=w.lr)
    x = prob.init_state(I.SEED_BASE + 2)
    rows = np.r_[0:16, 1008:1024]
    rng = np.random.default_rng(5)
    deg = np.diff(cnf.var_ptr)
    vars_ = np.unique(np.r_[rng.choice(cnf.n, 60, replace=False), np.argsort(deg)[-2:],
                            np.where(deg == 0)[0][:2]])[:64].astype(np.int32)
    done = 0
    for k in (0, 1, 100, 999):
        if k > done:
            prob.step(x, k - done)
            done = k
        say(f"  step {k}")
        xg = x.clone().requires_grad_(True)
        loss = GalsatLoss.apply(xg, prob)
        loss.sum().backward()
        torch.cuda.synchronize()
        xs = to_oracle(x, R)[rows]
        lo_ref, g_ref, A = oracle.grad(cnf, xs, with_abs=True)
        check_loss(loss.detach()[:, rows], lo_ref, cnf, f"step {k}")
        check_grad(xg.grad, g_ref, A, R, f"step {k}", rows=rows)
        fd = oracle.fd_grad(cnf, xs, vars_, 1e-3)
        gs = to_oracle(xg.grad, R)[rows][:, vars_]
        tol = 1e-5 * (np.abs(fd) + A[:, vars_]) + 1e-9
        assert np.all(np.abs(gs - fd) <= tol), f"FD mismatch at step {k}"
        if k in (0, 999):
            # the fused update x_{k+1} of the benchmark's plan (eight
            # XCD-pinned restart tiles, projected SGD epilogue) on a copy
            assert prob.info()["lanes_per_item"] == 32 and prob.info()["restarts_per_lane"] == 4
            x1 = x.clone()
            prob.step(x1, 1)
            check_update_oracle(x1, xs, g_ref, A, prob.lr, R, f"update at step {k}", rows=rows)
            del x1
    unsat, best, assign = prob.round_check(x)
    torch.cuda.synchronize()
    say(f"  min unsat after 1000 steps: {int(unsat.min())}")


@pytest.mark.timeout(300)
def test_planted3sat_n1e5_exact_counts():
    """Exact pins at full size: the planted assignment has 0 unsatisfied
    clauses; flipping one planted variable unsatisfies exactly the clauses
    in which it is the only true literal."""
    w = I.WORKLOADS["planted3sat_n1e5"]
    cnf = workload(w.key)
    R = 70
    prob = Problem(cnf, R)
    vs = np.random.default_rng(8).choice(cnf.n, R - 1, replace=False)
    xr = np.repeat(cnf.planted[None, :].astype(np.float64), R, axis=0)
    for i, v in enumerate(vs):
        xr[i + 1, v] = 1.0 - xr[i + 1, v]
    unsat, best, assign = prob.round_check(from_oracle(xr))
    torch.cuda.synchronize()
    got = unsat.cpu().numpy()[0]
    assert got[0] == 0
    assert list(got[1:]) == flip_counts(cnf, cnf.planted, vs)
    assert int(best[0]) == 0
    assert np.array_equal(assign.cpu().numpy(), cnf.planted)


@pytest.mark.timeout(300)
def test_mixed_n1e6_recompute():
    """Mixed lengths 2-30, Zipf 1.5 in 1,000 communities, n=1e6, R=256 with
    recomputed partials (nothing stored between passes)."""
    w = I.WORKLOADS["mixed_n1e6"]
    cnf = workload(w.key)
    R = w.restarts
    prob = Problem(cnf, R, lr=w.lr, partials="recompute")
    assert prob.info()["stored_lits"] == 0
    x = prob.init_state(I.SEED_BASE + 3)
    rows = np.r_[0:4, 252:256]
    sampled_parity(prob, cnf, x, rows, "mixed step 0")
    prob.step(x, 5)
    sampled_parity(prob, cnf, x, rows, "mixed step 5")


@pytest.mark.timeout(300)
def test_batch4096_general_vs_plain_and_oracle():
    """4,096 uneven formulas, R=32: the batched general schedule against the
    oracle on sampled formulas, and against the one-formula-at-a-time
    schedule (bitwise for states and counts)."""
    w = I.WORKLOADS["batch4096"]
    cnf = workload(w.key)
    R = w.restarts
    prob = Problem(cnf, R, lr=w.lr, schedule="general")
    x = prob.init_state(I.SEED_BASE + 4)
    loss, g = prob.loss_grad(x)
    unsat, best, _ = prob.round_check(x, want_assign=False)
    x1 = x.clone()
    prob.step(x1, 1)
    torch.cuda.synchronize()
    fs = np.r_[0, 1, np.random.default_rng(3).choice(cnf.F, 14, replace=False), cnf.F - 1]
    for f in fs:
        sub = cnf.sub(int(f))
        v0, v1 = cnf.formula_var_begin[f], cnf.formula_var_begin[f + 1]
        xs = to_oracle(x[v0:v1], R)
        lo_ref, g_ref, A = oracle.grad(sub, xs, with_abs=True)
        check_loss(loss[f:f + 1], lo_ref, sub, f"formula {f}")
        check_grad(g[v0:v1], g_ref, A, R, f"formula {f}")
        check_counts(unsat[f:f + 1], oracle.unsat(sub, xs), f"formula {f}")
        check_update_oracle(x1[v0:v1], xs, g_ref, A, prob.lr, R, f"formula {f} update")
    del x1
    say("  plain schedule")
    plain = Problem(cnf, R, lr=w.lr, schedule="plain")
    xa, xb = x.clone(), x.clone()
    la, ua = prob.step(xa, 2, trace=True)
    lb, ub = plain.step(xb, 2, trace=True)
    torch.cuda.synchronize()
    # same gradient sums in the same order: identical states and counts; the
    # loss partial sums are grouped by chunk, which differs between plans
    assert torch.equal(xa, xb)
    assert torch.equal(ua, ub)
    assert torch.allclose(la, lb, rtol=1e-6, atol=0)


@pytest.mark.timeout(600)
def test_large_n1e7_sampled():
    """n=1e7, m=4.2e7 with 5 % clauses of 50-200 literals and Zipf(1.2)
    popularity, R=16: sampled restarts against the oracle, split hot
    variables included; exact counts of the planted assignment."""
    w = I.WORKLOADS["large_n1e7"]
    cnf = workload(w.key)
    R = w.restarts
    say("  create")
    prob = Problem(cnf, R, lr=w.lr)
    say(f"  plan {prob.info()}")
    x = prob.init_state(I.SEED_BASE + 5)
    rows = np.array([0, 15])
    sampled_parity(prob, cnf, x, rows, "large step 0")
    # the fused update of the benchmark's plan on a copy of the state
    x1 = x.clone()
    prob.step(x1, 1)
    torch.cuda.synchronize()
    xs = to_oracle(x, R)[rows]
    _, g_ref, A = oracle.grad(cnf, xs, with_abs=True)
    check_update_oracle(x1, xs, g_ref, A, prob.lr, R, "large update at step 0", rows=rows)
    del x1
    prob.step(x, 2)
    sampled_parity(prob, cnf, x, np.array([3]), "large step 2")
    xr = np.repeat(cnf.planted[None, :].astype(np.float64), R, axis=0)
    unsat, _, _ = prob.round_check(from_oracle(xr), want_assign=False)
    torch.cuda.synchronize()
    assert int(unsat.max()) == 0
