"""GPU parity of the flat gradient plan: 3-literal clauses recomputed from
pair records, every other clause reduced to a per-clause row of the product
of its nonzero factors and its count of zero factors, each occurrence's
partial then formed by one division in the variable pass.

Every check is against the FP64 oracle at the same state (loss, gradient,
exact unsat counts, the update), plus bitwise agreements that the fixed
summation order guarantees (batched against one formula at a time, repeated
runs)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_28796_amd import inputs as I
from tests.gpu_util import (check_counts, check_grad, check_loss, check_update_oracle, from_oracle,
                            parity_at, say, to_oracle)
from tests.test_gpu_parity import CASES, _x0
from paper_2603_28796_amd.galsat import Problem

pytestmark = pytest.mark.gpu


def _flat(cnf, R, plan="", **kw):
    prob = Problem(cnf, R, plan_override="flat=1" + ("," + plan if plan else ""), **kw)
    assert prob.info()["flat"] == 1
    return prob


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("R", [1, 3, 16, 40, 100])
def test_flat_parity_and_steps(case, R):
    """Loss, gradient, counts and best restart at x0; then three fused steps,
    each step's traced loss and unsat count against the oracle at the state
    the step started from, and the update against the oracle's step."""
    say(f"[flat] case={case} R={R}")
    cnf = CASES[case]()
    prob = _flat(cnf, R, lr=0.1)
    x = _x0(cnf.n, R, seed=100 + R)
    parity_at(prob, cnf, x, f"flat {case} R={R}")
    for k in range(3):
        x0 = to_oracle(x, R)
        lo_ref, g_ref, A = oracle.grad(cnf, x0, with_abs=True)
        lt, ut = prob.step(x, 1, trace=True)
        torch.cuda.synchronize()
        check_loss(lt[0], lo_ref, cnf, f"step {k} trace")
        check_counts(ut[0], oracle.unsat(cnf, x0), f"step {k} trace")
        check_update_oracle(x, x0, g_ref, A, prob.lr, R, f"flat {case} R={R} step {k}")
    parity_at(prob, cnf, x, f"flat {case} R={R} after 3 steps")


@pytest.mark.parametrize("tile", ["lpi=4,rpl=1", "lpi=4,rpl=4", "lpi=8,rpl=2", "lpi=16,rpl=4",
                                  "lpi=64,rpl=1", "lpi=32,rpl=4"])
def test_flat_tiles(tile):
    say(f"[flat tiles] {tile}")
    for case in ("batch", "long_mix", "edge"):
        cnf = CASES[case]()
        R = 48
        prob = _flat(cnf, R, tile)
        parity_at(prob, cnf, _x0(cnf.n, R, 7), f"flat {tile} {case}")


def test_flat_exact_zero_factors():
    """States with many entries exactly 0 or 1 (clamped values): clauses with
    no, one and several exactly-zero factors, including the 60-literal
    clause of the edge case and the long clauses of long_mix."""
    say("[flat zeros]")
    for case in ("edge", "long_mix", "batch", "tseitin3"):
        cnf = CASES[case]()
        R = 32
        prob = _flat(cnf, R)
        rng = np.random.default_rng(17)
        xr = rng.random((R, cnf.n))
        pick = rng.random((R, cnf.n))
        xr[pick < 0.3] = 0.0
        xr[pick > 0.7] = 1.0
        xr[:4] = np.round(xr[:4])  # four restarts entirely at 0/1 points
        parity_at(prob, cnf, from_oracle(xr), f"zeros {case}")


def test_flat_states_outside_unit_interval():
    """loss_grad accepts any finite x: factors below 0 and above 1, where the
    clause products are not monotone (the row pass carries the exponent)."""
    say("[flat outside [0,1]]")
    for case in ("edge", "long_mix", "planted300"):
        cnf = CASES[case]()
        R = 16
        prob = _flat(cnf, R)
        xr = np.random.default_rng(23).uniform(-1.5, 2.5, (R, cnf.n))
        x = from_oracle(xr)
        lo_ref, g_ref, A = oracle.grad(cnf, to_oracle(x, R), with_abs=True)
        loss, g = prob.loss_grad(x)
        torch.cuda.synchronize()
        got = loss.detach().cpu().numpy().astype(np.float64)
        # signed terms: the loss is checked relative to the sum of |U_t|
        # (the oracle's clause values summed in magnitude)
        xo = to_oracle(x, R)
        cl, cp = cnf.clause_lits, cnf.clause_ptr
        absl = np.array([[sum(abs(oracle.clause_U(cl[cp[t]:cp[t + 1]], xo[r])) for t in range(cnf.m))
                          for r in range(R)]])
        assert np.all(np.abs(got - lo_ref) <= 1e-5 * absl + 1e-30), f"loss {case}"
        check_grad(g, g_ref, A, R, f"outside {case}")


def test_flat_adam_and_upstream():
    say("[flat adam / upstream]")
    cnf = CASES["batch"]()
    R = 8
    prob = _flat(cnf, R)
    up = torch.randn(cnf.F, R, device="cuda")
    parity_at(prob, cnf, _x0(cnf.n, R, 21), "flat upstream", upstream=up)
    pa = _flat(cnf, R, optimizer="adam", lr=0.5)
    x = _x0(cnf.n, R, 22)
    st = pa.new_opt_state(x)
    b1, b2, eps = float(np.float32(0.9)), float(np.float32(0.999)), float(np.float32(1e-8))
    for t in range(1, 3):
        xr = to_oracle(x, R)
        m0, v0 = to_oracle(st[0], R), to_oracle(st[1], R)
        _, g = pa.loss_grad(x)
        pa.step(x, 1, opt_state=st)
        torch.cuda.synchronize()
        g64 = to_oracle(g, R)
        x_ref, m_ref, v_ref = oracle.step_adam(xr, m0, v0, g64, t, lr=pa.lr, b1=b1, b2=b2, eps=eps)
        # the kernel's moments come from its FP64 gradient, the oracle's from
        # the FP32-rounded one: bound the difference by the magnitudes summed
        scale_m = b1 * np.abs(m0) + (1 - b1) * np.abs(g64)
        c1, c2 = 1 - b1 ** t, 1 - b2 ** t
        slack = pa.lr * 1e-6 * scale_m / c1 / (np.sqrt(v_ref / c2) + eps)
        err = np.abs(to_oracle(x, R) - x_ref)
        assert np.all(err <= 1e-5 * np.abs(x_ref - xr) + slack + 2.0 ** -24), f"flat adam t={t}"


def test_flat_batched_matches_plain_and_repeats():
    """The same per-variable sums in the same order whether all formulas
    share each launch or run one at a time, and on a second run: states and
    counts bitwise equal."""
    say("[flat plain / determinism]")
    cnf = CASES["batch"]()
    R = 16
    a = _flat(cnf, R)
    b = Problem(cnf, R, schedule="plain", plan_override="flat=1")
    x = _x0(cnf.n, R, 33)
    xa, xb, xc = x.clone(), x.clone(), x.clone()
    la, ua = a.step(xa, 3, trace=True)
    lb, ub = b.step(xb, 3, trace=True)
    lc, uc = a.step(xc, 3, trace=True)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb) and torch.equal(ua, ub)
    assert torch.allclose(la, lb, rtol=1e-6, atol=0)
    assert torch.equal(xa, xc) and torch.equal(ua, uc) and torch.equal(la, lc)


def test_flat_default_for_narrow_batches():
    """AUTO picks the flat plan for at most 64 restarts and keeps the other
    plans when a gradient plan or a recompute threshold is named."""
    cnf = CASES["planted300"]()
    assert Problem(cnf, 32).info()["flat"] == 1
    assert Problem(cnf, 128).info()["flat"] == 0
    assert Problem(cnf, 32, plan_override="two=1").info()["flat"] == 0
    assert Problem(cnf, 32, recompute_max_len=4).info()["flat"] == 0
    assert Problem(cnf, 32, partials="recompute").info()["flat"] == 0
    info = Problem(CASES["long_mix"](), 16).info()
    cnf = CASES["long_mix"]()
    lens = np.diff(cnf.clause_ptr)
    assert info["clause_rows"] == int(((lens != 3) & (lens > 0)).sum())


@pytest.mark.parametrize("case", ["long_mix", "mixed20k", "batch"])
def test_flat_orders_leave_every_sum_unchanged(case):
    """The trip-count order of a chunk's variables (and the record layout
    that follows it), the run order of split-variable segments and record
    prefetching change which wave does what, never the order of any
    variable's sum: the state and the unsat trace after two fused steps are
    bitwise those of the plan with each of them turned off."""
    say(f"[flat orders] {case}")
    cnf = CASES[case]()
    R = 16
    x = _x0(cnf.n, R, 41)
    ref = None
    for plan in ("", "dsort=0", "sord=0", "pf=1", "pf=0", "dsort=0,sord=0"):
        prob = _flat(cnf, R, plan)
        xs = x.clone()
        lt, ut = prob.step(xs, 2, trace=True)
        torch.cuda.synchronize()
        if ref is None:
            ref = (xs, ut, lt)
        else:
            assert torch.equal(xs, ref[0]) and torch.equal(ut, ref[1]), plan
            assert torch.allclose(lt, ref[2], rtol=1e-6, atol=0), plan
        prob.close()
