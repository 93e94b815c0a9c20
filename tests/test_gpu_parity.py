"""GPU parity of libgalsat against the FP64 oracle (through the C ABI).

Every case evaluates the HIP path and the oracle at the same state: loss,
gradient, rounded unsat counts, the hand-off selection, and one update
step checked against the oracle's update of the same state and gradient.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_28796_amd import inputs as I
from paper_2603_28796_amd.galsat import Problem, GalsatLoss, tseitin
from tests.gpu_util import (check_counts, check_grad, check_loss, check_update, parity_at, say,
                            to_oracle, from_oracle)

pytestmark = pytest.mark.gpu


def _x0(n, R, seed, ld=None):
    rng = np.random.default_rng(seed)
    return from_oracle(rng.random((R, n)), ld)


def _edge_formula():
    clauses = [
        [1, -2, 3], [-1], [2, 2, -5], [4, -4], [], [6, 7, 8, 9, 10, 11, 12],
        [-3, -6], [5], [], [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18],
        [13, -13, 14], [-14, -15, -16, -17],
    ]
    # a long clause of 60 distinct literals and a variable (id 99) in no clause
    clauses.append([((i * 7) % 90) + 1 if i % 2 else -(((i * 7) % 90) + 1) for i in range(60)])
    return I.from_clauses(clauses, n=100, name="edge")


def _batch():
    fs = [I.planted_ksat(20 + 13 * i, int((20 + 13 * i) * 4.0), 3, seed=300 + i) for i in range(12)]
    fs.append(I.from_clauses([[]], n=1))                    # one empty clause
    fs.append(I.structured_mixed(n=2000, m=8000, n_comm=10, seed=77))
    fs.append(I.from_clauses([[1, 2], [-1, 2], [1, -2], [-1, -2]], n=2))  # UNSAT
    return I.concat(fs, name="batch")


CASES = {
    "planted300": lambda: I.planted_ksat(300, 1278, 3, seed=11),
    "mixed20k": lambda: I.structured_mixed(n=20000, m=80000, n_comm=20, seed=12),
    "edge": _edge_formula,
    "batch": _batch,
    "long_mix": lambda: I.generate(I.spec(2, k0=3, ka=50, kb=200, p0=0.9, var_kind=1, zipf_s=1.2),
                                   13, [5000], [6000], "long_mix"),
    # the mixed-length instance after width-3 chain normalization (Eq. 6)
    "tseitin3": lambda: tseitin(I.structured_mixed(n=4000, m=16000, n_comm=4, seed=14), 3),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("R", [1, 3, 16, 64, 100])
@pytest.mark.parametrize("partials", ["recompute", "store", "auto"])
def test_parity_cases(case, R, partials):
    say(f"[parity] case={case} R={R} partials={partials}")
    cnf = CASES[case]()
    prob = Problem(cnf, R, partials=partials, lr=0.1)
    x = _x0(cnf.n, R, seed=R)
    parity_at(prob, cnf, x, f"{case}/R={R}/{partials}")
    # one fused step: compare with the oracle's update of the same state
    xr = to_oracle(x, R)
    _, g_gpu = prob.loss_grad(x)
    g_gpu64 = to_oracle(g_gpu, R)
    lo_ref, g_ref, A = oracle.grad(cnf, xr, with_abs=True)
    x1 = x.clone()
    lt, ut = prob.step(x1, 1, trace=True)
    torch.cuda.synchronize()
    check_loss(lt[0], lo_ref, cnf, "step trace")
    check_counts(ut[0], oracle.unsat(cnf, xr), "step trace")
    lr = prob.lr
    check_update(x1, oracle.step_sgd(xr, g_gpu64, lr), xr, R, "update vs GPU gradient")
    # against the oracle's own gradient the step error is bounded by lr * gradient tolerance
    err = np.abs(to_oracle(x1, R) - oracle.step_sgd(xr, g_ref, lr))
    assert np.all(err <= lr * 1e-5 * (np.abs(g_ref) + A) + 2.0 ** -24 + 1e-30)


@pytest.mark.parametrize("lpi", [4, 8, 16, 32, 64])
@pytest.mark.parametrize("rpl", [1, 2, 4])
@pytest.mark.parametrize("stream", [0, 1])
def test_tile_overrides(lpi, rpl, stream):
    say(f"[tiles] lpi={lpi} rpl={rpl} stream={stream}")
    cnf = CASES["edge"]() if lpi % 8 else CASES["batch"]()
    R = 40
    plan = f"lpi={lpi},rpl={rpl},stream={stream}"
    prob = Problem(cnf, R, partials="auto", recompute_max_len=4, plan_override=plan)
    parity_at(prob, cnf, _x0(cnf.n, R, 5), plan)
    # the streaming walk sums every gradient in the same order as the default
    ref = Problem(cnf, R, partials="auto", recompute_max_len=4,
                  plan_override=f"lpi={lpi},rpl={rpl},stream=0")
    x = _x0(cnf.n, R, 6)
    _, g1 = prob.loss_grad(x)
    _, g0 = ref.loss_grad(x)
    torch.cuda.synchronize()
    assert torch.equal(g1, g0)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("R", [3, 16, 40, 64])
@pytest.mark.parametrize("partials", ["auto", "store"])
def test_two_phase_matches_single_pass(case, R, partials):
    """The two-phase gradient (occurrence pass + variable sums) forms the same
    contributions and sums them in the same order as the single pass, so
    gradients, states and counts are bitwise equal; the loss partial sums
    are grouped differently (allclose)."""
    say(f"[two-phase] case={case} R={R} partials={partials}")
    cnf = CASES[case]()
    kw = dict(partials=partials, lr=0.1)
    if partials == "auto":
        kw["recompute_max_len"] = 4
    two = Problem(cnf, R, plan_override="two=1", **kw)
    inf = two.info()
    # same tile for both, so the wave-per-clause pass groups literals alike
    tile = f"lpi={inf['lanes_per_item']},rpl={inf['restarts_per_lane']}"
    one = Problem(cnf, R, plan_override="two=0," + tile, **kw)
    assert two.info()["two_phase"] == 1 and one.info()["two_phase"] == 0
    x = _x0(cnf.n, R, seed=40 + R)
    l2, g2 = two.loss_grad(x)
    l1, g1 = one.loss_grad(x)
    torch.cuda.synchronize()
    assert torch.equal(g2, g1)
    assert torch.allclose(l2, l1, rtol=1e-6, atol=1e-30)
    xa, xb = x.clone(), x.clone()
    la, ua = two.step(xa, 3, trace=True)
    lb, ub = one.step(xb, 3, trace=True)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb)
    assert torch.equal(ua, ub)
    assert torch.allclose(la, lb, rtol=1e-6, atol=1e-30)
    parity_at(two, cnf, xa, f"two-phase {case}/R={R}/{partials}")


@pytest.mark.parametrize("lpi", [4, 8, 16, 32, 64])
@pytest.mark.parametrize("rpl", [1, 2, 4])
def test_two_phase_tiles(lpi, rpl):
    say(f"[two-phase tiles] lpi={lpi} rpl={rpl}")
    cnf = CASES["long_mix"]() if lpi % 8 else CASES["batch"]()
    R = 40
    prob = Problem(cnf, R, partials="auto", recompute_max_len=4,
                   plan_override=f"lpi={lpi},rpl={rpl},two=1")
    parity_at(prob, cnf, _x0(cnf.n, R, 7), f"two-phase lpi={lpi} rpl={rpl}")


@pytest.mark.parametrize("plan", ["dsort=1", "csort=1", "dsort=1,csort=1,two=1",
                                  "dsort=1,two=0,lpi=4,rpl=4"])
def test_sorted_item_orders(plan):
    """Cost-sorted variable items and length-sorted stored clauses change
    only which lanes take which item: gradients, states and counts are
    bitwise those of the index order."""
    say(f"[sorted] {plan}")
    for case in ("long_mix", "batch", "edge"):
        cnf = CASES[case]()
        R = 16
        a = Problem(cnf, R, recompute_max_len=4, plan_override=plan)
        inf = a.info()
        # the same plan in index order: same tile and gradient form
        ref_plan = (f"two={inf['two_phase']},flat={inf['flat']},lpi={inf['lanes_per_item']},"
                    f"rpl={inf['restarts_per_lane']},dsort=0,csort=0")
        b = Problem(cnf, R, recompute_max_len=4, plan_override=ref_plan)
        x = _x0(cnf.n, R, 31)
        la, ga = a.loss_grad(x)
        lb, gb = b.loss_grad(x)
        xa, xb = x.clone(), x.clone()
        ta, ua = a.step(xa, 3, trace=True)
        tb, ub = b.step(xb, 3, trace=True)
        torch.cuda.synchronize()
        assert torch.equal(ga, gb), case
        assert torch.allclose(la, lb, rtol=1e-6, atol=1e-30), case
        assert torch.equal(xa, xb) and torch.equal(ua, ub), case
        parity_at(a, cnf, xa, f"{plan} {case}")


@pytest.mark.parametrize("plan", ["lpi=4,rpl=4", "lpi=4,rpl=1", "lpi=8,rpl=2", "lpi=16,rpl=1",
                                  "lpi=4,rpl=4,two=1", "lpi=8,rpl=4,two=0"])
@pytest.mark.parametrize("partials", ["auto", "store"])
def test_wave_clause_pass(plan, partials):
    """Stored clauses of G..KMAX literals (G = 64 / lanes per item) take the
    wave-per-clause pass: parity with the oracle, and agreement with the
    sweeping clause pass to the gradient tolerance (the products associate
    differently, so not bitwise)."""
    say(f"[wave] {plan} {partials}")
    cnf = CASES["long_mix"]()
    R = 16
    kw = dict(partials=partials, lr=0.1)
    if partials == "auto":
        kw["recompute_max_len"] = 8
    a = Problem(cnf, R, plan_override=plan, **kw)
    b = Problem(cnf, R, plan_override=plan + ",wave=0", **kw)
    x = _x0(cnf.n, R, 51)
    parity_at(a, cnf, x, f"wave {plan}")
    la, ga = a.loss_grad(x)
    lb, gb = b.loss_grad(x)
    torch.cuda.synchronize()
    assert torch.allclose(la, lb, rtol=2e-6, atol=1e-30)
    _, g_ref, A = oracle.grad(cnf, to_oracle(x, R), with_abs=True)
    scale = torch.from_numpy((np.abs(g_ref) + A).T.copy()).to(ga.device)[:, :R]
    assert torch.all((ga[:, :R] - gb[:, :R]).abs().double() <= 2e-5 * scale + 1e-30)
    # a few fused steps stay within the per-step tolerance of each other
    xa = x.clone()
    la, ua = a.step(xa, 2, trace=True)
    torch.cuda.synchronize()
    parity_at(a, cnf, xa, f"wave {plan} after 2 steps")


@pytest.mark.parametrize("case", ["mixed20k", "long_mix", "tseitin3", "edge", "batch"])
@pytest.mark.parametrize("plan", ["two=1", "two=1,short=0", "two=1,wave=0,short=0",
                                  "two=1,lpi=16,rpl=1", "two=0,krec=-1"])
def test_clause_centric_partials(case, plan):
    """Every clause storing its partials (the two-phase default): short
    clauses through the register pass, long ones through the wave-per-clause
    pass, the rest through the sweeping pass; parity with the oracle and
    agreement between the routes to the gradient tolerance."""
    say(f"[clause-centric] {case} {plan}")
    cnf = CASES[case]()
    R = 16
    a = Problem(cnf, R, plan_override=plan)
    if plan.startswith("two=1"):
        assert a.info()["stored_lits"] == cnf.L  # nothing recomputed per occurrence
    x = _x0(cnf.n, R, 61)
    parity_at(a, cnf, x, f"{case} {plan}")
    xa = x.clone()
    a.step(xa, 2)
    torch.cuda.synchronize()
    parity_at(a, cnf, xa, f"{case} {plan} after 2 steps")


@pytest.mark.parametrize("case", ["mixed20k", "planted300", "long_mix", "tseitin3"])
@pytest.mark.parametrize("chunks", [8, 64, 1000])
def test_xcd_contiguous_order(case, chunks):
    """One formula in many small chunks dealt to the XCDs in contiguous runs:
    only which workgroup takes which variables changes, so gradients,
    states and counts are bitwise those of the default order."""
    say(f"[xseq] {case} {chunks}")
    cnf = CASES[case]()
    for R in (16, 100):
        a = Problem(cnf, R, plan_override=f"xseq={chunks}")
        inf = a.info()
        assert inf["xseq_chunks"] == chunks
        tile = (f"lpi={inf['lanes_per_item']},rpl={inf['restarts_per_lane']},"
                f"two={inf['two_phase']},flat={inf['flat']}")
        b = Problem(cnf, R, plan_override=tile + ",xseq=0")
        x = _x0(cnf.n, R, 71)
        la, ga = a.loss_grad(x)
        lb, gb = b.loss_grad(x)
        xa, xb = x.clone(), x.clone()
        ta, ua = a.step(xa, 3, trace=True)
        tb, ub = b.step(xb, 3, trace=True)
        torch.cuda.synchronize()
        assert torch.equal(ga, gb) and torch.equal(xa, xb) and torch.equal(ua, ub)
        assert torch.allclose(la, lb, rtol=1e-6, atol=1e-30)
        parity_at(a, cnf, xa, f"xseq {case} {chunks} R={R}")


def test_two_phase_adam_and_upstream():
    say("[two-phase adam]")
    cnf = CASES["batch"]()
    R = 8
    up = torch.randn(cnf.F, R, device="cuda")
    two = Problem(cnf, R, plan_override="two=1")
    parity_at(two, cnf, _x0(cnf.n, R, 22), "two-phase upstream", upstream=up)
    # the two-phase default stores every clause's partials: the single pass
    # with the same partials sums the same values in the same order
    pa = Problem(cnf, R, optimizer="adam", lr=0.05, plan_override="two=1")
    pb = Problem(cnf, R, optimizer="adam", lr=0.05, plan_override="two=0,krec=0")
    x = _x0(cnf.n, R, 23)
    xa, xb = x.clone(), x.clone()
    sa, sb = pa.new_opt_state(xa), pb.new_opt_state(xb)
    pa.step(xa, 4, opt_state=sa)
    pb.step(xb, 4, opt_state=sb)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb)
    assert torch.equal(sa, sb)


@pytest.mark.parametrize("clauses,n", [([], 3), ([[]], 2), ([], 0), ([[1]], 1), ([[], []], 1),
                                       ([[1, -1], [2, 2, 2]], 2)])
@pytest.mark.parametrize("R", [1, 16, 100])
def test_degenerate_formulas(clauses, n, R):
    """No clauses, only empty clauses, no variables, a tautology and a
    repeated literal, through both gradient plans."""
    say(f"[degenerate] {clauses} n={n} R={R}")
    cnf = I.from_clauses(clauses, n=n)
    for plan in ("two=0", "two=1"):
        prob = Problem(cnf, R, plan_override=plan)
        x = _x0(cnf.n, R, 81)
        parity_at(prob, cnf, x, f"degenerate {plan}")
        xr = to_oracle(x, R)
        _, g_ref, _ = oracle.grad(cnf, xr, with_abs=True)
        x1 = x.clone()
        lt, ut = prob.step(x1, 1, trace=True)
        torch.cuda.synchronize()
        check_counts(ut[0], oracle.unsat(cnf, xr), "degenerate step trace")
        check_update(x1, oracle.step_sgd(xr, g_ref, prob.lr), xr, R, "degenerate step")


@pytest.mark.parametrize("case", ["planted300", "edge", "small_batch"])
@pytest.mark.parametrize("R", [1, 7, 16, 40])
def test_lds_schedule_matches_general(case, R):
    """The persistent LDS schedule forms the same products and sums them in
    the same order as the general single pass with recomputed partials:
    states and counts bitwise, loss allclose; and parity with the oracle."""
    say(f"[lds] {case} R={R}")
    if case == "small_batch":
        cnf = I.concat([I.planted_ksat(30 + 11 * i, 4 * (30 + 11 * i), 3, seed=600 + i)
                        for i in range(9)] + [I.from_clauses([[]], n=1),
                                              I.from_clauses([[1, 2], [-1, 2], [1, -2], [-1, -2]], n=2)])
    else:
        cnf = CASES[case]()
    a = Problem(cnf, R, schedule="lds", lr=0.1)
    info = a.info()
    assert info["schedule"] == "lds"
    # at most 512 workgroups: one restart each; the records fit LDS here
    assert info["lds_restarts_per_group"] == 1 and info["lds_staged"] == 1, info
    b = Problem(cnf, R, schedule="general", partials="recompute", lr=0.1, plan_override="two=0")
    x = _x0(cnf.n, R, 91)
    xa, xb = x.clone(), x.clone()
    la, ua = a.step(xa, 25, trace=True)
    lb, ub = b.step(xb, 25, trace=True)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb)
    assert torch.equal(ua, ub)
    assert torch.allclose(la, lb, rtol=1e-6, atol=1e-30)
    # records read from global memory, and other restart groups: same states
    for pb in ("ldsstage=0", "ldsrg=8,ldsstage=0", "ldsrg=1"):
        c = Problem(cnf, R, schedule="lds", lr=0.1, plan_override=pb)
        xc = x.clone()
        lc, uc = c.step(xc, 25, trace=True)
        torch.cuda.synchronize()
        assert torch.equal(xa, xc), pb
        assert torch.equal(ua, uc), pb
        assert torch.allclose(la, lc, rtol=1e-6, atol=1e-30), pb
    parity_at(a, cnf, xa, f"lds {case} R={R}")
    # one more step from there against the oracle (teacher forced)
    xr = to_oracle(xa, R)
    _, g_ref, _ = oracle.grad(cnf, xr, with_abs=True)
    x1 = xa.clone()
    lt, ut = a.step(x1, 1, trace=True)
    torch.cuda.synchronize()
    check_counts(ut[0], oracle.unsat(cnf, xr), "lds step trace")


@pytest.mark.parametrize("case", ["edge", "batch", "long_mix", "planted300"])
@pytest.mark.parametrize("R", [5, 64])
def test_lds_schedule_steps_against_oracle(case, R):
    """Each step of the persistent LDS schedule against the oracle, teacher
    forced from the GPU's state: the loss and unsat trace entries at x_k
    and the projected-SGD update x_k+1, over three steps. The cases have
    clauses of up to 200 literals (records that name their clause or carry
    extension records), Zipf-heavy variables (split in the general plan,
    not here), an empty clause and formulas of 2 to 5,000 variables."""
    say(f"[lds-oracle] {case} R={R}")
    cnf = CASES[case]()
    prob = Problem(cnf, R, schedule="lds", lr=0.1)
    assert prob.info()["schedule"] == "lds"
    x = _x0(cnf.n, R, 73)
    for k in range(3):
        xr = to_oracle(x, R)
        lo_ref, g_ref, _ = oracle.grad(cnf, xr, with_abs=True)
        x1 = x.clone()
        lt, ut = prob.step(x1, 1, trace=True)
        torch.cuda.synchronize()
        check_loss(lt[0], lo_ref, cnf, f"lds {case} R={R} step {k}")
        check_counts(ut[0], oracle.unsat(cnf, xr), f"lds {case} R={R} step {k}")
        check_update(x1, oracle.step_sgd(xr, g_ref, prob.lr), xr, R, f"lds {case} R={R} step {k}")
        x = x1


def test_lds_schedule_autotune():
    """Under the LDS schedule the autotuner chooses among restart groups and
    record staging, and the chosen plan keeps oracle parity."""
    from paper_2603_28796_amd.galsat import autotune
    say("[lds] autotune")
    cnf = CASES["planted300"]()
    R = 40
    x0 = _x0(cnf.n, R, 5)
    plan, ms = autotune(cnf, R, x0, steps=3, schedule="lds")
    assert plan.startswith("ldsrg=") and ms > 0, plan
    prob = Problem(cnf, R, schedule="lds", lr=0.1, plan_override=plan)
    x = x0.clone()
    xr = to_oracle(x, R)
    _, g_ref, _ = oracle.grad(cnf, xr, with_abs=True)
    prob.step(x, 1)
    torch.cuda.synchronize()
    check_update(x, oracle.step_sgd(xr, g_ref, prob.lr), xr, R, f"lds autotuned {plan}")


@pytest.mark.parametrize("plan", ["lpi=8,rpl=1,tg=8", "lpi=16,rpl=4,tg=8", "lpi=64,rpl=4,tg=2"])
def test_xcd_pinned_tiles(plan):
    """Restart tiles mapped to XCDs by linear block id (xpin=1) run the same
    (chunk, tile) pairs as the plain grid: states, counts and loss bitwise
    equal to the unpinned plan, and parity with the oracle."""
    say(f"[xpin] {plan}")
    cnf = CASES["planted300"]()
    R = 512 if "rpl=4" in plan else 64
    a = Problem(cnf, R, lr=0.1, plan_override=plan + ",two=0,xpin=1")
    b = Problem(cnf, R, lr=0.1, plan_override=plan + ",two=0")
    x = _x0(cnf.n, R, 29)
    xa, xb = x.clone(), x.clone()
    la, ua = a.step(xa, 5, trace=True)
    lb, ub = b.step(xb, 5, trace=True)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb) and torch.equal(ua, ub) and torch.equal(la, lb)
    parity_at(a, cnf, xa, f"xpin {plan}")


def test_lds_schedule_limits():
    from paper_2603_28796_amd.galsat import GalsatError
    say("[lds] limits")
    with pytest.raises(GalsatError):
        Problem(CASES["mixed20k"](), 16, schedule="lds")            # too many variables
    with pytest.raises(GalsatError):
        Problem(CASES["planted300"](), 16, schedule="lds", optimizer="adam")


def test_unaligned_and_padded_state():
    say("[layout] padded and odd row strides")
    cnf = CASES["planted300"]()
    R = 24
    for ld in (24, 25, 32, 37):
        prob = Problem(cnf, R)
        x = _x0(cnf.n, R, 9, ld=ld)
        parity_at(prob, cnf, x, f"ld={ld}")
        pad = x[:, R:].clone()
        prob.step(x, 2)
        torch.cuda.synchronize()
        assert torch.equal(x[:, R:], pad), "padding columns must not be written"


def test_upstream_scaling():
    say("[upstream]")
    cnf = CASES["batch"]()
    R = 8
    prob = Problem(cnf, R)
    up = torch.randn(cnf.F, R, device="cuda")
    parity_at(prob, cnf, _x0(cnf.n, R, 21), "upstream", upstream=up)


def test_init_state_bit_exact():
    say("[init]")
    cnf = CASES["planted300"]()
    for R, ld in ((64, 64), (13, 16)):
        prob = Problem(cnf, R)
        x = prob.init_state(0x6A150001, torch.zeros((cnf.n, ld), device="cuda"))
        torch.cuda.synchronize()
        ref = oracle.init_state(0x6A150001, cnf.n, R)
        assert np.array_equal(to_oracle(x, R), ref)


def test_planted3sat_n200_every_step():
    """Planted 3-SAT n=200, m=852, R=64, 500 projected-SGD steps at lr 0.1:
    loss, gradient and unsat counts per restart at every step, and every
    update, against the oracle evaluated at the GPU's state."""
    say("[trajectory] planted3sat n=200 R=64 500 steps")
    w = I.WORKLOADS["planted3sat_n200"]
    cnf = w.make()
    R = w.restarts
    prob = Problem(cnf, R, lr=w.lr)
    x = prob.init_state(I.SEED_BASE + 1)
    lr = prob.lr
    solved = None
    for k in range(w.steps):
        xr = to_oracle(x, R)
        lo_ref, g_ref, A = oracle.grad(cnf, xr, with_abs=True)
        _, g = prob.loss_grad(x)
        x1 = x.clone()
        lt, ut = prob.step(x1, 1, trace=True)
        torch.cuda.synchronize()
        check_loss(lt[0], lo_ref, cnf, f"step {k}")
        check_counts(ut[0], oracle.unsat(cnf, xr), f"step {k}")
        check_grad(g, g_ref, A, R, f"step {k}")
        check_update(x1, oracle.step_sgd(xr, to_oracle(g, R), lr), xr, R, f"step {k}")
        x = x1
        if solved is None and (ut[0] == 0).any():
            solved = k
    unsat, best, assign = prob.round_check(x)
    torch.cuda.synchronize()
    check_counts(unsat, oracle.unsat(cnf, to_oracle(x, R)), "final")
    say(f"  first restart with 0 unsat at step {solved}; final min unsat {int(unsat.min())}")


def test_multi_step_matches_single_steps():
    """steps=K in one call equals K calls of one step (same kernels, same order)."""
    say("[multistep]")
    cnf = CASES["mixed20k"]()
    R = 32
    prob = Problem(cnf, R)
    xa = _x0(cnf.n, R, 31)
    xb = xa.clone()
    la, ua = prob.step(xa, 5, trace=True)
    lb = []
    for _ in range(5):
        l1, _ = prob.step(xb, 1, trace=True)
        lb.append(l1[0])
    torch.cuda.synchronize()
    assert torch.equal(xa, xb)
    assert torch.equal(la, torch.stack(lb))


def test_determinism_bitwise():
    say("[determinism]")
    cnf = CASES["long_mix"]()
    R = 48
    outs = []
    for _ in range(2):
        prob = Problem(cnf, R, partials="auto")
        x = _x0(cnf.n, R, 41)
        loss, g = prob.loss_grad(x)
        lt, ut = prob.step(x, 3, trace=True)
        torch.cuda.synchronize()
        outs.append((loss.clone(), g.clone(), x.clone(), lt.clone(), ut.clone()))
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_restart_permutation():
    say("[permutation]")
    cnf = CASES["planted300"]()
    R = 64
    prob = Problem(cnf, R)
    x = _x0(cnf.n, R, 51)
    perm = torch.randperm(R, generator=torch.Generator().manual_seed(0)).cuda()
    loss, g = prob.loss_grad(x)
    loss_p, g_p = prob.loss_grad(x[:, perm].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(loss_p, loss[:, perm])
    assert torch.equal(g_p, g[:, perm])


def test_adam_teacher_forced():
    say("[adam]")
    cnf = CASES["mixed20k"]()
    R = 16
    prob = Problem(cnf, R, optimizer="adam", lr=0.5)
    x = _x0(cnf.n, R, 61)
    st = prob.new_opt_state(x)
    b1, b2, eps = float(np.float32(0.9)), float(np.float32(0.999)), float(np.float32(1e-8))
    for t in range(1, 4):
        xr = to_oracle(x, R)
        m0, v0 = to_oracle(st[0], R), to_oracle(st[1], R)
        _, g = prob.loss_grad(x)
        prob.step(x, 1, opt_state=st)
        torch.cuda.synchronize()
        g64 = to_oracle(g, R)
        x_ref, m_ref, v_ref = oracle.step_adam(xr, m0, v0, g64, t, lr=prob.lr, b1=b1, b2=b2, eps=eps)
        # the kernel updates the moments from its FP64 gradient, the oracle from
        # the FP32-rounded one: bound the difference by the magnitudes summed
        # (m can cancel) and carry it through the step
        scale_m = b1 * np.abs(m0) + (1 - b1) * np.abs(g64)
        assert np.all(np.abs(to_oracle(st[0], R) - m_ref) <= 1e-6 * scale_m + 1e-30)
        assert np.all(np.abs(to_oracle(st[1], R) - v_ref) <= 1e-6 * v_ref + 1e-30)
        c1, c2 = 1 - b1 ** t, 1 - b2 ** t
        slack = prob.lr * 1e-6 * scale_m / c1 / (np.sqrt(v_ref / c2) + eps)
        err = np.abs(to_oracle(x, R) - x_ref)
        assert np.all(err <= 1e-5 * np.abs(x_ref - xr) + slack + 2.0 ** -24), f"adam t={t}"
    assert prob.info()["adam_step"] == 3


def test_autograd_function():
    say("[autograd]")
    cnf = CASES["batch"]()
    R = 12
    prob = Problem(cnf, R)
    x = _x0(cnf.n, R, 71).requires_grad_(True)
    loss = GalsatLoss.apply(x, prob)
    wts = torch.rand(cnf.F, R, device="cuda")
    (loss * wts).sum().backward()
    torch.cuda.synchronize()
    xr = to_oracle(x.detach(), R)
    lo_ref, g_ref, A = oracle.grad(cnf, xr, with_abs=True)
    check_loss(loss.detach(), lo_ref, cnf, "autograd forward")
    w = wts.cpu().numpy().astype(np.float64)[cnf.formula_of_var(), :].T
    check_grad(x.grad, g_ref * w, A * np.abs(w), R, "autograd backward")


def test_autograd_padded_and_sliced_state():
    """The autograd backward on a state with padding columns (ld > R) and on
    a column slice of a wider tensor: the gradient has x's strides, its
    first R columns match the oracle and the padding columns are zero."""
    say("[autograd] padded and sliced")
    cnf = CASES["planted300"]()
    R = 12
    prob = Problem(cnf, R)
    xr = np.random.default_rng(72).random((R, cnf.n))
    lo_ref, g_ref, A = oracle.grad(cnf, xr, with_abs=True)
    padded = from_oracle(xr, ld=16).requires_grad_(True)
    wide = from_oracle(xr, ld=20)
    sliced = wide[:, :R].detach().requires_grad_(True)
    for name, x in (("padded", padded), ("sliced", sliced)):
        loss = GalsatLoss.apply(x, prob)
        loss.sum().backward()
        torch.cuda.synchronize()
        check_loss(loss.detach(), lo_ref, cnf, f"{name} forward")
        check_grad(x.grad, g_ref, A, R, f"{name} backward")
        assert x.grad.shape == x.shape
        if x.shape[1] > R:
            assert torch.count_nonzero(x.grad[:, R:]) == 0, "padding columns of grad"


def test_round_check_ties_and_exact_points():
    say("[round]")
    cnf = CASES["mixed20k"]()
    R = 130
    prob = Problem(cnf, R)
    rng = np.random.default_rng(81)
    xr = rng.random((R, cnf.n))
    xr[:, ::5] = 0.5
    xr[:, 1::7] = 0.0
    xr[:, 2::7] = 1.0
    xr[3] = cnf.planted
    x = from_oracle(xr)
    unsat, best, assign = prob.round_check(x)
    torch.cuda.synchronize()
    ref = oracle.unsat(cnf, to_oracle(x, R))
    check_counts(unsat, ref)
    assert int(unsat[0, 3]) == 0
    assert int(best[0]) == int(oracle.best(ref)[0])


def test_graph_replay_matches_eager():
    """galsat_step replayed from a captured graph, with eager work and
    synchronisation between replays, equals eager execution every time."""
    say("[graph]")
    cnf = CASES["mixed20k"]()
    R = 32
    eager = Problem(cnf, R, partials="auto")
    graph = Problem(cnf, R, partials="auto", use_graph=True)
    x0 = _x0(cnf.n, R, 91)
    xe, xg = x0.clone(), x0.clone()
    lt_e = torch.empty((3, cnf.F, R), device="cuda")
    ut_e = torch.empty((3, cnf.F, R), dtype=torch.int32, device="cuda")
    lt_g, ut_g = torch.empty_like(lt_e), torch.empty_like(ut_e)
    for rep in range(4):
        eager.step(xe, 3, loss_trace=lt_e, unsat_trace=ut_e, trace=True)
        graph.step(xg, 3, loss_trace=lt_g, unsat_trace=ut_g, trace=True)
        junk = (xe * 2).sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(xe, xg), f"replay {rep}: state differs"
        assert torch.equal(lt_e, lt_g) and torch.equal(ut_e, ut_g), f"replay {rep}: traces differ"
        del junk


def test_autotune_and_plan_cache(tmp_path, monkeypatch):
    """The autotuner returns one of its candidate plans; with a plan cache a
    later galsat_create without a plan override uses the recorded plan."""
    say("[autotune]")
    from paper_2603_28796_amd.galsat import autotune
    cnf = CASES["long_mix"]()
    R = 16
    cache = tmp_path / "plans.txt"
    monkeypatch.setenv("GALSAT_PLAN_CACHE", str(cache))
    x0 = _x0(cnf.n, R, 99)
    plan, ms = autotune(cnf, R, x0, steps=2)
    assert ms > 0 and ("flat=1" in plan or "two=1" in plan)
    assert plan in cache.read_text()
    prob = Problem(cnf, R)
    info = prob.info()
    want = dict(kv.split("=") for kv in plan.split(","))
    assert info["flat"] == int(want.get("flat", 0))
    assert info["two_phase"] == int(want.get("two", 0))
    parity_at(prob, cnf, x0, f"autotuned {plan}")
    # a wider restart batch tunes tiles and the recompute threshold
    R2 = 128
    plan2, ms2 = autotune(cnf, R2, _x0(cnf.n, R2, 98), steps=2)
    assert ms2 > 0 and "lpi=" in plan2 and "krec=" in plan2
    prob2 = Problem(cnf, R2)
    want2 = dict(kv.split("=") for kv in plan2.split(","))
    assert prob2.info()["lanes_per_item"] == int(want2["lpi"])
    parity_at(prob2, cnf, _x0(cnf.n, R2, 98), f"autotuned {plan2}")


def test_autotune_adam():
    """The autotuner times Adam candidates with their own zeroed moments."""
    say("[autotune] adam")
    from paper_2603_28796_amd.galsat import autotune
    cnf = CASES["planted300"]()
    R = 16
    x0 = _x0(cnf.n, R, 98)
    plan, ms = autotune(cnf, R, x0, steps=2, optimizer="adam", lr=0.5)
    assert ms > 0 and plan
    prob = Problem(cnf, R, optimizer="adam", lr=0.5, plan_override=plan)
    parity_at(prob, cnf, x0, f"autotuned adam {plan}")
