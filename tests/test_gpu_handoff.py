"""GPU parity of the hand-off kernels (Section 3.3, Eq. 8-10, Lemma 1)
against the oracle, with the selections decided on the kernel's FP32
confidences on both sides."""
import numpy as np
import pytest
import torch

from oracle import handoff as H
from paper_2603_28796_amd import inputs as I
from paper_2603_28796_amd.galsat import Problem
from tests.gpu_util import from_oracle, say, to_oracle

pytestmark = pytest.mark.gpu


def _batch():
    fs = [I.planted_ksat(30 + 400 * i, int((30 + 400 * i) * 4.2), 3, seed=500 + i) for i in range(5)]
    fs.append(I.from_clauses([[1, -2], [2]], n=2))
    return I.concat(fs, name="handoff")


@pytest.mark.parametrize("tau", [1.0, 0.5])
def test_candidates_confidence_and_selection(tau):
    say(f"[handoff] tau={tau}")
    cnf = _batch()
    R, N = 12, 9
    prob = Problem(cnf, R)
    rng = np.random.default_rng(41)
    d = from_oracle(rng.normal(size=(R, cnf.n)) * 2.0)
    best = torch.tensor(rng.integers(0, R, size=cnf.F), dtype=torch.int32, device="cuda")
    assign, conf = prob.candidates(d, best, num=N, seed=77, tau=tau)
    torch.cuda.synchronize()
    dsel = to_oracle(d, R)[best.cpu().numpy()[cnf.formula_of_var()], np.arange(cnf.n)]
    # candidate k uses the noise of step k, restart 0
    noise = np.stack([to_oracle(prob.gumbel_noise(77, k), R)[0] for k in range(N)])
    x_ref, c_ref = H.candidates(dsel, noise, tau)
    assert np.array_equal(assign.cpu().numpy(), x_ref)
    np.testing.assert_allclose(conf.cpu().numpy(), c_ref, rtol=1e-6, atol=0)
    # top 0.05 % (at least one) per formula and candidate, on the kernel's FP32 confidences
    off, ids = prob.select_vars(conf, highest=True, frac=0.0005, min_count=1)
    torch.cuda.synchronize()
    c32 = conf.cpu().numpy()
    for f in range(cnf.F):
        v0, v1 = cnf.formula_var_begin[f], cnf.formula_var_begin[f + 1]
        cnt = H.select_count(v1 - v0, 0.0005, 1)
        assert off[f + 1] - off[f] == cnt
        for k in range(N):
            want = v0 + H.select(c32[k, v0:v1], cnt, highest=True)
            assert np.array_equal(ids[k, off[f]:off[f + 1]].cpu().numpy(), want)
    # the d = 7 least confident variables of the selected restart (Lemma 1 branching)
    c0 = prob.confidence(d, best, tau)
    off0, br = prob.select_vars(c0, highest=False, frac=0.0, min_count=7)
    torch.cuda.synchronize()
    np.testing.assert_allclose(c0.cpu().numpy()[0], H.unperturbed_confidence(dsel, tau), rtol=1e-6)
    c0n = c0.cpu().numpy()[0]
    for f in range(cnf.F):
        v0, v1 = cnf.formula_var_begin[f], cnf.formula_var_begin[f + 1]
        cnt = H.select_count(v1 - v0, 0.0, 7)
        want = v0 + H.select(c0n[v0:v1], cnt, highest=False)
        assert np.array_equal(br[0, off0[f]:off0[f + 1]].cpu().numpy(), want)


def test_selection_with_many_ties_and_large_formula():
    say("[handoff] ties")
    cnf = I.planted_ksat(200_000, 800_000, 3, seed=42)
    R = 4
    prob = Problem(cnf, R)
    rng = np.random.default_rng(43)
    conf = torch.tensor(rng.choice([0.5, 0.75, 0.875, 1.0], size=(3, cnf.n)), dtype=torch.float32,
                        device="cuda")
    for highest, frac, mc in ((True, 0.0005, 1), (True, 0.01, 1), (False, 0.0, 7)):
        off, ids = prob.select_vars(conf, highest=highest, frac=frac, min_count=mc)
        torch.cuda.synchronize()
        c = conf.cpu().numpy()
        for k in range(3):
            want = H.select(c[k], int(off[1]), highest=highest)
            assert np.array_equal(ids[k].cpu().numpy(), want)


def test_selection_counts_from_one_to_all():
    """Selections of 1, most and all variables of each formula, on distinct
    confidences (the radix select stops once a digit's bin holds exactly the
    remaining count) and on all-equal ones (every choice falls to the index
    digits)."""
    say("[handoff] counts 1..all")
    cnf = _batch()
    prob = Problem(cnf, 4)
    rng = np.random.default_rng(47)
    distinct = rng.uniform(0.5, 1.0, size=(2, cnf.n)).astype(np.float32)
    equal = np.full((2, cnf.n), 0.75, dtype=np.float32)
    for vals in (distinct, equal):
        conf = torch.tensor(vals, device="cuda")
        for highest, frac, mc in ((True, 0.0, 1), (False, 0.9, 1), (True, 1.0, 1), (False, 1.0, 0)):
            off, ids = prob.select_vars(conf, highest=highest, frac=frac, min_count=mc)
            torch.cuda.synchronize()
            for f in range(cnf.F):
                v0, v1 = cnf.formula_var_begin[f], cnf.formula_var_begin[f + 1]
                cnt = H.select_count(v1 - v0, frac, mc)
                assert off[f + 1] - off[f] == cnt
                for k in range(2):
                    want = v0 + H.select(vals[k, v0:v1], cnt, highest=highest)
                    assert np.array_equal(ids[k, off[f]:off[f + 1]].cpu().numpy(), want), (f, k, frac)
