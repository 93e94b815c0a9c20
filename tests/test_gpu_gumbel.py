"""GPU parity of the straight-through Gumbel mode (Section 3.2, Eq. 3-5)
against the oracle at the same logit differences and the same noise."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_28796_amd import inputs as I
from paper_2603_28796_amd.galsat import Problem
from tests.gpu_util import say, to_oracle, from_oracle

pytestmark = pytest.mark.gpu


def test_noise_matches_generator_definition():
    say("[gumbel] noise")
    cnf = I.planted_ksat(500, 2000, 3, seed=31)
    R = 40
    prob = Problem(cnf, R)
    for t in (0, 1, 17):
        l = prob.gumbel_noise(0x5EED, t, ld=48)
        torch.cuda.synchronize()
        ref = oracle.gumbel_noise(0x5EED, t, cnf.n, R)
        # the kernel evaluates the same definition in FP64 and rounds once
        np.testing.assert_allclose(to_oracle(l, R), ref, rtol=2e-7, atol=1e-7)


def _check_d(d_gpu, d_ref, d0, R, lr, what):
    got = to_oracle(d_gpu, R)
    tol = 1e-5 * np.abs(d_ref - d0) + 2e-6 * lr + 2.0 ** -23 * np.abs(d_ref)
    err = np.abs(got - d_ref)
    assert np.all(err <= tol), f"{what}: {np.sum(err > tol)} entries, worst {np.max(err / tol):.3g} x tol"


@pytest.mark.parametrize("optimizer", ["adam", "sgd"])
@pytest.mark.parametrize("case", ["planted", "mixed"])
def test_gumbel_steps_teacher_forced(optimizer, case):
    say(f"[gumbel] {case} {optimizer}")
    cnf = (I.planted_ksat(800, 3408, 3, seed=32) if case == "planted"
           else I.structured_mixed(n=6000, m=24000, n_comm=6, seed=33))
    R = 24
    lr = 0.5 if optimizer == "adam" else 0.05
    prob = Problem(cnf, R, optimizer=optimizer, lr=lr)
    rng = np.random.default_rng(34)
    d = from_oracle(rng.normal(size=(R, cnf.n)))
    st = prob.new_opt_state(d) if optimizer == "adam" else None
    mom = vel = None
    seed, tau = 0xC0FFEE, 1.0
    for t in range(3):
        d0 = to_oracle(d, R)
        noise = prob.gumbel_noise(seed, t)
        if optimizer == "adam":
            mom, vel = to_oracle(st[0], R), to_oracle(st[1], R)
        lt, ut = prob.gumbel_step(d, 1, opt_state=st, seed=seed, step0=t, tau=tau, trace=True)
        torch.cuda.synchronize()
        ref = oracle.gumbel_step(cnf, d0, to_oracle(noise, R), tau=tau, lr=prob.lr,
                                 b1=float(np.float32(0.9)), b2=float(np.float32(0.999)),
                                 eps=float(np.float32(1e-8)), t=t + 1, adam=optimizer == "adam",
                                 mom=mom, vel=vel)
        # loss' at the hard point is an exact integer count on both sides
        assert np.array_equal(lt[0].cpu().numpy().astype(np.float64), ref["loss"])
        assert np.array_equal(ut[0].cpu().numpy(), ref["unsat"])
        _check_d(d, ref["d"], d0, R, prob.lr, f"step {t}")


def test_explicit_noise_equals_drawn_noise():
    say("[gumbel] explicit noise")
    cnf = I.planted_ksat(300, 1278, 3, seed=35)
    R = 16
    a = Problem(cnf, R, optimizer="sgd", lr=0.1)
    b = Problem(cnf, R, optimizer="sgd", lr=0.1)
    d0 = from_oracle(np.random.default_rng(36).normal(size=(R, cnf.n)))
    da, db = d0.clone(), d0.clone()
    noise = torch.stack([a.gumbel_noise(9, t) for t in range(4)])
    a.gumbel_step(da, 4, seed=9, step0=0)
    b.gumbel_step(db, 4, noise=noise)
    torch.cuda.synchronize()
    assert torch.equal(da, db)


def test_paper_setting_descends():
    """Adam lr 0.5, tau 1.0 (the appendix's setting) on a planted 3-SAT
    instance: the best restart's unsatisfied count goes down."""
    say("[gumbel] paper setting")
    cnf = I.planted_ksat(2000, 8520, 3, seed=37)
    R = 64
    prob = Problem(cnf, R, optimizer="adam", lr=0.5)
    d = from_oracle(np.random.default_rng(38).normal(size=(R, cnf.n)) * 0.1)
    st = prob.new_opt_state(d)
    lt, ut = prob.gumbel_step(d, 60, opt_state=st, seed=1, tau=1.0, trace=True)
    torch.cuda.synchronize()
    first, last = int(ut[0].min()), int(ut[-10:].min())
    say(f"  min unsat {first} -> {last}")
    assert last < first
