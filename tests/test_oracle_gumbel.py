"""Pins of the oracle's straight-through Gumbel mode (Section 3.2, Eq. 3-5;
appendix: Adam, lr 0.5, tau 1.0): the noise generator against the logistic
law of a difference of two Gumbel(0,1) variables, and one training step
against torch autograd on the paper's two-logit formulation (softmax with
Gumbel noise, hard argmax forward, soft backward) with torch.optim."""
import numpy as np
import pytest
import torch
from scipy import stats

import oracle
from paper_2603_28796_amd import inputs as I


def test_noise_is_logistic():
    l = oracle.gumbel_noise(0x6A15ABCD, 3, 1000, 64).ravel()
    # g1 - g0 of independent Gumbel(0,1) variables is Logistic(0,1)
    assert stats.kstest(l, stats.logistic.cdf).pvalue > 1e-3
    assert abs(l.mean()) < 0.03
    assert abs(l.var() - np.pi ** 2 / 3) < 0.1
    l2 = oracle.gumbel_noise(0x6A15ABCD, 4, 1000, 64).ravel()
    assert abs(np.corrcoef(l, l2)[0, 1]) < 0.02          # steps are independent
    assert not np.array_equal(l, l2)


def _torch_two_logit_step(clauses, d, l, tau, lr, adam, steps_state=None):
    R, n = d.shape
    theta = torch.zeros((R, n, 2), dtype=torch.float64)
    theta[..., 1] = torch.from_numpy(d)
    theta.requires_grad_(True)
    g = torch.zeros((R, n, 2), dtype=torch.float64)
    g[..., 1] = torch.from_numpy(l.astype(np.float64))
    y = torch.softmax((theta + g) / tau, dim=-1)                 # Eq. (3)
    hard = torch.nn.functional.one_hot(y.argmax(-1), 2).double()  # Eq. (4), first max on ties
    x1 = (hard - y.detach() + y)[..., 1]                          # straight-through
    total = x1.new_zeros(R)
    for c in clauses:                                             # Eq. (2)
        u = x1.new_ones(R)
        for lit in c:
            s = x1[:, abs(lit) - 1] if lit > 0 else 1.0 - x1[:, abs(lit) - 1]
            u = u * (1.0 - s)
        total = total + u
    loss_paper = -(len(clauses) - total)                          # Eq. (5): -sum C
    loss_paper.sum().backward()
    opt = torch.optim.Adam([theta], lr=lr) if adam else torch.optim.SGD([theta], lr=lr)
    opt.step()
    with torch.no_grad():
        d_new = (theta[..., 1] - theta[..., 0]).numpy()
    return d_new, total.detach().numpy(), hard[..., 1].detach().numpy()


@pytest.mark.parametrize("adam", [True, False])
@pytest.mark.parametrize("tau", [1.0, 0.5])
def test_step_matches_two_logit_autograd(adam, tau):
    rng = np.random.default_rng(9)
    n, R = 12, 6
    clauses = []
    for _ in range(40):
        k = int(rng.integers(1, 5))
        vs = rng.choice(n, size=k, replace=False)
        clauses.append([int(v + 1) * (1 if rng.random() < 0.5 else -1) for v in vs])
    cnf = I.from_clauses(clauses, n=n)
    d = rng.normal(size=(R, n)).astype(np.float32).astype(np.float64)
    l = oracle.gumbel_noise(77, 1, n, R).astype(np.float32)
    got = oracle.gumbel_step(cnf, d, l, tau=tau, lr=0.5, t=1, adam=adam)
    d_ref, total_ref, xh_ref = _torch_two_logit_step(clauses, d, l, tau, 0.5, adam)
    np.testing.assert_array_equal(got["xh"], xh_ref)
    np.testing.assert_allclose(got["loss"][0], total_ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(got["d"], d_ref, rtol=1e-12, atol=1e-12)
    # at the hard point the loss is the exact unsatisfied-clause count
    assert np.array_equal(got["loss"][0], got["unsat"][0].astype(np.float64))


def test_adam_steps_keep_matching():
    """Several Adam steps: the single-difference state tracks the two-logit
    optimizer exactly (theta0's moments are the negatives of theta1's)."""
    rng = np.random.default_rng(10)
    n, R = 10, 4
    clauses = [[int(v + 1) * (1 if rng.random() < 0.5 else -1)
                for v in rng.choice(n, size=3, replace=False)] for _ in range(35)]
    cnf = I.from_clauses(clauses, n=n)
    d0 = rng.normal(size=(R, n)).astype(np.float32).astype(np.float64)
    theta = torch.zeros((R, n, 2), dtype=torch.float64)
    theta[..., 1] = torch.from_numpy(d0)
    theta.requires_grad_(True)
    opt = torch.optim.Adam([theta], lr=0.5)
    d, mom, vel = d0.copy(), None, None
    for t in range(1, 5):
        l = oracle.gumbel_noise(5, t, n, R).astype(np.float32)
        got = oracle.gumbel_step(cnf, d.astype(np.float32).astype(np.float64), l, t=t, mom=mom,
                                 vel=vel)
        # torch side on the same (FP32-representable) state
        opt.zero_grad()
        g = torch.zeros((R, n, 2), dtype=torch.float64)
        g[..., 1] = torch.from_numpy(l.astype(np.float64))
        y = torch.softmax(theta + g, dim=-1)
        x1 = (torch.nn.functional.one_hot(y.argmax(-1), 2).double() - y.detach() + y)[..., 1]
        total = x1.new_zeros(R)
        for c in clauses:
            u = x1.new_ones(R)
            for lit in c:
                s = x1[:, abs(lit) - 1] if lit > 0 else 1.0 - x1[:, abs(lit) - 1]
                u = u * (1.0 - s)
            total = total + u
        total.sum().backward()
        opt.step()
        with torch.no_grad():
            d_ref = (theta[..., 1] - theta[..., 0]).numpy().copy()
            theta[..., 1] = torch.from_numpy(d_ref.astype(np.float32).astype(np.float64))
            theta[..., 0] = 0.0
        np.testing.assert_allclose(got["d"], d_ref, rtol=1e-10, atol=1e-10)
        d, mom, vel = got["d"], got["mom"], got["vel"]


def test_tie_goes_to_state_zero():
    """d + l exactly 0: the argmax of Eq. (4) picks the first state (value 0),
    as torch.argmax does."""
    clauses = [[1, 2], [-1, 3], [2, -3]]
    cnf = I.from_clauses(clauses, n=3)
    l = np.array([[0.25, -1.5, 3.0], [0.0, 0.0, 0.0]], dtype=np.float32)
    d = -l.astype(np.float64)
    got = oracle.gumbel_step(cnf, d, l, adam=False)
    assert np.array_equal(got["xh"], np.zeros_like(d))
    d_ref, total_ref, xh_ref = _torch_two_logit_step(clauses, d, l, 1.0, 0.5, False)
    np.testing.assert_array_equal(xh_ref, got["xh"])
    np.testing.assert_allclose(got["d"], d_ref, rtol=1e-12, atol=1e-12)
