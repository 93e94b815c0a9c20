"""The allocation-free round check (galsat_round_check_static) against
galsat_round_check through the C ABI: identical unsat counts, best restarts
and best assignments (integers, bit-exact) on two calls in a row on one GPU,
the second on a smaller problem, and a clear refusal above its fixed
scratch size."""
import numpy as np
import pytest
import torch

from paper_2603_28796_amd import inputs as I
from paper_2603_28796_amd.galsat import GalsatError, Problem
from tests.gpu_util import from_oracle, say

pytestmark = pytest.mark.gpu


def _case(cnf, R, seed):
    prob = Problem(cnf, R)
    xr = np.random.default_rng(seed).random((R, cnf.n))
    xr[:, ::7] = 0.5  # ties round to 0
    x = from_oracle(xr, ld=R + 3)
    u_ref, b_ref, a_ref = prob.round_check(x)
    unsat = torch.full((cnf.F, R), -1, dtype=torch.int32, device="cuda")
    best = torch.full((cnf.F,), -1, dtype=torch.int32, device="cuda")
    assign = torch.full((cnf.n,), 7, dtype=torch.uint8, device="cuda")
    prob.round_check_static(x, unsat, best, assign)
    torch.cuda.synchronize()
    assert torch.equal(unsat, u_ref), "unsat counts differ"
    assert torch.equal(best, b_ref), "best restarts differ"
    assert torch.equal(assign, a_ref), "best assignments differ"
    # counts only (no best restart or assignment asked for)
    unsat2 = torch.full((cnf.F, R), -1, dtype=torch.int32, device="cuda")
    prob.round_check_static(x, unsat2)
    torch.cuda.synchronize()
    assert torch.equal(unsat2, u_ref)
    prob.close()


def test_static_round_check_two_calls_then_smaller():
    say("[static] large then small")
    big = I.concat([I.planted_ksat(400 + 37 * i, int((400 + 37 * i) * 4.2), 3, seed=500 + i)
                    for i in range(9)] + [I.structured_mixed(n=20000, m=80000, n_comm=20, seed=12)],
                   name="static_big")
    _case(big, 130, 1)
    small = I.planted_ksat(300, 1278, 3, seed=11)
    _case(small, 17, 2)


def test_static_round_check_refuses_above_its_scratch():
    """70,000 variables x 8,192 restarts: the bit-planes alone (8 bytes per
    variable and 64 restarts, 71.7 MB) exceed the 64 MiB array."""
    say("[static] limit")
    cnf = I.planted_ksat(70000, 298200, 3, seed=13)
    R = 8192
    prob = Problem(cnf, R)
    x = torch.zeros((cnf.n, R), dtype=torch.float32, device="cuda")
    unsat = torch.empty((1, R), dtype=torch.int32, device="cuda")
    with pytest.raises(GalsatError) as err:
        prob.round_check_static(x, unsat)
    assert err.value.status == -4 and "scratch" in str(err.value)
    # the handle stays usable
    u_ref, _, _ = prob.round_check(x, want_assign=False)
    torch.cuda.synchronize()
    assert int(u_ref.min()) >= 0
