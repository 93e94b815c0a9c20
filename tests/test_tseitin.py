"""Fixed-width clause normalization (Section 3.2, Eq. 6-7): the oracle is
pinned by the appendix example and by brute-force equisatisfiability; the
library's host implementation must produce exactly the oracle's formula."""
import itertools

import numpy as np
import pytest

from oracle import tseitin as T
from paper_2603_28796_amd import galsat as G
from paper_2603_28796_amd import inputs as I


def _sat(clauses, assign):
    return all(any((assign[abs(l) - 1] == 1) if l > 0 else (assign[abs(l) - 1] == 0) for l in c)
               for c in clauses)


def test_appendix_example():
    """phi = (x1 v ~x2 v x3 v x4) ^ (~x1 v x3): the chain of Eq. (6) gives
    (x1 v ~x2 v z1) ^ (~z1 v x3 v x4) and the short clause is padded to
    (~x1 v x3 v x3)."""
    n2, out = T.normalize([[1, -2, 3, 4], [-1, 3]], 4)
    assert n2 == 5
    assert out == [[1, -2, 5], [-5, 3, 4], [-1, 3, 3]]


def test_chain_shape_eq6():
    n2, out = T.normalize([[1, 2, 3, 4, 5, 6]], 6)
    assert n2 == 6 + 3                                  # u - 3 auxiliaries
    assert out == [[1, 2, 7], [-7, 3, 8], [-8, 4, 9], [-9, 5, 6]]   # u - 2 clauses


@pytest.mark.parametrize("width", [3, 4, 5])
@pytest.mark.parametrize("seed", range(6))
def test_equisatisfiable_brute_force(width, seed):
    """Eq. (7), checked exhaustively: every satisfying assignment of the
    original extends to one of the normalized formula, and every satisfying
    assignment of the normalized formula restricts to one of the original."""
    rng = np.random.default_rng(seed)
    n = 6
    clauses = []
    for _ in range(int(rng.integers(2, 6))):
        k = int(rng.integers(1, 7))
        vs = rng.choice(n, size=k, replace=False)
        clauses.append([int(v + 1) * (1 if rng.random() < 0.5 else -1) for v in vs])
    n2, out = T.normalize(clauses, n, width)
    assert all(len(c) == width for c in out)
    orig_sat = {bits for bits in itertools.product([0, 1], repeat=n) if _sat(clauses, bits)}
    proj = set()
    for bits in itertools.product([0, 1], repeat=n2):
        if _sat(out, bits):
            proj.add(bits[:n])
    assert proj == orig_sat


def test_empty_clause_kept():
    n2, out = T.normalize([[1, 2], []], 2)
    assert out == [[1, 2, 2], []]


@pytest.mark.parametrize("width", [3, 4, 7])
def test_library_matches_oracle(width):
    cnf = I.generate(I.spec(1, k0=3, kmax=30, geom_p=1.0 / 3.0), 21, [300], [900], "mixed")
    clauses = [[(c >> 1) + 1 if not c & 1 else -((c >> 1) + 1) for c in cl] for cl in cnf.clauses()]
    clauses += [[], [5], [-7, 7]]
    src = I.from_clauses(clauses, n=cnf.n)
    got = G.tseitin(src, width)
    n2, want = T.normalize(clauses, cnf.n, width)
    assert got.n == n2
    got_dimacs = [[(c >> 1) + 1 if not c & 1 else -((c >> 1) + 1) for c in cl] for cl in got.clauses()]
    assert got_dimacs == want


def test_library_rejects_bad_input():
    src = I.from_clauses([[1, 2, 3, 4]], n=4)
    with pytest.raises(G.GalsatError):
        G.tseitin(src, 2)
