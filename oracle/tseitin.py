"""Fixed-width clause normalization written from the paper -- TEST
INFRASTRUCTURE ONLY (only tests may import it).

Section 3.2, "Clause Normalization for Vectorization", Eq. (6): a clause
(l1 v ... v lu) with u > 3 is replaced by the chain
    (l1 v l2 v f1) ^ (~f1 v l3 v f2) ^ ... ^ (~f_{u-3} v l_{u-1} v lu)
with fresh auxiliary variables f1 .. f_{u-3}; Eq. (7) states that the chain
is satisfiable exactly when the clause is.  Clauses shorter than the width
are padded by duplicating literals; the appendix example pads
(~x1 v x3) to (~x1 v x3 v x3), i.e. repeats the last literal.

The general width w >= 3 keeps the same shape: the first link carries w-1
literals and f1, each middle link ~f_i, w-2 literals and f_{i+1}, the last
link ~f_last and the rest, padded like a short clause.  Literals are DIMACS
integers here (+v / -v, 1-based); auxiliaries are numbered n+1, n+2, ... in
order of creation.
"""


def normalize(clauses, n, width=3):
    """Returns (n_out, clauses_out)."""
    out = []
    next_var = n + 1
    for c in clauses:
        u = len(c)
        if u == 0:
            out.append([])
            continue
        if u <= width:
            out.append(list(c) + [c[-1]] * (width - u))
            continue
        # first link
        f = next_var
        next_var += 1
        out.append(list(c[:width - 1]) + [f])
        i = width - 1
        prev = f
        # middle links while more than width-1 literals remain
        while u - i > width - 1:
            f = next_var
            next_var += 1
            out.append([-prev] + list(c[i:i + width - 2]) + [f])
            i += width - 2
            prev = f
        last = [-prev] + list(c[i:])
        out.append(last + [c[-1]] * (width - len(last)))
    return next_var - 1, out
