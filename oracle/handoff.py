"""Hand-off from the GPU stage to the CPU solvers, written from the paper --
TEST INFRASTRUCTURE ONLY (only tests may import it).

Section 3.3.1, Eq. (8): from the selected logits theta_sel, N candidates are
drawn by adding independent Gumbel noise to each variable's logits and
taking the argmax (Eq. 4); each candidate keeps its assignment x^(k) and a
confidence vector c^(k) of the perturbed probabilities.  With two states and
logit difference d, the perturbed probability of the value 1 is
y1 = sigma((d + l) / tau), x = [d + l > 0] (tie -> 0, decided in FP32), and
the confidence of a variable is the probability of the value it took,
max(y1, 1 - y1).  The top |S| most confident variables of a candidate are
fixed as unit clauses (Eq. 9-10; |S| = 0.05 % of n in the appendix).

Section 3.3.2: for UNSAT instances the d least confident variables of
theta_sel (unperturbed probabilities, d = 7 in the appendix) are the
branching variables of Lemma 1.

Readings: |S_f| = min(n_f, max(min_count, ceil(frac * n_f))); ties in
confidence go to the lower variable index; a selection is reported in
increasing variable order.
"""
import math

import numpy as np


def candidates(d_sel, noise, tau=1.0):
    """d_sel [n] (the selected restart's logit differences), noise [N, n]
    (FP32 noise differences).  Returns (assign [N, n] uint8, conf [N, n])."""
    d32 = np.asarray(d_sel, dtype=np.float32)
    l32 = np.asarray(noise, dtype=np.float32)
    x = ((d32[None, :] + l32) > np.float32(0.0)).astype(np.uint8)   # FP32 decision
    z = (d32[None, :].astype(np.float64) + l32.astype(np.float64)) / tau
    y1 = 1.0 / (1.0 + np.exp(-z))
    conf = np.where(x == 1, y1, 1.0 - y1)
    return x, conf


def unperturbed_confidence(d_sel, tau=1.0):
    p = 1.0 / (1.0 + np.exp(-np.asarray(d_sel, dtype=np.float64) / tau))
    return np.maximum(p, 1.0 - p)


def select_count(n_f, frac, min_count):
    return min(n_f, max(min_count, int(math.ceil(frac * n_f))))


def select(conf_row, count, highest=True):
    """Indices of the `count` most (or least) confident entries, ties to the
    lower index, returned in increasing index order."""
    c = np.asarray(conf_row)
    v = np.arange(c.shape[0])
    order = np.lexsort((v, -c)) if highest else np.lexsort((v, c))
    return np.sort(order[:count])
