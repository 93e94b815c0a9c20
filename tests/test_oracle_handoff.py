"""Pins of the hand-off oracle (Section 3.3, Eq. 8-10 and Lemma 1): the
candidate assignment is torch's argmax of the perturbed two-logit softmax
and the confidence its probability; selections agree with a full stable
sort."""
import numpy as np
import pytest
import torch

from oracle import handoff as H


def test_candidates_match_two_logit_softmax():
    rng = np.random.default_rng(3)
    d = rng.normal(size=50).astype(np.float32)
    noise = rng.logistic(size=(7, 50)).astype(np.float32)
    noise[0, :5] = -d[:5]                            # exact ties -> value 0
    x, conf = H.candidates(d, noise, tau=0.7)
    theta = torch.zeros((7, 50, 2), dtype=torch.float64)
    theta[..., 1] = torch.from_numpy(d.astype(np.float64))[None, :]
    g = torch.zeros_like(theta)
    g[..., 1] = torch.from_numpy(noise.astype(np.float64))
    y = torch.softmax((theta + g) / 0.7, dim=-1)
    idx = y.argmax(-1)
    assert np.array_equal(x, idx.numpy().astype(np.uint8))
    np.testing.assert_allclose(conf, y.gather(-1, idx[..., None])[..., 0].numpy(), rtol=1e-12)
    assert np.all(x[0, :5] == 0)


def test_select_matches_sorting():
    rng = np.random.default_rng(4)
    c = rng.choice([0.5, 0.6, 0.75, 0.9, 1.0], size=200)   # many ties
    for count in (1, 7, 37, 200):
        top = H.select(c, count, highest=True)
        # brute force: the set of the first `count` of (-c, index) order
        want = sorted(range(200), key=lambda i: (-c[i], i))[:count]
        assert top.tolist() == sorted(want)
        low = H.select(c, count, highest=False)
        want = sorted(range(200), key=lambda i: (c[i], i))[:count]
        assert low.tolist() == sorted(want)


def test_counts():
    assert H.select_count(100000, 0.0005, 1) == 50
    assert H.select_count(50, 0.0005, 1) == 1
    assert H.select_count(5, 0.0, 7) == 5
    assert H.select_count(20000, 0.0, 7) == 7


def pin_unperturbed_confidence(conf_fn):
    """Section 3.3.2: the confidence of a variable in the selected restart is
    the unperturbed softmax probability of the value it takes.  Checked
    against torch's softmax over the two logits (0, d) at temperature tau,
    taking the probability of the argmax, plus the special values: exactly
    1/2 at d = 0, symmetric under d -> -d, and tending to 1 for large |d|."""
    rng = np.random.default_rng(11)
    d = np.concatenate([rng.normal(scale=3.0, size=200), [0.0, 1e-9, -1e-9, 40.0, -40.0]])
    for tau in (1.0, 0.5, 2.0):
        got = conf_fn(d, tau=tau)
        logits = torch.zeros((d.shape[0], 2), dtype=torch.float64)
        logits[:, 1] = torch.from_numpy(d)
        y = torch.softmax(logits / tau, dim=-1)
        want = y.max(dim=-1).values.numpy()
        np.testing.assert_allclose(got, want, rtol=1e-13, atol=0)
        np.testing.assert_allclose(conf_fn(-d, tau=tau), got, rtol=1e-13, atol=0)
        assert got[200] == 0.5
    # at d = tau * log(3) the two-state softmax is (1/4, 3/4) for any tau
    for tau in (1.0, 0.5):
        assert conf_fn(np.array([tau * np.log(3.0)]), tau=tau)[0] == pytest.approx(0.75, abs=1e-15)


def test_unperturbed_confidence_matches_softmax():
    pin_unperturbed_confidence(H.unperturbed_confidence)


def pin_candidates(cand_fn):
    rng = np.random.default_rng(13)
    d = rng.normal(size=40).astype(np.float32)
    noise = rng.logistic(size=(5, 40)).astype(np.float32)
    noise[0, :4] = -d[:4]
    for tau in (1.0, 0.5):
        x, conf = cand_fn(d, noise, tau=tau)
        logits = torch.zeros((5, 40, 2), dtype=torch.float64)
        logits[..., 1] = torch.from_numpy(d.astype(np.float64))[None, :] + \
            torch.from_numpy(noise.astype(np.float64))
        y = torch.softmax(logits / tau, dim=-1)
        idx = y.argmax(-1)
        assert np.array_equal(x, idx.numpy().astype(np.uint8))
        np.testing.assert_allclose(conf, y.gather(-1, idx[..., None])[..., 0].numpy(), rtol=1e-12)


def pin_select(select_fn):
    c = np.array([0.9, 0.5, 0.9, 0.7, 0.5, 1.0, 0.7])
    assert select_fn(c, 3, highest=True).tolist() == [0, 2, 5]
    assert select_fn(c, 3, highest=False).tolist() == [1, 3, 4]


# Plausible mistakes planted in a copy of handoff.py: each must make one of
# the pins above fail.
HANDOFF_MUTANTS = {
    "confidence_no_temperature": ("np.asarray(d_sel, dtype=np.float64) / tau))",
                                  "np.asarray(d_sel, dtype=np.float64)))"),
    "confidence_min_for_max": ("return np.maximum(p, 1.0 - p)", "return np.minimum(p, 1.0 - p)"),
    "confidence_of_value_one": ("return np.maximum(p, 1.0 - p)", "return p"),
    "candidates_tie_to_one": ("(d32[None, :] + l32) > np.float32(0.0)",
                              "(d32[None, :] + l32) >= np.float32(0.0)"),
    "candidates_no_temperature": ("l32.astype(np.float64)) / tau", "l32.astype(np.float64))"),
    "select_ties_to_higher": ("order = np.lexsort((v, -c)) if highest else np.lexsort((v, c))",
                              "order = np.lexsort((-v, -c)) if highest else np.lexsort((-v, c))"),
}


@pytest.mark.parametrize("name", sorted(HANDOFF_MUTANTS))
def test_handoff_mutant_is_caught(name):
    import types

    old, new = HANDOFF_MUTANTS[name]
    src = open(H.__file__).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mod = types.ModuleType(f"handoff_mutant_{name}")
    exec(compile(src.replace(old, new), mod.__name__, "exec"), mod.__dict__)
    failures = 0
    for pin in (lambda: pin_unperturbed_confidence(mod.unperturbed_confidence),
                lambda: pin_candidates(mod.candidates),
                lambda: pin_select(mod.select)):
        try:
            pin()
        except AssertionError:
            failures += 1
    assert failures >= 1, f"no pin detects the hand-off mutant {name}"


def test_handoff_pins_pass_on_the_oracle():
    pin_candidates(H.candidates)
    pin_select(H.select)
