"""Pins of the hand-off oracle (Section 3.3, Eq. 8-10 and Lemma 1): the
candidate assignment is torch's argmax of the perturbed two-logit softmax
and the confidence its probability; selections agree with a full stable
sort."""
import numpy as np
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
