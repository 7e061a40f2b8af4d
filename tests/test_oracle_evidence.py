"""Pins for the oracle's evidence S and beliefs p."""
import itertools
import math

import numpy as np
import pytest

from oracle.evidence import count_posterior, evidence


def _brute_evidence(y, sigma2, K):
    """Enumerate all 2^K bit patterns of the K users at one slot."""
    pats = list(itertools.product([0, 1], repeat=K))
    logw = np.array([-(y - sum(1 - 2 * b for b in p)) ** 2 / (2 * sigma2) for p in pats])
    w = np.exp(logw - logw.max())
    w /= w.sum()
    p0 = sum(wi for wi, p in zip(w, pats) if 0 in p)
    p1 = sum(wi for wi, p in zip(w, pats) if 1 in p)
    return math.log(p0), math.log(p1)


@pytest.mark.parametrize("K", [1, 2, 3, 5, 8])
def test_evidence_matches_enumeration(K):
    rng = np.random.default_rng(K)
    y = rng.normal(0, 1.5, size=16) + rng.integers(-K, K + 1, size=16)
    sigma2 = 0.4
    S, p = evidence(y, sigma2, K)
    for l in range(16):
        s0, s1 = _brute_evidence(float(y[l]), sigma2, K)
        assert abs(S[l, 0] - s0) < 1e-10 * max(1, abs(s0))
        assert abs(S[l, 1] - s1) < 1e-10 * max(1, abs(s1))
    np.testing.assert_allclose(p.sum(axis=1), 1.0, rtol=1e-14)


def test_single_user_is_bpsk_llr():
    y = np.linspace(-3, 3, 25)
    sigma2 = 0.5
    S, _ = evidence(y, sigma2, 1)
    llr = 2 * y / sigma2
    np.testing.assert_allclose(S[:, 0], -np.log1p(np.exp(-llr)), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(S[:, 1], -np.log1p(np.exp(llr)), rtol=1e-12, atol=1e-14)


def test_count_posterior_normalised_and_peaked():
    K = 4
    lp = count_posterior(np.array([4.0, 0.0, -4.0]), 0.01, K)
    np.testing.assert_allclose(np.exp(lp).sum(axis=1), 1.0, rtol=1e-13)
    assert list(np.argmax(lp, axis=1)) == [0, 2, 4]


def test_noiseless_extremes():
    K = 3
    S, p = evidence(np.array([3.0, -3.0, 1.0]), 1e-3, K)
    # y = K: all users sent 0 -> bit 1 absent; y = -K: bit 0 absent; mixed: both present
    assert S[0, 0] > -1e-9 and S[0, 1] < -100
    assert S[1, 1] > -1e-9 and S[1, 0] < -100
    assert S[2, 0] > -1e-9 and S[2, 1] > -1e-9
    np.testing.assert_allclose(p[2], [0.5, 0.5], atol=1e-9)
