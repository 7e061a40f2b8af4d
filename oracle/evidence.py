"""Evidence interface S (Appendix, per-slot channel model and evidence).

The paper defines S[l, a] = log Pr(U_a != 0 | Y_l): the log-posterior that
at least one active user sent symbol a in slot l, and feeds the decoder the
per-slot normalisation p[l, a] proportional to exp(S[l, a]).

Binary BPSK case: each user sends x = +1 (bit 0) or -1 (bit 1) and
y = sum_k x_k + N(0, sigma2).  With m = number of users sending bit 1, the
noiseless sum is K - 2m and, for independent uniform bits, the prior on m is
Binomial(K, 1/2).  So the exact posterior over m is

    P(m | y) proportional to C(K, m) exp(-(y - (K - 2m))^2 / (2 sigma2)),

bit 0 is present iff m < K and bit 1 iff m > 0.  Everything is done with
log-sum-exp so that no probability is formed by subtraction from one.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import logsumexp


def count_posterior(y, sigma2: float, K: int) -> np.ndarray:
    """log P(m | y_l) for m = 0..K; shape [n][K+1]."""
    y = np.asarray(y, dtype=np.float64)
    m = np.arange(K + 1, dtype=np.float64)
    log_prior = np.array([math.lgamma(K + 1) - math.lgamma(j + 1) - math.lgamma(K - j + 1)
                          for j in range(K + 1)])
    mean = K - 2.0 * m
    logw = log_prior[None, :] - (y[:, None] - mean[None, :]) ** 2 / (2.0 * float(sigma2))
    return logw - logsumexp(logw, axis=1, keepdims=True)


def evidence(y, sigma2: float, K: int):
    """Return (S, p), each float64 [n][2].

    S[:, 0] = log Pr(m < K | y)   (some user sent bit 0)
    S[:, 1] = log Pr(m > 0 | y)   (some user sent bit 1)
    p       = softmax over a of S (the decoder's per-slot belief)
    """
    lp = count_posterior(y, sigma2, K)
    S0 = logsumexp(lp[:, :K], axis=1)
    S1 = logsumexp(lp[:, 1:], axis=1)
    S = np.stack([S0, S1], axis=1)
    p = np.exp(S - logsumexp(S, axis=1, keepdims=True))
    return S, p
