"""Brute force on tiny codes: the codebook, joint MAP over message sets, and a
genie denoiser that returns exact conditional per-site posteriors.

For K = 2 users sending distinct codewords {c_i, c_j} over the BPSK sum
channel, the likelihood of the unordered pair is
prod_l N(y_l; x_i,l + x_j,l, sigma2) (x = 1 - 2c).  The MAP set maximises it
over all C(M, 2) pairs.  The genie, given a partially revealed 2-row grid,
weighs every ordered pair (c_i, c_j), i != j, consistent with the revealed
tokens and returns log marginals of each site's symbol, which is the ideal
denoiser of the paper's masked refinement loop.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np
from scipy.special import logsumexp

MASK = 2


def codebook(code) -> np.ndarray:
    """All 2^k codewords, uint8 [M][n], message m = integer of the info bits."""
    k = code.k
    info = ((np.arange(2 ** k)[:, None] >> np.arange(k)[None, :]) & 1).astype(np.uint8)
    return code.encode(info)


def pair_loglik(C: np.ndarray, y, sigma2: float) -> np.ndarray:
    """L[i, j] = log prod_l N(y_l; x_i,l + x_j,l, sigma2) up to a constant."""
    x = 1.0 - 2.0 * C.astype(np.float64)
    s = x[:, None, :] + x[None, :, :]
    return -((np.asarray(y, np.float64)[None, None, :] - s) ** 2).sum(axis=2) / (2.0 * float(sigma2))


def map_pair(C: np.ndarray, y, sigma2: float) -> Tuple[Tuple[int, int], float]:
    """MAP unordered pair of distinct messages and its posterior mass."""
    L = pair_loglik(C, y, sigma2)
    M = C.shape[0]
    iu = np.triu_indices(M, k=1)
    vals = L[iu]
    best = int(np.argmax(vals))
    mass = float(np.exp(vals[best] - logsumexp(vals)))
    return (int(iu[0][best]), int(iu[1][best])), mass


def genie_denoiser(C: np.ndarray, y, sigma2: float):
    """den(X, gamma) -> log marginals [2][n][2] given the revealed tokens of X."""
    L = pair_loglik(C, y, sigma2)
    M, n = C.shape
    L = L.copy()
    L[np.arange(M), np.arange(M)] = -np.inf          # distinct messages only

    def den(X, gamma):
        ok0 = np.ones(M, bool)
        ok1 = np.ones(M, bool)
        for l in range(n):
            if X[0, l] != MASK:
                ok0 &= C[:, l] == X[0, l]
            if X[1, l] != MASK:
                ok1 &= C[:, l] == X[1, l]
        Lc = np.where(ok0[:, None] & ok1[None, :], L, -np.inf)
        out = np.full((2, n, 2), -np.inf)
        for a in (0, 1):
            sel = (C == a)                             # [M][n]
            for l in range(n):
                row0 = Lc[sel[:, l], :]
                out[0, l, a] = logsumexp(row0) if row0.size else -np.inf
                col1 = Lc[:, sel[:, l]]
                out[1, l, a] = logsumexp(col1) if col1.size else -np.inf
        tot = logsumexp(out, axis=2, keepdims=True)
        out = out - tot
        return np.maximum(out, -1e3)                 # keep margins finite
    return den
