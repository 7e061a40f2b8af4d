"""FP64 oracle of the protocol-level wrapper (Appendix, protocol-level
scaling by stochastic binning).  Test infrastructure only: the HIP library
never imports or calls it.

K_tot users pick one of zeta preambles uniformly, so the bin loads
(K_1, ..., K_zeta) are multinomial and each K_chi is Binomial(K_tot, 1/zeta),
close to Poisson(kappa), kappa = K_tot / zeta.  A bin with K_chi > K_max is an
overflow: its users are erased.  Frame-level errors count, over all K_tot
users, every user in an overflow bin and every user whose codeword is not
among the rows its bin's decoder returns (a user is recovered when its
transmitted codeword appears as a decoded row: the per-user reading of the
system CER, which equals the per-user probability of error).
"""
from __future__ import annotations

import math
from typing import Dict, Sequence

import numpy as np


def bin_loads(choice: Sequence[int], zeta: int) -> np.ndarray:
    """K_chi = number of users that picked preamble chi, for chi in [zeta]."""
    loads = np.zeros(zeta, dtype=np.int64)
    for c in choice:
        loads[int(c)] += 1
    return loads


def poisson_overflow(kappa: float, K_max: int) -> float:
    """Pr[Poisson(kappa) > K_max] = 1 - sum_{j <= K_max} e^-kappa kappa^j / j!."""
    head = sum(math.exp(-kappa) * kappa ** j / math.factorial(j) for j in range(K_max + 1))
    return max(0.0, 1.0 - head)


def binomial_pmf(K_tot: int, zeta: int, j: int) -> float:
    """Pr[K_chi = j] = C(K_tot, j) (1/zeta)^j (1 - 1/zeta)^(K_tot - j)."""
    p = 1.0 / zeta
    return math.comb(K_tot, j) * p ** j * (1 - p) ** (K_tot - j)


def binomial_overflow(K_tot: int, zeta: int, K_max: int) -> float:
    """Pr[K_chi > K_max] for one bin, K_chi ~ Binomial(K_tot, 1/zeta), as one
    minus the head j <= K_max (the head's binomial coefficients stay small)."""
    return max(0.0, 1.0 - sum(binomial_pmf(K_tot, zeta, j) for j in range(min(K_max, K_tot) + 1)))


def expected_overflow_users(K_tot: int, zeta: int, K_max: int) -> float:
    """E[users in overflow bins] = zeta E[K_chi 1{K_chi > K_max}]
    = K_tot - zeta sum_{j <= K_max} j Pr[K_chi = j]; divided by K_tot it is the
    floor the frame CER cannot go below."""
    head = sum(j * binomial_pmf(K_tot, zeta, j) for j in range(min(K_max, K_tot) + 1))
    return max(0.0, K_tot - zeta * head)


def frame_user_errors(loads: np.ndarray, K_max: int, sent: Dict[int, np.ndarray],
                      decoded: Dict[int, np.ndarray]) -> int:
    """Users of one frame that are not recovered.  sent[chi] and decoded[chi]
    are the bin's transmitted and decoded grids [K_chi][n] for every bin with
    1 <= K_chi <= K_max; overflow bins lose all their users."""
    err = 0
    for chi, K in enumerate(np.asarray(loads)):
        K = int(K)
        if K == 0:
            continue
        if K > K_max:
            err += K
            continue
        got = {row.tobytes() for row in np.asarray(decoded[chi], dtype=np.uint8)}
        for row in np.asarray(sent[chi], dtype=np.uint8):
            if row.tobytes() not in got:
                err += 1
    return err
