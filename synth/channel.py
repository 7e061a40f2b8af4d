"""Noisy BPSK superposition of K codewords (binary special case of the
paper's slot-superposition channel: one real dimension per slot, bit 0 sent
as +1 and bit 1 as -1, unit amplitude per user, real AWGN)."""
from __future__ import annotations

from dataclasses import dataclass
from typing import Sequence, Tuple

import numpy as np

from .code import LdpcCode


def ebn0_to_sigma2(ebn0_db: float, rate: float) -> float:
    """Noise variance for unit-energy BPSK at a per-user Eb/N0 (dB) and code rate."""
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


@dataclass
class BinBatch:
    info: np.ndarray        # uint8 [B][K][k]
    codewords: np.ndarray   # uint8 [B][K][n]
    y: np.ndarray           # float32 [B][n]
    sigma2: np.ndarray      # float32 [B]
    ebn0_db: np.ndarray     # float64 [B]


def make_bins(code: LdpcCode, K: int, num_bins: int, ebn0_db: Sequence[float] | float,
              seed: int) -> BinBatch:
    """Draw ``num_bins`` independent bins of K distinct uniform messages each.

    ``ebn0_db`` may be a scalar or a list; a list is cycled over the bins
    (bin b uses ebn0_db[b % len]).  y is rounded once to float32 and sigma2 is
    stored as float32; both sides of any comparison read these same values.
    """
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    ebs = np.atleast_1d(np.asarray(ebn0_db, dtype=np.float64))
    k, n = code.k, code.n
    if K > 2 ** k:
        raise ValueError("more users than codewords")
    info = np.zeros((num_bins, K, k), dtype=np.uint8)
    for b in range(num_bins):
        while True:
            u = rng.integers(0, 2, size=(K, k), dtype=np.uint8)
            if len({row.tobytes() for row in u}) == K:
                break
        info[b] = u
    cw = code.encode(info)
    x = 1.0 - 2.0 * cw.astype(np.float64)              # bit 0 -> +1, bit 1 -> -1
    eb = ebs[np.arange(num_bins) % ebs.size]
    rate = k / n
    sigma2 = np.array([ebn0_to_sigma2(e, rate) for e in eb], dtype=np.float64)
    noise = rng.standard_normal((num_bins, n)) * np.sqrt(sigma2)[:, None]
    y = (x.sum(axis=1) + noise).astype(np.float32)
    return BinBatch(info=info, codewords=cw, y=y, sigma2=sigma2.astype(np.float32), ebn0_db=eb)


@dataclass
class RaggedBin:
    K: int
    n: int
    ebn0_db: float
    y: np.ndarray          # float32 [n]
    sigma2: float          # float32 value
    codewords: np.ndarray  # uint8 [K][n]


def make_ragged_bins(codes: dict, num_bins: int, K_choices: Sequence[int], n_choices: Sequence[int],
                     ebn0_range: Tuple[float, float], seed: int):
    """Bins of uneven size: K uniform over K_choices, n uniform over n_choices
    (codes[n] gives the code), Eb/N0 uniform over ebn0_range.  Each bin's
    payload is drawn from its own child seed, so bin i is the same whatever
    num_bins is."""
    children = np.random.SeedSequence(seed).spawn(num_bins)
    out = []
    for i in range(num_bins):
        g = np.random.Generator(np.random.PCG64(children[i]))
        K = int(g.choice(np.asarray(K_choices)))
        n = int(g.choice(np.asarray(n_choices)))
        eb = float(g.uniform(ebn0_range[0], ebn0_range[1]))
        b = make_bins(codes[n], K, 1, eb, int(g.integers(0, 2**31 - 1)))
        out.append(RaggedBin(K=K, n=n, ebn0_db=eb, y=b.y[0], sigma2=float(b.sigma2[0]), codewords=b.codewords[0]))
    return out
