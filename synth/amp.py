"""Per-slot observations of the paper's non-binary channel (Appendix,
simulation pipeline and channel model; sensing-matrix construction).

Each slot l of a frame carries K signature indices, one per active user, and
the receiver sees Y_l = A_l U_l + eps with U_l = sqrt(P_sym) times the count
vector of the chosen indices (collisions add up), eps ~ CN(0, sigma2 I) and
A_l the partial-DFT matrix of n_s rows R_l of the Q-point DFT, scaled by
1/sqrt(n_s).  P_sym = B 10^(Eb/10) / L for a B-bit payload over L slots.

Data only: the channel is synthesised here, the detector is not.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np


@dataclass
class AmpSlots:
    rows: np.ndarray        # int32 [S][n_s]: the DFT rows R_l of each slot's A_l
    y: np.ndarray           # float32 [S][n_s][2]: Y_l, real and imaginary parts
    counts: np.ndarray      # int32 [S][Q]: how many users chose signature a in slot l
    p_sym: np.ndarray       # float64 [S]: transmit power of the slot's frame
    ebn0_db: np.ndarray     # float64 [S]


def p_sym_of(ebn0_db: float, payload_bits: int, L: int) -> float:
    """Transmit power per symbol for a per-bit Eb/N0 (dB) at unit noise power."""
    return payload_bits * 10.0 ** (ebn0_db / 10.0) / L


def make_amp_slots(frames: int, L: int, Q: int, n_s: int, K: int, payload_bits: int,
                   ebn0_db: Sequence[float] | float, seed: int, sigma2: float = 1.0,
                   shared_rows: bool = False, idx: Optional[np.ndarray] = None) -> AmpSlots:
    """``frames`` frames of L slots each (S = frames * L slots, frame-major).

    Every frame draws its K users' signature indices independently and
    uniformly per slot, and its Eb/N0 from ``ebn0_db`` in turn.  The DFT rows
    of each slot are n_s distinct indices drawn uniformly (one set for all
    slots when ``shared_rows``).  ``idx`` [S][K], if given, fixes the users'
    symbols instead (codeword symbols of a coded frame)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    levels = np.atleast_1d(np.asarray(ebn0_db, dtype=np.float64))
    S = frames * L
    # n_s distinct rows per slot: the first n_s of a uniform random permutation
    if shared_rows:
        rows = np.repeat(np.sort(np.argsort(rng.random(Q))[:n_s])[None, :], S, axis=0).astype(np.int32)
    else:
        rows = np.sort(np.argsort(rng.random((S, Q)), axis=1)[:, :n_s], axis=1).astype(np.int32)
    if idx is None:
        idx = rng.integers(0, Q, size=(S, K))
    idx = np.asarray(idx, dtype=np.int64)
    counts = np.zeros((S, Q), dtype=np.int32)
    for k in range(K):
        np.add.at(counts, (np.arange(S), idx[:, k]), 1)
    eb = np.repeat(levels[np.arange(frames) % len(levels)], L)
    p_sym = np.array([p_sym_of(e, payload_bits, L) for e in eb])
    # channel: A_l U_l = sqrt(P_sym) sum_k column idx_k of A_l, with
    # A_l[j, a] = exp(-2 pi i R_l[j] a / Q) / sqrt(n_s)
    Y = np.zeros((S, n_s), dtype=np.complex128)
    for k in range(K):
        ph = (rows.astype(np.int64) * idx[:, k:k + 1]) % Q
        Y += np.exp(-2j * np.pi * ph / Q)
    Y *= np.sqrt(p_sym)[:, None] / np.sqrt(n_s)
    Y += (rng.standard_normal((S, n_s)) + 1j * rng.standard_normal((S, n_s))) * np.sqrt(sigma2 / 2.0)
    y = np.stack([Y.real, Y.imag], axis=-1).astype(np.float32)
    return AmpSlots(rows=rows, y=y, counts=counts, p_sym=p_sym, ebn0_db=eb)
