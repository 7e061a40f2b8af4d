"""Frames of the two-step random-access protocol that wraps the decoder
(Appendix, protocol-level scaling by stochastic binning).

Every one of K_tot active users picks one of zeta preambles uniformly; the
users that picked preamble chi form payload bin chi, with load K_chi.  A bin
with 1 <= K_chi <= K_max becomes one decoding instance (a superposition of
K_chi codewords of distinct messages); a bin with K_chi > K_max is an
overflow and gets no payload (the receiver erases it); an empty bin is
skipped.

Data only: the loads and the channel are synthesised here; the overflow
rule and the frame-level error count are the protocol's, on the host.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

from .channel import RaggedBin, make_bins
from .code import LdpcCode


@dataclass
class ProtocolFrame:
    K_tot: int
    zeta: int
    K_max: int
    choice: np.ndarray                  # int32 [K_tot]: the preamble (bin) of each user
    loads: np.ndarray                   # int32 [zeta]: K_chi
    bins: List[Tuple[int, RaggedBin]] = field(default_factory=list)   # (chi, payload) per decodable bin
    members: dict = field(default_factory=dict)                       # chi -> users, in codeword-row order

    @property
    def overflow(self) -> np.ndarray:
        """Bins with more users than the decoder bank serves."""
        return np.nonzero(self.loads > self.K_max)[0]


def make_protocol_frames(code: LdpcCode, frames: int, K_tot: int, zeta: int, K_max: int,
                         ebn0_range: Tuple[float, float] | Sequence[float], seed: int) -> List[ProtocolFrame]:
    """``frames`` independent frames.  Each decodable bin draws its Eb/N0
    uniformly from ``ebn0_range`` and its payload from a child seed of the
    frame, so frame f is the same whatever ``frames`` is."""
    lo, hi = float(ebn0_range[0]), float(ebn0_range[1])
    out = []
    for child in np.random.SeedSequence(seed).spawn(frames):
        g = np.random.Generator(np.random.PCG64(child))
        choice = g.integers(0, zeta, size=K_tot).astype(np.int32)
        loads = np.bincount(choice, minlength=zeta).astype(np.int32)
        fr = ProtocolFrame(K_tot=K_tot, zeta=zeta, K_max=K_max, choice=choice, loads=loads)
        for chi in range(zeta):
            users = np.nonzero(choice == chi)[0]
            fr.members[chi] = users
            K = int(loads[chi])
            if K == 0 or K > K_max:
                continue
            eb = float(g.uniform(lo, hi))
            b = make_bins(code, K, 1, eb, int(g.integers(0, 2**31 - 1)))
            fr.bins.append((chi, RaggedBin(K=K, n=code.n, ebn0_db=eb, y=b.y[0], sigma2=float(b.sigma2[0]),
                                           codewords=b.codewords[0])))
        out.append(fr)
    return out
