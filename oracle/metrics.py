"""Set recovery metrics (Appendix, problem statement: grid -> message set,
permutation invariance and Hungarian row matching; main text, SER/CER).

SER = (1/(K L)) sum_{k,l} 1[Xhat[k,l] != X*[pi(k), l]] and CER = (1/K) sum_k
1[Xhat[k,:] != X*[pi(k),:]] under the row permutation pi that minimises the
total Hamming distance.
"""
from __future__ import annotations

from itertools import permutations
from typing import Dict, List, Tuple

import numpy as np
from scipy.optimize import linear_sum_assignment


def hamming_cost(Xhat: np.ndarray, Xstar: np.ndarray) -> np.ndarray:
    """D[k, k'] = Hamming distance between row k of Xhat and row k' of Xstar."""
    return (Xhat[:, None, :] != Xstar[None, :, :]).sum(axis=2)


def match_rows(Xhat: np.ndarray, Xstar: np.ndarray) -> np.ndarray:
    """pi with Xhat row k matched to Xstar row pi[k] (minimum total Hamming)."""
    rows, cols = linear_sum_assignment(hamming_cost(Xhat, Xstar))
    pi = np.empty(Xhat.shape[0], dtype=np.int64)
    pi[rows] = cols
    return pi


def match_rows_bruteforce(Xhat: np.ndarray, Xstar: np.ndarray) -> Tuple[np.ndarray, int]:
    """Exhaustive search over all K! permutations (small K only)."""
    D = hamming_cost(Xhat, Xstar)
    K = D.shape[0]
    best, best_pi = None, None
    for perm in permutations(range(K)):
        c = int(sum(D[k, perm[k]] for k in range(K)))
        if best is None or c < best:
            best, best_pi = c, np.array(perm)
    return best_pi, best


def ser_cer(Xhat: np.ndarray, Xstar: np.ndarray) -> Tuple[float, float]:
    pi = match_rows(Xhat, Xstar)
    err = Xhat != Xstar[pi]
    return float(err.mean()), float(err.any(axis=1).mean())


def decoded_set(Xhat: np.ndarray, codebook: Dict[bytes, int]) -> set:
    """Message indices whose codeword equals some row of Xhat."""
    out = set()
    for row in np.asarray(Xhat, dtype=np.uint8):
        key = row.tobytes()
        if key in codebook:
            out.add(codebook[key])
    return out


def valid_rows(Xhat: np.ndarray, H: np.ndarray) -> np.ndarray:
    """1 where H x_k = 0 (mod 2): the LDPC form of the row -> message rule."""
    return ((np.asarray(Xhat, np.int64) @ np.asarray(H, np.int64).T) % 2 == 0).all(axis=1)


def same_multiset(A: np.ndarray, B: np.ndarray) -> bool:
    """Unordered equality of the rows of two grids."""
    ka = sorted(r.tobytes() for r in np.asarray(A, np.uint8))
    kb = sorted(r.tobytes() for r in np.asarray(B, np.uint8))
    return ka == kb
