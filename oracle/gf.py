"""FP64 oracle pieces of the non-binary (GF(2^m), Q = 2^m) parity layer
(Q-ary LDPC code; FFT-BP's check update; the coefficient action Pi_alpha of
the latent Module B).  Test infrastructure only: the HIP library never
imports or calls it.

Readings where the text leaves a choice:
- the field is GF(2^m) in polynomial basis with a fixed primitive
  polynomial (GF(64): x^6 + x + 1; GF(8): x^3 + x + 1; GF(2): x + 1), and
  the bijection [Q] -> F_Q maps a symbol index to the element whose
  coefficient bits are the index's bits;
- Pi_alpha is the permutation a -> alpha a of symbol indices, as a matrix
  with (Pi_alpha)[alpha a, a] = 1, so that Pi_alpha applied to a one-hot
  vector of a gives the one-hot vector of alpha a.
"""
from __future__ import annotations

from itertools import product
from typing import Sequence

import numpy as np

PRIMITIVE = {1: 0b11, 3: 0b1011, 6: 0b1000011}


def gf_mul(a: int, b: int, m: int = 6) -> int:
    """Product in GF(2^m): carry-less multiply, then reduce by the primitive polynomial."""
    poly = PRIMITIVE[m]
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if a >> m:
            a ^= poly
    return r


def gf_inv(a: int, m: int = 6) -> int:
    """Multiplicative inverse by search (a != 0)."""
    if a == 0:
        raise ZeroDivisionError("0 has no inverse")
    for b in range(1, 1 << m):
        if gf_mul(a, b, m) == 1:
            return b
    raise ArithmeticError("not a field")


def pi_alpha(alpha: int, m: int = 6) -> np.ndarray:
    """Pi_alpha as a Q x Q permutation matrix: column a has its one at row alpha a."""
    Q = 1 << m
    P = np.zeros((Q, Q))
    for a in range(Q):
        P[gf_mul(alpha, a, m), a] = 1.0
    return P


def syndrome(H: np.ndarray, c: Sequence[int], m: int = 6) -> np.ndarray:
    """H c in F_Q (rows of H dotted with c, sums are XOR)."""
    out = np.zeros(H.shape[0], dtype=np.int64)
    for j in range(H.shape[0]):
        s = 0
        for l in range(H.shape[1]):
            if H[j, l]:
                s ^= gf_mul(int(H[j, l]), int(c[l]), m)
        out[j] = s
    return out


def check_message_brute(p_in: Sequence[np.ndarray], alphas_in: Sequence[int], alpha_out: int,
                        m: int = 6) -> np.ndarray:
    """Message of one check to the variable with coefficient alpha_out:
    m(a) = sum over the other variables' symbols x_i with
    alpha_out a + sum_i alpha_i x_i = 0 of prod_i p_i(x_i), normalised."""
    Q = 1 << m
    out = np.zeros(Q)
    for xs in product(range(Q), repeat=len(p_in)):
        s = 0
        w = 1.0
        for x, al, p in zip(xs, alphas_in, p_in):
            s ^= gf_mul(al, x, m)
            w *= p[x]
        # alpha_out a = s (in characteristic 2, -s = s)
        a = gf_mul(gf_inv(alpha_out, m), s, m)
        out[a] += w
    return out / out.sum()


def wht(v: np.ndarray) -> np.ndarray:
    """Walsh-Hadamard transform of length Q = 2^m: V[k] = sum_x (-1)^{popcount(k & x)} v[x]."""
    Q = v.shape[0]
    k = np.arange(Q)
    sign = np.array([[(-1) ** bin(int(a) & int(b)).count("1") for b in k] for a in k], dtype=np.float64)
    return sign @ v


def check_message_wht(p_in: Sequence[np.ndarray], alphas_in: Sequence[int], alpha_out: int,
                      m: int = 6) -> np.ndarray:
    """The same message through the transform domain (FFT-BP): permute each
    input by its coefficient, multiply the transforms (XOR convolution),
    transform back, and read the sum at alpha_out a."""
    Q = 1 << m
    acc = np.ones(Q)
    for p, al in zip(p_in, alphas_in):
        acc = acc * wht(pi_alpha(al, m) @ np.asarray(p, dtype=np.float64))
    s_dist = wht(acc) / Q
    out = np.array([s_dist[gf_mul(alpha_out, a, m)] for a in range(Q)])
    return out / out.sum()
