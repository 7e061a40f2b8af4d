"""Pins of the GF(2^m) parity pieces in the oracle (Q-ary LDPC code;
FFT-BP's check update; the coefficient action Pi_alpha)."""
import math

import numpy as np
import pytest

from oracle import gf


def _table(m):
    Q = 1 << m
    return np.array([[gf.gf_mul(a, b, m) for b in range(Q)] for a in range(Q)])


@pytest.mark.parametrize("m", [1, 3, 6])
def test_field_axioms_exhaustively(m):
    Q = 1 << m
    T = _table(m)
    a = np.arange(Q)
    assert np.array_equal(T, T.T)                                         # commutative
    assert np.array_equal(T[T[:, :, None], a[None, None, :]], T[a[:, None, None], T[None, :, :]])  # associative
    assert np.array_equal(T[:, 1], a) and np.all(T[:, 0] == 0)            # 1 and 0
    # distributive over XOR: a (b ^ c) = ab ^ ac
    assert np.array_equal(T[a[:, None, None], a[None, :, None] ^ a[None, None, :]],
                          T[:, :, None] ^ T[:, None, :])
    for x in range(1, Q):                                                 # every nonzero invertible
        assert T[x, gf.gf_inv(x, m)] == 1
    # the class of x is primitive: its powers run through all Q - 1 nonzero elements
    if m > 1:
        seen, y = set(), 1
        for _ in range(Q - 1):
            y = gf.gf_mul(y, 2, m)
            seen.add(y)
        assert len(seen) == Q - 1


def test_pi_alpha_is_the_multiplication_action():
    m = 6
    Q = 1 << m
    assert np.array_equal(gf.pi_alpha(1, m), np.eye(Q))
    rng = np.random.default_rng(0)
    for _ in range(5):
        al, be = (int(v) for v in rng.integers(1, Q, 2))
        Pa, Pb = gf.pi_alpha(al, m), gf.pi_alpha(be, m)
        assert np.array_equal(Pa.sum(0), np.ones(Q)) and np.array_equal(Pa.sum(1), np.ones(Q))
        assert np.array_equal(Pa @ Pb, gf.pi_alpha(gf.gf_mul(al, be, m), m))
        a = int(rng.integers(0, Q))
        assert np.argmax(Pa @ np.eye(Q)[a]) == gf.gf_mul(al, a, m)


def test_syndrome_of_a_check_solved_for_its_last_symbol():
    m = 6
    rng = np.random.default_rng(1)
    H = np.zeros((1, 4), dtype=np.int64)
    H[0, :3] = rng.integers(1, 64, 3)
    c = [int(v) for v in rng.integers(0, 64, 4)]
    s = gf.gf_mul(int(H[0, 0]), c[0], m) ^ gf.gf_mul(int(H[0, 1]), c[1], m)
    c[2] = gf.gf_mul(gf.gf_inv(int(H[0, 2]), m), s, m)
    assert gf.syndrome(H, c, m)[0] == 0
    c[1] ^= 5
    assert gf.syndrome(H, c, m)[0] != 0


def test_wht_is_an_involution_up_to_q():
    v = np.random.default_rng(2).random(64)
    np.testing.assert_allclose(gf.wht(gf.wht(v)), 64 * v, rtol=1e-12)


@pytest.mark.parametrize("m,deg", [(3, 3), (6, 2)])
def test_check_message_transform_equals_brute_force(m, deg):
    Q = 1 << m
    rng = np.random.default_rng(3 + m)
    p = [rng.random(Q) for _ in range(deg)]
    p = [x / x.sum() for x in p]
    al = [int(v) for v in rng.integers(1, Q, deg)]
    out = int(rng.integers(1, Q))
    np.testing.assert_allclose(gf.check_message_wht(p, al, out, m), gf.check_message_brute(p, al, out, m),
                               rtol=1e-9, atol=1e-12)


def test_binary_check_message_is_the_tanh_rule():
    """GF(2): the message's log-ratio is 2 atanh(prod tanh(L_i / 2))."""
    rng = np.random.default_rng(4)
    L = rng.normal(0, 2, 3)
    p = [np.array([1 / (1 + math.exp(-x)), 1 / (1 + math.exp(x))]) for x in L]
    msg = gf.check_message_brute(p, [1, 1, 1], 1, m=1)
    assert math.isclose(math.log(msg[0] / msg[1]), 2 * math.atanh(np.prod(np.tanh(L / 2))), rel_tol=1e-10)
