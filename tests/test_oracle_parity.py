"""Pins for Module B (binary logit-bias parity messages) in the oracle."""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle.parity import check_messages, module_b, parity_bias, phi, site_llr, syndrome


def _brute_extrinsic(lams):
    """Exact LLR of the parity of independent bits with LLRs lams (bit 0 vs 1):
    log P(sum of bits even) - log P(odd), by enumerating all assignments."""
    p0 = [1.0 / (1.0 + math.exp(-l)) for l in lams]      # P(bit = 0)
    even = odd = 0.0
    for bits in itertools.product([0, 1], repeat=len(lams)):
        pr = 1.0
        for b, q in zip(bits, p0):
            pr *= q if b == 0 else 1.0 - q
        if sum(bits) % 2 == 0:
            even += pr
        else:
            odd += pr
    return math.log(even) - math.log(odd)


def test_phi_self_inverse():
    x = np.linspace(0.05, 15, 50)
    np.testing.assert_allclose(phi(phi(x)), x, rtol=1e-9)


def test_phi_form_equals_tanh_rule():
    rng = np.random.default_rng(0)
    for _ in range(50):
        lams = rng.normal(0, 2.0, size=5)
        sgn = np.prod(np.where(lams >= 0, 1.0, -1.0))
        m = sgn * phi(np.sum(phi(np.abs(lams))))
        ref = 2.0 * np.arctanh(np.prod(np.tanh(lams / 2.0)))
        assert abs(m - ref) < 1e-9 * max(1.0, abs(ref))


def _code(n, seed):
    return synth.regular_ldpc(n, seed=seed)


@pytest.mark.parametrize("n,seed", [(12, 3), (32, 1032)])
def test_messages_equal_bruteforce_check_marginal(n, seed):
    code = _code(n, seed)
    rng = np.random.default_rng(n)
    lam = rng.normal(0, 3.0, size=(2, n))
    for j, l, msg in check_messages(lam, code, 1e-6):
        others = [int(v) for v in code.col_idx[code.row_ptr[j]:code.row_ptr[j + 1]] if v != l]
        for k in range(2):
            ref = _brute_extrinsic(lam[k, others].tolist())
            assert abs(msg[k] - ref) < 1e-8 * max(1, abs(ref)), (j, l, k)


def test_bias_sums_messages_over_checks_of_slot():
    code = _code(32, 1032)
    rng = np.random.default_rng(1)
    lam = rng.normal(0, 2.0, size=(3, 32))
    b = parity_bias(lam, code, 1e-6)
    for l in range(32):
        checks = [j for j in range(code.m) if code.H[j, l]]
        assert len(checks) == 3
        for k in range(3):
            ref = 0.0
            for j in checks:
                others = [v for v in np.nonzero(code.H[j])[0] if v != l]
                ref += _brute_extrinsic(lam[k, others].tolist())
            assert abs(b[k, l] - ref) < 1e-8 * max(1, abs(ref))


def test_zero_syndrome_is_fixed_point():
    code = _code(64, 1064)
    bins = synth.make_bins(code, 3, 1, 4.0, seed=9)
    cw = bins.codewords[0]
    rng = np.random.default_rng(2)
    mag = rng.uniform(0.01, 5.0, size=cw.shape)
    lam = np.where(cw == 0, mag, -mag)
    lbar = np.stack([lam / 2, -lam / 2], axis=-1)
    X = np.full(cw.shape, 2, np.uint8)
    out = module_b(lbar, X, code)
    d = out[..., 0] - out[..., 1]
    assert np.all(np.sign(d) == np.sign(lam))
    b = parity_bias(lam, code, 1e-6)
    assert np.all(np.sign(b) == np.sign(lam))


def test_single_erasure_message():
    code = _code(32, 1032)
    cw = synth.make_bins(code, 1, 1, 6.0, seed=4).codewords[0][0]
    X = cw[None, :].copy()
    X[0, 5] = 2
    lbar = np.zeros((1, 32, 2))
    lam = site_llr(lbar, X, 20.0)
    b = parity_bias(lam, code, 1e-6)
    expect_mag = phi(5 * phi(20.0))
    assert abs(expect_mag - 18.39) < 0.01
    want_sign = 1.0 if cw[5] == 0 else -1.0
    # each of the 3 checks on slot 5 sees all other bits revealed
    assert abs(b[0, 5] - 3 * want_sign * expect_mag) < 1e-9


def test_bias_is_split_symmetrically_with_eta():
    code = _code(32, 1032)
    rng = np.random.default_rng(3)
    lbar = rng.normal(0, 0.3, size=(2, 32, 2))
    X = rng.integers(0, 3, size=(2, 32)).astype(np.uint8)
    lam = site_llr(lbar, X, 20.0)
    b = parity_bias(lam, code, 1e-6)
    for eta in (0.5, 1.0, 2.0):
        out = module_b(lbar, X, code, eta=eta)
        np.testing.assert_allclose(out[..., 0] - lbar[..., 0], eta * b / 2, atol=1e-12)
        np.testing.assert_allclose(out[..., 1] - lbar[..., 1], -eta * b / 2, atol=1e-12)


def test_revealed_sites_enter_saturated_and_clip():
    lbar = np.array([[[30.0, 0.0], [0.0, 0.1], [0.3, 0.0]]])
    X = np.array([[2, 0, 1]], np.uint8)
    lam = site_llr(lbar, X, 20.0)
    np.testing.assert_allclose(lam, [[20.0, 20.0, -20.0]])


def test_syndrome_zero_on_codewords():
    code = _code(128, 1128)
    cw = synth.make_bins(code, 4, 3, 4.0, seed=1).codewords.reshape(-1, 128)
    assert not syndrome(cw, code).any()
    bad = cw.copy()
    bad[0, 7] ^= 1
    assert syndrome(bad, code)[0].sum() == 3
