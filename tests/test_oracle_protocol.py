"""Pins of the protocol-level wrapper in the oracle and of the frame
generator (Appendix, protocol-level scaling by stochastic binning)."""
import itertools
import math

import numpy as np

import synth
from oracle import protocol as Pr
from oracle.metrics import valid_rows


def test_overflow_below_the_papers_bound_at_25_bins():
    """With zeta = 25 bins and a bank up to K_max = 8, the paper puts the
    Poisson overflow probability below 1e-3 for every K_tot <= 60; it grows
    with the load."""
    vals = [Pr.poisson_overflow(K_tot / 25.0, 8) for K_tot in range(10, 101, 10)]
    assert all(v < 1e-3 for v in vals[:6])
    assert all(a < b for a, b in zip(vals, vals[1:]))


def test_poisson_overflow_special_cases():
    for kappa in (0.3, 1.0, 4.0):
        assert math.isclose(Pr.poisson_overflow(kappa, 0), 1.0 - math.exp(-kappa), rel_tol=1e-12)
        assert math.isclose(Pr.poisson_overflow(kappa, 1), 1.0 - math.exp(-kappa) * (1 + kappa), rel_tol=1e-12)
    assert Pr.poisson_overflow(1e-9, 3) < 1e-30 + 1e-16
    assert Pr.poisson_overflow(2.0, 60) < 1e-15


def test_binomial_overflow_by_enumeration():
    """Every one of zeta^K_tot preamble choices, counted."""
    for K_tot, zeta, K_max in ((6, 3, 2), (5, 2, 3), (7, 4, 1)):
        over = users = 0
        for choice in itertools.product(range(zeta), repeat=K_tot):
            loads = Pr.bin_loads(choice, zeta)
            over += int(loads[0] > K_max)
            users += int(loads[loads > K_max].sum())
        total = zeta ** K_tot
        assert math.isclose(Pr.binomial_overflow(K_tot, zeta, K_max), over / total, rel_tol=1e-10)
        assert math.isclose(Pr.expected_overflow_users(K_tot, zeta, K_max), users / total, rel_tol=1e-10)


def test_binomial_tends_to_poisson():
    """At fixed kappa = K_tot / zeta the binomial load tends to Poisson(kappa),
    with a gap shrinking like 1 / zeta."""
    gaps = [abs(Pr.binomial_overflow(int(2.4 * z), z, 8) - Pr.poisson_overflow(2.4, 8)) for z in (10, 50, 250)]
    assert gaps[0] > gaps[1] > gaps[2] and 0.5 < (gaps[2] * 250) / (gaps[1] * 50) < 2.0


def _frame_and_grids():
    code = synth.regular_ldpc(32, seed=1032)
    fr = synth.make_protocol_frames(code, 1, 30, 6, 6, (3.0, 5.0), seed=4)[0]
    sent = {chi: b.codewords for chi, b in fr.bins}
    return fr, sent


def test_frame_errors_count_overflow_users_and_missing_codewords():
    fr, sent = _frame_and_grids()
    ov_users = int(fr.loads[fr.loads > fr.K_max].sum())
    assert Pr.frame_user_errors(fr.loads, fr.K_max, sent, sent) == ov_users
    # row order does not matter
    perm = {chi: g[::-1].copy() for chi, g in sent.items()}
    assert Pr.frame_user_errors(fr.loads, fr.K_max, sent, perm) == ov_users
    chi, g = next((c, g) for c, g in sent.items() if g.shape[0] >= 2)
    bad = dict(sent)
    flip = g.copy()
    flip[0, 3] ^= 1
    bad[chi] = flip
    assert Pr.frame_user_errors(fr.loads, fr.K_max, sent, bad) == ov_users + 1
    dup = g.copy()
    dup[1] = dup[0]                       # one user returned twice, another missing
    bad[chi] = dup
    assert Pr.frame_user_errors(fr.loads, fr.K_max, sent, bad) == ov_users + 1


def test_generator_loads_bins_and_overflow_rate():
    code = synth.regular_ldpc(32, seed=1032)
    K_tot, zeta, K_max = 40, 5, 8
    H = np.zeros((code.m, code.n), dtype=np.int64)
    for j in range(code.m):
        H[j, code.col_idx[code.row_ptr[j]:code.row_ptr[j + 1]]] = 1
    frames = synth.make_protocol_frames(code, 200, K_tot, zeta, K_max, (3.0, 5.0), seed=11)
    over = 0
    for fr in frames:
        assert fr.loads.sum() == K_tot
        assert np.array_equal(fr.loads, Pr.bin_loads(fr.choice, zeta))
        assert sorted(chi for chi, _ in fr.bins) == [c for c in range(zeta) if 1 <= fr.loads[c] <= K_max]
        for chi, b in fr.bins:
            assert b.K == fr.loads[chi] == len(fr.members[chi])
            assert len({r.tobytes() for r in b.codewords}) == b.K          # distinct messages
            assert valid_rows(b.codewords, H).all()                        # codewords of the code
        over += int((fr.loads > K_max).sum())
    p = Pr.binomial_overflow(K_tot, zeta, K_max)
    N = 200 * zeta
    assert abs(over / N - p) < 5 * math.sqrt(p * (1 - p) / N)


def test_generator_frames_do_not_depend_on_the_frame_count():
    code = synth.regular_ldpc(32, seed=1032)
    a = synth.make_protocol_frames(code, 3, 20, 5, 6, (3.0, 5.0), seed=2)
    b = synth.make_protocol_frames(code, 5, 20, 5, 6, (3.0, 5.0), seed=2)
    for fa, fb in zip(a, b):
        assert np.array_equal(fa.choice, fb.choice)
        assert [c for c, _ in fa.bins] == [c for c, _ in fb.bins]
        assert all(np.array_equal(x.y, y.y) for (_, x), (_, y) in zip(fa.bins, fb.bins))
