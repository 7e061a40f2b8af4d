"""Pins for the reveal schedule, the reveal rule, the refinement loop with
remasking, and the set-recovery metrics."""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import brute, metrics
from oracle.decode import DecodeOpts, decode_bin, decode_grid, row_status
from oracle.schedule import MASK, cosine_targets, linear_targets, reveal, step_counts

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_cosine_schedule_matches_paper_figures():
    g = json.load(open(os.path.join(GOLDEN, "cosine_reveal_T12_N24.json")))
    counts = step_counts(g["sites"], g["T"], "cosine")
    cum = np.concatenate([[0], np.cumsum(counts)])
    for t, want in g["cumulative_revealed"].items():
        assert cum[int(t)] == want, (t, cum[int(t)], want)
    # the float64 floor is what gives 5 at t=4 (rho(4)*24 rounds below 6)
    assert cosine_targets(24, 12)[3] == 5


@pytest.mark.parametrize("K,n,T,per", [(2, 32, 8, 8), (4, 128, 16, 32), (8, 256, 32, 64)])
def test_linear_schedule_counts(K, n, T, per):
    c = step_counts(K * n, T, "linear")
    assert c == [per] * T and sum(c) == K * n
    assert linear_targets(K * n, T)[-1] == K * n


@pytest.mark.parametrize("N,T", [(7, 3), (24, 12), (100, 7), (5, 5), (3, 1)])
def test_schedules_reveal_everything(N, T):
    for kind in ("linear", "cosine"):
        c = step_counts(N, T, kind)
        assert sum(c) == N and len(c) == T and min(c) >= 0


def test_reveal_picks_top_margins_with_index_tiebreak():
    X = np.full((2, 4), MASK, np.uint8)
    X[1, 3] = 1
    lg = np.zeros((2, 4, 2))
    marg = np.array([[0.5, -0.9, 0.9, 0.1], [0.9, 0.2, -0.3, 5.0]])
    lg[..., 0] = marg
    info = reveal(X, lg, 3, first_reveal=False)
    # margins 0.9 at (0,1),(0,2),(1,0) tie -> flat order 1, 2, 4; (1,3) is not masked
    assert info["selected"] == [(0, 1), (0, 2), (1, 0)]
    assert X[0, 1] == 1 and X[0, 2] == 0 and X[1, 0] == 0 and X[1, 3] == 1
    assert (X == MASK).sum() == 8 - 1 - 3


def test_first_reveal_restricts_to_best_row_per_slot():
    X = np.full((3, 4), MASK, np.uint8)
    marg = np.array([[0.1, 0.7, 0.3, 0.3],
                     [0.6, 0.2, 0.3, 0.1],
                     [0.9, 0.8, 0.3, 0.0]])
    lg = np.zeros((3, 4, 2))
    lg[..., 1] = -marg
    info = reveal(X, lg, 2, first_reveal=True)
    # slot winners: l0 -> k2 (0.9), l1 -> k2 (0.8), l2 -> k0 (tie 0.3, smallest k), l3 -> k0
    assert info["selected"] == [(2, 0), (2, 1)]
    info = reveal(X, lg, 5, first_reveal=True)
    # second call: slot winners among still-masked rows are (1,0) 0.6, (0,1) 0.7,
    # (0,2) 0.3 and (0,3) 0.3; only 4 candidates exist for r = 5
    assert info["selected"] == [(0, 1), (1, 0), (0, 2), (0, 3)]


def test_argmax_tie_goes_to_bit_zero():
    X = np.full((1, 2), MASK, np.uint8)
    lg = np.zeros((1, 2, 2))
    reveal(X, lg, 2, first_reveal=False)
    assert (X == 0).all()


def _tiny():
    return synth.regular_ldpc(12, seed=12)


def test_genie_refinement_recovers_map_set():
    """With an exact-posterior denoiser, confidence-ranked refinement must end
    on the brute-force joint-MAP message set whenever that set holds >= 0.99
    of the posterior mass (tiny code n=12, k=6, K=2)."""
    code = _tiny()
    C = brute.codebook(code)
    checked = 0
    for seed in range(40):
        bins = synth.make_bins(code, 2, 1, 5.0 + (seed % 4), seed=1000 + seed)
        y, s2 = bins.y[0].astype(np.float64), float(bins.sigma2[0])
        (i, j), mass = brute.map_pair(C, y, s2)
        if mass < 0.99:
            continue
        den = brute.genie_denoiser(C, y, s2)
        res = decode_grid(2, 12, code, den, T=24, opts=DecodeOpts(first_reveal=True, parity=False))
        assert metrics.same_multiset(res.X, C[[i, j]]), seed
        assert res.row_valid.all()
        checked += 1
    assert checked >= 10


def test_map_pair_beats_truth_likelihood():
    code = _tiny()
    C = brute.codebook(code)
    bins = synth.make_bins(code, 2, 1, 1.0, seed=3)
    y, s2 = bins.y[0].astype(np.float64), float(bins.sigma2[0])
    (i, j), _ = brute.map_pair(C, y, s2)
    L = brute.pair_loglik(C, y, s2)
    ti = int(np.nonzero((C == bins.codewords[0][0]).all(axis=1))[0][0])
    tj = int(np.nonzero((C == bins.codewords[0][1]).all(axis=1))[0][0])
    assert L[i, j] >= L[ti, tj] - 1e-12
    iu = np.triu_indices(C.shape[0], 1)
    assert abs(L[i, j] - L[iu].max()) < 1e-12


def _small_setup(K=3, n=32, L=2, d=32, h=4):
    cfg = synth.ModelCfg(L, d, h, n_max=n)
    w = synth.unpack_weights(synth.make_weights(cfg, 5, bias_std=0.02), cfg)
    code = synth.regular_ldpc(n, seed=1000 + n)
    bins = synth.make_bins(code, K, 2, 4.0, seed=77)
    return cfg, w, code, bins


def test_decode_invariants_hold_fixed_and_counts():
    cfg, w, code, bins = _small_setup()
    K, n, T = 3, 32, 8
    res = decode_bin(bins.y[0], bins.sigma2[0], code, K, w, cfg.n_layers, cfg.heads, T,
                     DecodeOpts(), keep=True)
    assert len(res.steps) == T
    for a, b in zip(res.steps[:-1], res.steps[1:]):
        rev = a["X_in"] != MASK
        assert np.array_equal(a["X_in"][rev], b["X_in"][rev])   # revealed tokens never change
    for s in res.steps:
        assert len(s["selected"]) == s["r"] == K * n // T
        assert len(set(s["selected"])) == s["r"]
        assert all(s["X_in"][k, l] == MASK for k, l in s["selected"])
    assert res.steps[0]["first"] and not res.steps[1]["first"]
    assert (res.X != MASK).all()
    assert np.isclose(res.steps[0]["gamma"], 1.0) and np.isclose(res.steps[-1]["gamma"], 1.0 / T)


def test_remask_rounds_clamp_and_trm():
    cfg, w, code, bins = _small_setup()
    K, n, T = 3, 32, 8
    opts = DecodeOpts(remask=True, remask_thr=0.9, remask_max_rounds=2)
    res = decode_bin(bins.y[0], bins.sigma2[0], code, K, w, cfg.n_layers, cfg.heads, T, opts, keep=True)
    assert res.rounds <= 2 and len(res.finals) == res.rounds + 1
    start = T
    grid_after = res.steps[T - 1]["X_in"].copy()
    for r in range(res.rounds):
        low = res.finals[r]["low"]
        T_rm = max(1, int(math.floor(T * int(low.sum()) / K)))
        seg = res.steps[start:start + T_rm]
        assert len(seg) == T_rm
        for s in seg:
            assert not s["first"]
            assert all(low[k] for k, _ in s["selected"])             # only remasked rows change
            assert (s["X_in"][~low] != MASK).all()
        assert sum(len(s["selected"]) for s in seg) == int(low.sum()) * n
        start += T_rm
    assert start == len(res.steps)


def test_remask_criterion():
    code = synth.regular_ldpc(32, seed=1032)
    cw = synth.make_bins(code, 2, 1, 4.0, seed=2).codewords[0]
    X = cw.copy()
    X[1, 0] ^= 1                                   # row 1 fails parity
    fin = np.zeros((2, 32, 2))
    fin[0, :, 0] = np.where(cw[0] == 0, 5.0, -5.0)  # confident row 0
    fin[1, :, 0] = 10.0
    syn, q, low = row_status(X, fin, code, 0.9)
    assert list(syn) == [False, True] and list(low) == [False, True]
    fin[0, :, 0] = 0.1                              # unconfident row 0: q = sigmoid(0.1) < 0.9
    _, q, low = row_status(X, fin, code, 0.9)
    assert low[0] and abs(q[0] - 1 / (1 + math.exp(-0.1))) < 1e-15


def test_hungarian_matches_bruteforce():
    rng = np.random.default_rng(0)
    for K in range(1, 7):
        for _ in range(5):
            A = rng.integers(0, 2, size=(K, 12))
            B = A[rng.permutation(K)] ^ (rng.random((K, 12)) < 0.2)
            pi = metrics.match_rows(A, B)
            _, best = metrics.match_rows_bruteforce(A, B)
            assert int(metrics.hamming_cost(A, B)[np.arange(K), pi].sum()) == best


def test_toy_example_set_rule():
    g = json.load(open(os.path.join(GOLDEN, "toy_set_recovery.json")))
    alpha = {c: i for i, c in enumerate(g["alphabet"])}
    enc = lambda s: np.array([alpha[c] for c in s], np.uint8)
    book = {enc(s).tobytes(): int(m) for m, s in g["codebook"].items()}
    grid = np.stack([enc(s) for s in g["decoded_grid"]])
    assert metrics.decoded_set(grid, book) == set(g["message_set"])
    assert metrics.decoded_set(grid[::-1], book) == set(g["message_set"])
    truth = np.stack([enc(g["codebook"]["3"]), enc(g["codebook"]["4"])])
    assert metrics.ser_cer(grid, truth) == (0.0, 0.0)


def test_single_step_reveals_everything():
    cfg, w, code, bins = _small_setup(K=2)
    res = decode_bin(bins.y[0], bins.sigma2[0], code, 2, w, cfg.n_layers, cfg.heads, 1, DecodeOpts())
    assert (res.X != MASK).all()


def test_remask_step_counts_by_hand():
    """Stub denoiser: row 0 always decodes to the all-zero codeword, rows 1 and
    2 to a word with a single 1 (nonzero syndrome).  With K=3, T=8 both
    remask rounds remask rows {1, 2}, so T_rm = floor(8*2/3) = 5 steps each:
    8 + 5 + 5 = 18 reveal steps and 3 final passes."""
    code = synth.regular_ldpc(32, seed=1032)

    def den(X, gamma):
        lg = np.zeros((3, 32, 2))
        lg[..., 0] = 3.0
        lg[1:, 0, 0] = -3.0
        return lg

    res = decode_grid(3, 32, code, den, T=8, opts=DecodeOpts(remask=True, remask_max_rounds=2))
    assert res.rounds == 2 and len(res.finals) == 3
    assert [len(s["selected"]) for s in res.steps] == [12] * 8 + [12, 13, 13, 13, 13] * 2
    assert list(res.row_valid) == [1, 0, 0]


def test_tau_schedule_endpoints_and_monotone():
    """Cosine temperature annealing (Appendix, inference temperature): tau_max
    at the first step, tau_min at the last, their mean half way, monotone."""
    from oracle.schedule import tau_schedule
    T = 9
    taus = [tau_schedule(t, T, 2.0, 0.5) for t in range(1, T + 1)]
    assert taus[0] == 2.0 and abs(taus[-1] - 0.5) < 1e-15
    assert abs(taus[(T - 1) // 2] - 1.25) < 1e-15        # w = 1/2 at t = (T + 1) / 2
    assert all(a >= b for a, b in zip(taus[:-1], taus[1:]))
    assert tau_schedule(1, 1, 2.0, 0.5) == 2.0


@pytest.mark.parametrize("tau", [0.25, 1.0, 4.0])
def test_max_probability_order_is_margin_order_at_any_temperature(tau):
    """With two symbols, max_a softmax(L / tau)_a is increasing in |L0 - L1|, so
    the reveal ranking (by margin) is the paper's confidence ranking at every
    temperature -- the reason tau_t changes no reveal."""
    rng = np.random.default_rng(3)
    L = rng.normal(0, 2, size=(400, 2))
    z = L / tau
    p = np.exp(z - z.max(axis=1, keepdims=True))
    p /= p.sum(axis=1, keepdims=True)
    conf = p.max(axis=1)
    margin = np.abs(L[:, 0] - L[:, 1])
    assert np.array_equal(np.argsort(-conf, kind="stable"), np.argsort(-margin, kind="stable"))


def _verbatim_den(K, n):
    # fixed logits: site (k, l) favours bit (k + l) % 2 with margin 1 + ((7 k + 3 l) % 11) / 10
    lg = np.zeros((K, n, 2))
    for k in range(K):
        for l in range(n):
            m = 1.0 + ((7 * k + 3 * l) % 11) / 10.0
            lg[k, l, (k + l) % 2] = m
    return lambda X, gamma: lg, lg


class _TinyCode:
    """A 3 x 6 parity-check matrix; only the final pass's syndrome reads it."""
    n, m = 6, 3
    H = np.array([[1, 1, 0, 1, 0, 0], [0, 1, 1, 0, 1, 0], [1, 0, 1, 0, 0, 1]], dtype=np.uint8)


@pytest.mark.parametrize("kind,counts", [("linear", [6, 0, 3, 3, 3, 3]), ("cosine", [6, 1, 1, 5, 3, 2])])
def test_verbatim_first_reveal_counts_by_hand(kind, counts):
    """first_reveal = 2 (the paper's wording): step 1 reveals each slot's most
    confident site, then the cumulative targets resume.  K = 3, n = 6, T = 6,
    N = 18: linear targets 3, 6, 9, 12, 15, 18 give 6, max(0, 6-6)=0, 3, 3, 3, 3;
    cosine targets floor(rho(t) 18) in float64 = 1, 4, 8, 13, 16, 18 (rho(3) 18
    evaluates to 8.999999999999998, the rounding the paper's figures pin)
    give 6, max(1, 4-6)=1, 8-7=1, 5, 3 and the remaining 2."""
    den, lg = _verbatim_den(3, 6)
    res = decode_grid(3, 6, _TinyCode(), den, T=6, opts=DecodeOpts(schedule=kind, first_reveal=2), keep=True)
    assert [len(s["selected"]) for s in res.steps] == counts
    first = res.steps[0]["selected"]
    assert sorted(l for _, l in first) == list(range(6))          # one site per slot
    c = np.abs(lg[..., 0] - lg[..., 1])
    for k, l in first:
        assert k == int(np.argmax(c[:, l]))                       # its most confident row
    hybrid = decode_grid(3, 6, _TinyCode(), den, T=6, opts=DecodeOpts(schedule=kind, first_reveal=1), keep=True)
    assert len(hybrid.steps[0]["selected"]) == (3 if kind == "linear" else 1)


def test_remask_confidence_at_tau_min():
    """q_k = mean_l max_a softmax(L / tau_min): sigmoid(|L0 - L1| / tau_min)."""
    code = synth.regular_ldpc(32, seed=1032)
    X = np.zeros((1, 32), np.uint8)                                # all-zero word: zero syndrome
    fin = np.zeros((1, 32, 2))
    fin[0, :16, 0] = 2.0                                           # margins 2 on half the slots, 0 on the rest
    for tau in (1.0, 0.5, 2.0):
        _, q, _ = row_status(X, fin, code, 0.9, tau)
        want = 0.5 * (1 / (1 + math.exp(-2.0 / tau)) + 0.5)
        assert abs(q[0] - want) < 1e-15


def test_relative_gaps_put_each_decision_against_its_logits():
    """Three masked sites with margins 3, 2.5 and 0.5 (logits up to 10):
    revealing one leaves the cut 3 - 2.5 = 0.5 between sites of largest
    |L| 10 and 4, so rcut = 0.5 / (4 * 10); the revealed site's argmax
    margin 3 over its logits (10, 7) gives rsel = 3 / (2 * 10)."""
    from oracle.schedule import reveal
    X = np.full((1, 3), 2, dtype=np.uint8)
    logits = np.array([[[10.0, 7.0], [1.5, 4.0], [0.25, -0.25]]])
    info = reveal(X, logits, 1, False)
    assert info["selected"] == [(0, 0)] and X[0, 0] == 0
    assert info["gaps"]["cut"] == pytest.approx(0.5) and info["gaps"]["rcut"] == pytest.approx(0.5 / 40.0)
    assert info["gaps"]["sel"] == pytest.approx(3.0) and info["gaps"]["rsel"] == pytest.approx(3.0 / 20.0)


def test_a_tie_between_identical_rows_measures_the_gap_past_it():
    """Rows 1 and 2 identical (margin 2 at slot 0), row 0 margin 2.3, row 3
    margin 1.9: revealing two sites takes row 0 and, by index, row 1; the
    decision turns only if row 3 crosses the tied pair (gap 0.1) or the
    tied pair crosses row 0 (gap 0.3), so cut = 0.1 and one tie is counted."""
    from oracle.schedule import reveal
    X = np.full((4, 1), 2, dtype=np.uint8)
    logits = np.array([[[2.3, 0.0]], [[2.0, 0.0]], [[2.0, 0.0]], [[1.9, 0.0]]])
    info = reveal(X, logits, 2, False)
    assert info["selected"] == [(0, 0), (1, 0)]
    assert info["gaps"]["cut"] == pytest.approx(0.1) and info["gaps"]["ties"] == 1
    assert info["gaps"]["rcut"] == pytest.approx(0.1 / (4 * 2.0))
