"""The refinement loop with final pass and quality-guided remasking.

Paper: refinement loop (method section), final gamma = 0 pass (Appendix,
inference schedule), quality-guided remasking (Appendix, PRISM-style
remasking and its algorithm).  The learned quality head is replaced by a
fixed row criterion: a row is low-quality when its syndrome H x is nonzero
or when its mean over slots of the final-pass max probability is below a
threshold; low rows are remasked, the others clamped, and T_rm =
max(1, floor(T |K_low| / K)) steps are run, for at most a set number of
rounds.  First-reveal applies only to the initial pass from the all-mask
grid, and only when that pass has more than one step (a single step must
reveal every site); ``first_reveal`` = 1 narrows the step-1 candidates to each
slot's best row (hybrid), 2 reveals all of those candidates at step 1 (the
paper's wording).  The remask confidence is taken at the annealed
temperature's end value tau_min.  By default the output is the held-fixed
grid; ``final_argmax`` returns the per-site argmax of the last final pass
instead.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from .denoiser import denoise
from .evidence import evidence
from .parity import syndrome
from .schedule import MASK, cosine_targets, linear_targets, reveal, tau_schedule


@dataclass
class DecodeOpts:
    schedule: str = "linear"
    first_reveal: int = 1          # 0 off, 1 hybrid (candidates only), 2 verbatim (reveal them all)
    remask: bool = False
    remask_thr: float = 0.9
    remask_max_rounds: int = 2
    final_argmax: bool = False
    tau: float = 1.0
    eta: float = 1.0
    lam_max: float = 20.0
    lam_min: float = 1e-6
    tau_max: float = 1.0           # inference temperature at the first refinement step
    tau_min: float = 1.0           # ... at the last; the remask confidence uses it
    parity: bool = True
    # PRISM-style head instead of the fixed criterion: row_conf(den output) -> [K]
    # confidences, remasked while below phi[s] after pass s, at most len(phi) rounds
    row_conf: Optional[Callable] = None
    phi: tuple = (0.96, 0.90, 0.85)


@dataclass
class DecodeResult:
    X: np.ndarray                 # uint8 [K][n] output grid
    final_logits: np.ndarray      # float64 [K][n][2] logits of the last final pass
    row_valid: np.ndarray         # uint8 [K], 1 iff H x_k = 0
    rounds: int                   # remask rounds run
    steps: List[Dict] = field(default_factory=list)   # per-step trace
    finals: List[Dict] = field(default_factory=list)  # per final pass: logits, low rows, q, gaps
    min_gap: float = float("inf")


def row_status(X: np.ndarray, fin_logits: np.ndarray, code, thr: float, tau: float = 1.0):
    """(syndrome nonzero [K] bool, q [K] mean max-prob at temperature tau, low [K] bool).
    For two symbols max_a softmax(L / tau)_a = sigmoid(|L0 - L1| / tau)."""
    syn = syndrome(X, code).any(axis=1)
    c = np.abs(fin_logits[..., 0] - fin_logits[..., 1])
    q = (1.0 / (1.0 + np.exp(-c / tau))).mean(axis=1)
    return syn, q, syn | (q < thr)


def _targets(kind: str, n_masked: int, T: int):
    return linear_targets(n_masked, T) if kind == "linear" else cosine_targets(n_masked, T)


def run_pass(X: np.ndarray, T: int, den: Callable, opts: DecodeOpts, first: bool,
             steps: List[Dict], keep: bool) -> None:
    """One decoding pass of T reveal steps over the currently masked sites of X."""
    K, n = X.shape
    n_masked = int((X == MASK).sum())
    R = _targets(opts.schedule, n_masked, T)
    done = 0
    for t in range(1, T + 1):
        r = R[t - 1] - done
        if opts.schedule == "cosine":
            r = max(1, r)
            if t == T:
                r = n_masked - done
        r = max(0, min(r, n_masked - done))
        gamma = float((X == MASK).sum()) / float(K * n)
        X_in = X.copy()
        out = den(X, gamma)
        logits = out["logits"] if isinstance(out, dict) else out
        use_first = bool(first) and t == 1 and T > 1
        if use_first and int(first) == 2:
            r = K * n                             # verbatim: every slot's selected site
        info = reveal(X, logits, r, use_first)
        done += len(info["selected"])
        rec = {"t": t, "r": r, "gamma": gamma, "first": use_first, "gaps": info["gaps"],
               "selected": info["selected"], "tau": tau_schedule(t, T, opts.tau_max, opts.tau_min)}
        if keep:
            rec["X_in"] = X_in
            rec["logits"] = logits
            rec["lbar"] = out.get("lbar") if isinstance(out, dict) else None
        steps.append(rec)


def decode_grid(K: int, n: int, code, den: Callable, T: int, opts: DecodeOpts,
                keep: bool = False) -> DecodeResult:
    """Decode with any denoiser den(X, gamma) -> logits [K][n][2] (or dict with 'logits')."""
    X = np.full((K, n), MASK, dtype=np.uint8)
    steps: List[Dict] = []
    finals: List[Dict] = []
    run_pass(X, T, den, opts, opts.first_reveal, steps, keep)
    rounds = 0
    while True:
        out = den(X, float((X == MASK).sum()) / float(K * n))
        fin = out["logits"] if isinstance(out, dict) else out
        if opts.row_conf is None:
            syn, q, low = row_status(X, fin, code, opts.remask_thr, opts.tau_min)
            finals.append({"logits": fin, "low": low.copy(), "q": q, "syn": syn,
                           "gap_q": float(np.min(np.abs(q - opts.remask_thr))) if opts.remask else float("inf")})
            max_rounds = opts.remask_max_rounds
        else:
            max_rounds = len(opts.phi)
            q = opts.row_conf(out)
            thr = opts.phi[rounds] if rounds < max_rounds else -np.inf
            low = q < thr
            finals.append({"logits": fin, "low": low.copy(), "q": q, "syn": None,
                           "gap_q": float(np.min(np.abs(q - thr))) if opts.remask and rounds < max_rounds
                           else float("inf")})
        if not opts.remask or rounds >= max_rounds or not low.any():
            break
        X[low, :] = MASK
        T_rm = max(1, int(math.floor(T * int(low.sum()) / K)))
        run_pass(X, T_rm, den, opts, False, steps, keep)
        rounds += 1
    Xout = X.copy()
    if opts.final_argmax:
        Xout = np.where(fin[..., 0] >= fin[..., 1], 0, 1).astype(np.uint8)
    valid = (~syndrome(Xout, code).any(axis=1)).astype(np.uint8)
    gaps = [min(s["gaps"][k] for k in ("cut", "sel", "slot")) for s in steps] + [f["gap_q"] for f in finals]
    return DecodeResult(X=Xout, final_logits=fin, row_valid=valid, rounds=rounds, steps=steps,
                        finals=finals, min_gap=float(min(gaps)) if gaps else float("inf"))


def decode_bin(y, sigma2: float, code, K: int, w: Dict[str, np.ndarray], n_layers: int,
               heads: int, T: int, opts: Optional[DecodeOpts] = None, keep: bool = False) -> DecodeResult:
    """Decode one bin with the seeded-weight CIDER denoiser."""
    opts = opts or DecodeOpts()
    _, p = evidence(y, sigma2, K)

    def den(X, gamma):
        return denoise(X, p, code, w, n_layers, heads, gamma, tau=opts.tau, eta=opts.eta,
                       lam_max=opts.lam_max, lam_min=opts.lam_min, parity=opts.parity)

    return decode_grid(K, code.n, code, den, T, opts, keep)
