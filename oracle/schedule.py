"""Reveal schedules and the confidence-ranked reveal rule.

Paper (overall refinement loop; Appendix, masked-diffusion inference):
at each step the masked sites with the highest confidence are set to their
argmax symbol, the number revealed so far following a schedule; on the
first step of decoding from the all-mask grid each slot is first narrowed
to its single most confident row ("first-reveal stabilisation").

Readings taken here (all stated in the design notes):
  * confidence is ranked by the logit margin |L0 - L1|, which orders sites
    exactly as max softmax probability does for two symbols (and as it does
    at any temperature), without saturating to 1.0;
  * ties in the ranking go to the smaller flat index k*n + l, ties in the
    first-reveal row choice to the smaller k, ties in the argmax to bit 0;
  * first-reveal restricts the step-1 candidate set, and the number revealed
    still follows the schedule ("hybrid", the default); the paper's verbatim
    rule -- step 1 reveals every slot's selected site -- is the other mode,
    after which the cumulative targets resume (steps whose target is already
    met reveal nothing under the linear schedule, one site under cosine);
  * the inference temperature is annealed from tau_max at the first step to
    tau_min at the last by the paper's cosine weight; with two symbols the
    max-probability order of softmax(L / tau) is the margin order for every
    tau > 0, so tau_t changes no reveal, and only the final pass's
    confidence (the remask test, taken at tau_min) depends on it;
  * linear schedule (R_t = floor(t N / T)) by default; the cosine schedule
    R_t = floor(rho(t) N), rho(t) = (1 - cos(pi t / T)) / 2, evaluated in
    float64 with at least one site per step.
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

MASK = 2


def linear_targets(n_masked: int, T: int) -> List[int]:
    """Cumulative reveal targets R_1..R_T with R_t = floor(t * N / T)."""
    return [(t * n_masked) // T for t in range(1, T + 1)]


def cosine_targets(n_masked: int, T: int) -> List[int]:
    """Cumulative targets R_t = floor(rho(t) * N) computed in float64."""
    return [int(math.floor(0.5 * (1.0 - math.cos(math.pi * t / T)) * n_masked)) for t in range(1, T + 1)]


def step_counts(n_masked: int, T: int, kind: str = "linear") -> List[int]:
    """Per-step reveal counts r_t assuming every requested site is available."""
    if kind == "linear":
        R = linear_targets(n_masked, T)
    elif kind == "cosine":
        R = cosine_targets(n_masked, T)
    else:
        raise ValueError(kind)
    out, done = [], 0
    for t, Rt in enumerate(R, start=1):
        r = Rt - done
        if kind == "cosine":
            r = max(1, r)
            if t == T:
                r = n_masked - done
        r = max(0, min(r, n_masked - done))
        out.append(r)
        done += r
    return out


def tau_schedule(t: int, T: int, tau_max: float, tau_min: float) -> float:
    """Inference temperature of refinement step t in 1..T:
    tau_max w(t) + tau_min (1 - w(t)), w(t) = (1 + cos(pi (t - 1) / (T - 1))) / 2,
    with w = 1 when T = 1 (the first step is also the last)."""
    w = 1.0 if T == 1 else 0.5 * (1.0 + math.cos(math.pi * (t - 1) / (T - 1)))
    return tau_max * w + tau_min * (1.0 - w)


def margins(logits: np.ndarray) -> np.ndarray:
    return np.abs(logits[..., 0] - logits[..., 1])


def _boundary_gap(vals, scales, i):
    """Distance from a tie of the decision between positions i (kept) and
    i + 1 (dropped) of the descending values `vals`: their difference; or,
    when they are equal -- identical user rows, whose logits are
    bit-identical in any precision and whose order the index tie-break fixes
    -- the distance from the tied value to the nearest distinct value on
    either side, since only a value crossing the tied group changes the
    outcome.  Returns (gap, relative gap, tied); the relative gap divides by 4
    max(1, |logits|) of the two sites compared (inf when nothing competes)."""
    inf = float("inf")
    v, w = vals[i], vals[i + 1]
    if v > w:
        return float(v - w), float(v - w) / (4.0 * max(scales[i], scales[i + 1])), False
    gap, rel = inf, inf
    up = np.nonzero(vals[:i] > v)[0]
    if up.size:
        j = up[-1]
        gap = float(vals[j] - v)
        rel = gap / (4.0 * max(scales[j], scales[i]))
    down = np.nonzero(vals[i + 1:] < v)[0]
    if down.size:
        j = i + 1 + down[0]
        g = float(v - vals[j])
        if g < gap:
            gap = g
        rel = min(rel, g / (4.0 * max(scales[j], scales[i])))
    return gap, rel, True


def reveal(X: np.ndarray, logits: np.ndarray, r: int, first_reveal: bool) -> Dict:
    """Reveal up to r masked sites of X [K][n] in place; returns selection info.

    'gaps' reports how far each integer decision in this step sits from a
    tie: cut (between the r-th and the (r+1)-th candidate), sel (smallest
    selected margin, i.e. the argmax decision) and slot (first-reveal choice
    of a slot's row), each through _boundary_gap, which looks past ties
    between identical rows ('ties' counts them).  The r-prefixed entries put
    each gap against the logits it is made of: a margin difference of two
    sites over 4 max(1, |logits of both sites|), an argmax margin over
    2 max(1, |its two logits|) -- the gap a relative logit error of that
    size, max |dL| / max(1, |L|), can close at most.
    """
    K, n = X.shape
    c = margins(logits)
    scale = np.maximum(1.0, np.abs(logits).max(axis=-1))
    masked = X == MASK
    inf = float("inf")
    gaps = {"cut": inf, "sel": inf, "slot": inf, "rcut": inf, "rsel": inf, "rslot": inf, "ties": 0}
    if first_reveal:
        cm = np.where(masked, c, -np.inf)
        cand = []
        for l in range(n):
            if not masked[:, l].any():
                continue
            k = int(np.argmax(cm[:, l]))           # first maximum -> smallest k
            cand.append((k, l))
            ks = np.nonzero(masked[:, l])[0]
            if ks.size > 1:
                o = ks[np.argsort(-cm[ks, l], kind="stable")]
                g, rg, tied = _boundary_gap(cm[o, l], scale[o, l], 0)
                gaps["slot"] = min(gaps["slot"], g)
                gaps["rslot"] = min(gaps["rslot"], rg)
                gaps["ties"] += int(tied)
    else:
        ks, ls = np.nonzero(masked)
        cand = list(zip(ks.tolist(), ls.tolist()))
    if not cand or r <= 0:
        return {"selected": [], "gaps": gaps}
    cvals = np.array([c[k, l] for k, l in cand])
    flat = np.array([k * n + l for k, l in cand])
    order = np.lexsort((flat, -cvals))             # by margin desc, then flat index asc
    take = order[:min(r, len(cand))]
    if len(cand) > r:
        sc = np.array([scale[cand[i]] for i in order])
        g, rg, tied = _boundary_gap(cvals[order], sc, r - 1)
        gaps["cut"], gaps["rcut"] = g, rg
        gaps["ties"] += int(tied)
    sel = [cand[i] for i in take]
    gaps["sel"] = float(min(cvals[i] for i in take))
    gaps["rsel"] = float(min(cvals[i] / (2.0 * scale[cand[i]]) for i in take))
    for k, l in sel:
        X[k, l] = 0 if logits[k, l, 0] >= logits[k, l, 1] else 1
    return {"selected": sel, "gaps": gaps}
