"""The CIDER decode over a Q-ary LDPC code, Q = 2^m (the paper's main
setting: GF(64) codes, K users, evidence from the slot-wise detector), in
float64.  Test infrastructure only: the HIP library never imports it.

It follows the paper's refinement loop (method section) with the Q-symbol
forms of its pieces:
  embedding   Z[k,l] = E[X[k,l]] + P[l] + gamma u, E with Q + 1 rows (row Q
              is the mask token; Appendix, CIDER architecture)
  Module A    Lbar = Z W^T over the Q symbols, responsibilities softmax over
              rows, e = sum_a r p_a v_a, gated blend (method section,
              Module A equations)
  layers      the binary path's blocks (denoiser.layer)
  projection  Lout = LN_f(Z) W^T
  Module B    per row and check, the exact extrinsic check message of the
              c2v rule of the Q-ary LDPC appendix -- the distribution of the
              other edges' weighted sum sum_i H[j,l'] x_l' read at H[j,l] a
              -- from per-site distributions of the projected logits, added
              to the logits as eta times its centred logarithm, summed over
              the site's checks (method section, check message and update)
  reveal      confidence max_a softmax(L / tau_t)_a at the annealed
              temperature tau_t (Appendix, confidence ranking and cosine
              schedule), argmax symbol, first-reveal on step 1
Readings (the text fixes none of these for the logit-bias form):
  * a masked site's distribution is softmax of its projected logits clipped
    to lam_max below their maximum; a revealed symbol x enters as
    exp(lam_max [a = x]) normalised -- at Q = 2 exactly the binary path's
    clipped log-likelihood ratios;
  * the message enters as eta (log m(a) - mean_a log m(a)): at Q = 2 this is
    the binary +-eta b / 2 split;
  * sites are ranked by the uncertainty u = log sum_a exp((L_a - max L) / tau_t)
    = -log(max probability), ascending (the same order, without the
    saturation of the probability to 1), ties to the smaller flat index
    k n + l; first-reveal keeps each slot's row of smallest u (ties to the
    smaller k); the argmax ties to the smaller symbol;
  * no remasking (the paper's K = 2 scales run without it).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np
from scipy.special import logsumexp

from .denoiser import gelu, layer, layer_norm, sigmoid, softmax
from .gf import gf_inv, gf_mul
from .schedule import _boundary_gap, cosine_targets, linear_targets, tau_schedule


def embed_q(X: np.ndarray, gamma: float, w: Dict[str, np.ndarray]) -> np.ndarray:
    K, n = X.shape
    return w["E"][X] + w["P"][:n][None, :, :] + gamma * w["u"][None, None, :]


def module_a_q(Z: np.ndarray, p: np.ndarray, w: Dict[str, np.ndarray], tau: float = 1.0):
    """Z [K][n][d], p [n][Q] -> (Z~, parts)."""
    lbar = Z @ w["W"].T                               # [K][n][Q]
    r = softmax(lbar / tau, axis=0)                   # over the rows k
    e = np.einsum("kla,la,ad->kld", r, p, w["v"])
    h = gelu(np.concatenate([Z, e], axis=-1) @ w["Wg1"].T + w["bg1"])
    g = sigmoid(h @ w["Wg2"].T + w["bg2"])
    return g * Z + (1.0 - g) * e, {"lbar": lbar, "r": r, "e": e, "g": g}


def site_dists(lbar: np.ndarray, X: np.ndarray, Q: int, lam_max: float) -> np.ndarray:
    """Per-site symbol distributions fed to the checks: [K][n][Q]."""
    z = lbar - lbar.max(axis=-1, keepdims=True)
    q = np.exp(np.maximum(z, -lam_max))
    q = q / q.sum(axis=-1, keepdims=True)
    onehot = np.full(Q, 1.0)
    for k in range(X.shape[0]):
        for l in range(X.shape[1]):
            x = int(X[k, l])
            if x < Q:
                v = onehot.copy()
                v[x] = math.exp(lam_max)
                q[k, l] = v / v.sum()
    return q


def xor_convolve(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Distribution of x ^ y for independent x ~ a, y ~ b: out[c] = sum_x a[x] b[x ^ c]
    (the sum over x as one matrix-vector product with the table b[x ^ c])."""
    idx = np.arange(a.shape[0])
    return a @ np.asarray(b)[np.bitwise_xor.outer(idx, idx)]


def check_message(q_in: List[np.ndarray], alphas_in: List[int], alpha_out: int, m: int) -> np.ndarray:
    """m(a) proportional to Pr(sum_i alpha_i x_i = alpha_out a) with x_i ~ q_i,
    formed by convolving the permuted distributions y_i = alpha_i x_i in the
    given order; normalised."""
    Q = 1 << m
    s = np.zeros(Q)
    s[0] = 1.0                                        # empty sum is 0
    for q, al in zip(q_in, alphas_in):
        y = np.zeros(Q)
        for x in range(Q):
            y[gf_mul(al, x, m)] += q[x]
        s = xor_convolve(s, y)
    out = np.array([s[gf_mul(alpha_out, a, m)] for a in range(Q)])
    return out / out.sum()


def module_b_q(lbar: np.ndarray, X: np.ndarray, code, eta: float = 1.0, lam_max: float = 20.0) -> np.ndarray:
    """Logits after the Q-ary Module B: [K][n][Q]."""
    K, n, Q = lbar.shape
    m = int(round(math.log2(Q)))
    q = site_dists(lbar, X, Q, lam_max)
    msg = {}
    for j in range(code.m):
        e0, e1 = int(code.row_ptr[j]), int(code.row_ptr[j + 1])
        nb = [int(v) for v in code.col_idx[e0:e1]]
        al = [int(v) for v in code.coef[e0:e1]]
        for o in range(len(nb)):
            others = [i for i in range(len(nb)) if i != o]          # ascending, target excluded
            for k in range(K):
                mm = check_message([q[k, nb[i]] for i in others], [al[i] for i in others], al[o], m)
                lm = np.log(mm)
                msg[(k, j, nb[o])] = lm - lm.mean()
    out = np.array(lbar, dtype=np.float64, copy=True)
    for l in range(n):
        for j in code.var_idx[code.var_ptr[l]:code.var_ptr[l + 1]]:   # ascending checks
            for k in range(K):
                out[k, l] += eta * msg[(k, int(j), l)]
    return out


def denoise_q(X: np.ndarray, p: np.ndarray, code, w: Dict[str, np.ndarray], n_layers: int, heads: int,
              gamma: float, tau: float = 1.0, eta: float = 1.0, lam_max: float = 20.0) -> Dict[str, np.ndarray]:
    Z = embed_q(X, gamma, w)
    Z, parts = module_a_q(Z, p, w, tau)
    for l in range(n_layers):
        Z = layer(Z, w, l, heads)
    lbar = layer_norm(Z, w["lnf_g"], w["lnf_b"]) @ w["W"].T
    logits = module_b_q(lbar, X, code, eta, lam_max)
    return {"lbar": lbar, "logits": logits, "z": Z, "module_a": parts}


def uncertainty(logits: np.ndarray, tau: float) -> np.ndarray:
    """u = log sum_a exp((L_a - max_a L) / tau) = -log max_a softmax(L / tau)_a."""
    z = (logits - logits.max(axis=-1, keepdims=True)) / tau
    return logsumexp(z, axis=-1)


def reveal_q(X: np.ndarray, logits: np.ndarray, r: int, first: bool, tau: float, Q: int) -> Dict:
    """Reveal up to r masked sites (grid value Q = mask) in place."""
    K, n = X.shape
    u = uncertainty(logits, tau)
    scale = np.maximum(1.0, np.abs(logits).max(axis=-1))
    masked = X == Q
    inf = float("inf")
    gaps = {"cut": inf, "sel": inf, "slot": inf, "ties": 0}
    if first:
        cand = []
        for l in range(n):
            ks = np.nonzero(masked[:, l])[0]
            if ks.size == 0:
                continue
            o = ks[np.lexsort((ks, u[ks, l]))]         # smallest u, ties to the smaller k
            cand.append((int(o[0]), l))
            if o.size > 1:
                g, _, tied = _boundary_gap(-u[o, l], scale[o, l], 0)
                gaps["slot"] = min(gaps["slot"], g)
                gaps["ties"] += int(tied)
    else:
        ks, ls = np.nonzero(masked)
        cand = list(zip(ks.tolist(), ls.tolist()))
    if not cand or r <= 0:
        return {"selected": [], "gaps": gaps}
    uv = np.array([u[k, l] for k, l in cand])
    flat = np.array([k * n + l for k, l in cand])
    order = np.lexsort((flat, uv))
    take = order[:min(r, len(cand))]
    if len(cand) > r:
        g, _, tied = _boundary_gap(-uv[order], np.array([scale[cand[i]] for i in order]), r - 1)
        gaps["cut"] = g
        gaps["ties"] += int(tied)
    sel = [cand[i] for i in take]
    for k, l in sel:
        srt = np.sort(logits[k, l])[::-1]
        gaps["sel"] = min(gaps["sel"], float(srt[0] - srt[1]))
        X[k, l] = int(np.argmax(logits[k, l]))        # first maximum: smaller symbol
    return {"selected": sel, "gaps": gaps}


@dataclass
class DecodeResultQ:
    X: np.ndarray
    final_logits: np.ndarray
    row_valid: np.ndarray
    steps: List[Dict] = field(default_factory=list)


def gf_syndrome_ok(X: np.ndarray, code) -> np.ndarray:
    """1 where row k of X satisfies every check of the Q-ary code."""
    m = int(code.q_bits)
    ok = np.ones(X.shape[0], dtype=np.uint8)
    for k in range(X.shape[0]):
        for j in range(code.m):
            s = 0
            for e in range(int(code.row_ptr[j]), int(code.row_ptr[j + 1])):
                s ^= gf_mul(int(code.coef[e]), int(X[k, int(code.col_idx[e])]), m)
            if s:
                ok[k] = 0
    return ok


def decode_grid_q(K: int, n: int, Q: int, code, den: Callable, T: int, schedule: str = "linear",
                  first_reveal: bool = True, tau_max: float = 1.0, tau_min: float = 1.0,
                  keep: bool = False) -> DecodeResultQ:
    """The refinement loop with the Q-ary reveal: T steps from the all-mask
    grid, then the final gamma = 0 pass; the output is the held-fixed grid."""
    X = np.full((K, n), Q, dtype=np.uint8)
    N = K * n
    R = linear_targets(N, T) if schedule == "linear" else cosine_targets(N, T)
    done = 0
    steps = []
    for t in range(1, T + 1):
        r = R[t - 1] - done
        if schedule == "cosine":
            r = max(1, r)
            if t == T:
                r = N - done
        r = max(0, min(r, N - done))
        gamma = float((X == Q).sum()) / float(N)
        X_in = X.copy()
        out = den(X, gamma)
        logits = out["logits"] if isinstance(out, dict) else out
        tau_t = tau_schedule(t, T, tau_max, tau_min)
        info = reveal_q(X, logits, r, bool(first_reveal) and t == 1 and T > 1, tau_t, Q)
        done += len(info["selected"])
        rec = {"t": t, "r": r, "gamma": gamma, "tau": tau_t, "gaps": info["gaps"], "selected": info["selected"]}
        if keep:
            rec["X_in"] = X_in
            rec["logits"] = logits
        steps.append(rec)
    out = den(X, 0.0)
    fin = out["logits"] if isinstance(out, dict) else out
    return DecodeResultQ(X=X, final_logits=fin, row_valid=gf_syndrome_ok(X, code), steps=steps)


def decode_bin_q(S: np.ndarray, code, K: int, w: Dict[str, np.ndarray], n_layers: int, heads: int, T: int,
                 keep: bool = False, **kw) -> DecodeResultQ:
    """Decode one bin from its evidence S [n][Q] (p = softmax_a S per slot)."""
    Q = S.shape[1]
    p = softmax(np.asarray(S, dtype=np.float64), axis=1)

    def den(X, gamma):
        return denoise_q(X, p, code, w, n_layers, heads, gamma)

    return decode_grid_q(K, code.n, Q, code, den, T, keep=keep, **kw)


# ---------------------------------------------------------------------------
# Brute force on tiny codes (test pins): the codebook by exhaustive search,
# joint MAP over unordered pairs, and the genie denoiser.  The channel of
# these pins is the orthogonal-signature special case of the slot channel
# (n_s = Q, A = I): y_l = e_{x1,l} + e_{x2,l} + N(0, sigma2 I) in R^Q.

def codebook_q(code) -> np.ndarray:
    """Every c in GF(2^m)^n with H c = 0, by exhaustive search: [M][n]."""
    m, n, Q = int(code.q_bits), code.n, 1 << int(code.q_bits)
    T = np.array([[gf_mul(a, b, m) for b in range(Q)] for a in range(Q)])
    grid = np.stack(np.meshgrid(*[np.arange(Q)] * n, indexing="ij"), axis=-1).reshape(-1, n)
    ok = np.ones(grid.shape[0], bool)
    for j in range(code.m):
        s = np.zeros(grid.shape[0], dtype=np.int64)
        for e in range(int(code.row_ptr[j]), int(code.row_ptr[j + 1])):
            s ^= T[int(code.coef[e]), grid[:, int(code.col_idx[e])]]
        ok &= s == 0
    return grid[ok].astype(np.uint8)


def pair_loglik_q(C: np.ndarray, y: np.ndarray, sigma2: float) -> np.ndarray:
    """L[i, j] = log prod_l N(y_l; e_{C_i,l} + e_{C_j,l}, sigma2 I) up to a constant."""
    M, n = C.shape
    Q = y.shape[1]
    tab = np.zeros((n, Q, Q))
    for l in range(n):
        for a in range(Q):
            for b in range(Q):
                s = np.zeros(Q)
                s[a] += 1.0
                s[b] += 1.0
                tab[l, a, b] = -float(((y[l] - s) ** 2).sum()) / (2.0 * sigma2)
    L = np.zeros((M, M))
    for l in range(n):
        L += tab[l][C[:, l][:, None], C[:, l][None, :]]
    return L


def map_pair_q(C: np.ndarray, y: np.ndarray, sigma2: float):
    L = pair_loglik_q(C, y, sigma2)
    M = C.shape[0]
    iu = np.triu_indices(M, k=1)
    vals = L[iu]
    best = int(np.argmax(vals))
    return (int(iu[0][best]), int(iu[1][best])), float(np.exp(vals[best] - logsumexp(vals)))


def genie_denoiser_q(C: np.ndarray, y: np.ndarray, sigma2: float):
    """den(X, gamma) -> log marginals [2][n][Q] of each row's symbols given the
    revealed tokens of X (mask = Q), over ordered pairs of distinct codewords."""
    L = pair_loglik_q(C, y, sigma2)
    M, n = C.shape
    Q = y.shape[1]
    L[np.arange(M), np.arange(M)] = -np.inf

    def den(X, gamma):
        ok0 = np.ones(M, bool)
        ok1 = np.ones(M, bool)
        for l in range(n):
            if X[0, l] != Q:
                ok0 &= C[:, l] == X[0, l]
            if X[1, l] != Q:
                ok1 &= C[:, l] == X[1, l]
        Lc = np.where(ok0[:, None] & ok1[None, :], L, -np.inf)
        r0 = logsumexp(Lc, axis=1)                     # [M]: row 0 is codeword i
        r1 = logsumexp(Lc, axis=0)                     # [M]: row 1 is codeword j
        out = np.full((2, n, Q), -np.inf)
        for l in range(n):
            for a in range(Q):
                sel = C[:, l] == a
                if sel.any():
                    out[0, l, a] = logsumexp(r0[sel])
                    out[1, l, a] = logsumexp(r1[sel])
        out = out - logsumexp(out, axis=2, keepdims=True)
        return np.maximum(out, -1e3)
    return den
