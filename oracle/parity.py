"""Module B in its binary logit-bias form.

The paper's Module B sends extrinsic check-to-slot messages along the
Tanner graph of H and fuses their sum back into each site (method section,
check-message and update equations).  For a binary code every coefficient
is 1 (the coefficient action is the identity) and the exact extrinsic
message of a parity check is the Q=2 case of the classical check update
(Appendix, LDPC details, check-to-variable rule).  In log-likelihood-ratio
form, with lambda = logit(bit 0) - logit(bit 1):

    m[j -> l] = prod_{l' in N(j), l' != l} sgn(lambda[l'])
                * phi( sum_{l' in N(j), l' != l} phi(|lambda[l']|) ),
    phi(x)    = log((e^x + 1) / (e^x - 1)) = log1p(2 / expm1(x)),

which equals 2 atanh(prod tanh(lambda[l'] / 2)).  The bias on slot l is
b[l] = sum_{j in N_chk(l)} m[j -> l]; it is added as +eta*b/2 to the bit-0
logit and -eta*b/2 to the bit-1 logit, so the logit difference moves by
eta*b.  Sites already revealed enter with lambda = +-lam_max; masked sites
use their (clipped) predicted logit difference; |lambda| is floored at
lam_min inside phi.  Each message is formed by explicit exclusion of the
target edge (never "total minus own"), summing in ascending slot order;
b sums messages in ascending check order.  sgn(0) is taken as +1.
"""
from __future__ import annotations

import numpy as np

MASK = 2


def phi(x):
    x = np.asarray(x, dtype=np.float64)
    return np.log1p(2.0 / np.expm1(x))


def site_llr(lbar: np.ndarray, X: np.ndarray, lam_max: float) -> np.ndarray:
    """lambda[k, l] fed to the checks: clipped predicted LLR, or +-lam_max if revealed."""
    lam = np.clip(lbar[..., 0] - lbar[..., 1], -lam_max, lam_max)
    lam = np.where(X == 0, lam_max, lam)
    lam = np.where(X == 1, -lam_max, lam)
    return lam


def check_messages(lam: np.ndarray, code, lam_min: float):
    """All check-to-slot messages.  lam [K][n]; returns list of (j, l, msg[K])."""
    out = []
    for j in range(code.m):
        nbrs = [int(v) for v in code.col_idx[code.row_ptr[j]:code.row_ptr[j + 1]]]
        for l in nbrs:
            sgn = np.ones(lam.shape[0])
            acc = np.zeros(lam.shape[0])
            for l2 in nbrs:                       # ascending, target edge excluded
                if l2 == l:
                    continue
                sgn = sgn * np.where(lam[:, l2] >= 0.0, 1.0, -1.0)
                acc = acc + phi(np.maximum(np.abs(lam[:, l2]), lam_min))
            out.append((j, l, sgn * phi(acc)))
    return out


def parity_bias(lam: np.ndarray, code, lam_min: float) -> np.ndarray:
    """b[k, l] = sum over checks j containing l (ascending j) of m[j -> l]."""
    msgs = {(j, l): m for j, l, m in check_messages(lam, code, lam_min)}
    b = np.zeros_like(lam)
    for l in range(code.n):
        for j in code.var_idx[code.var_ptr[l]:code.var_ptr[l + 1]]:
            b[:, l] = b[:, l] + msgs[(int(j), l)]
    return b


def module_b(lbar: np.ndarray, X: np.ndarray, code, eta: float = 1.0, lam_max: float = 20.0,
             lam_min: float = 1e-6) -> np.ndarray:
    """Logits after Module B: lbar [K][n][2] -> [K][n][2]."""
    lam = site_llr(lbar, X, lam_max)
    b = parity_bias(lam, code, lam_min)
    out = np.array(lbar, dtype=np.float64, copy=True)
    out[..., 0] += 0.5 * eta * b
    out[..., 1] -= 0.5 * eta * b
    return out


def syndrome(x_rows: np.ndarray, code) -> np.ndarray:
    """H x mod 2 for each row of x_rows [K][n] (symbols 0/1); returns [K][m]."""
    return (np.asarray(x_rows, dtype=np.int64) @ code.H.T.astype(np.int64)) % 2
