"""FP64 oracle of the slot-wise AMP-MMSE detector (Appendix, slot-wise
AMP-MMSE detector; sensing-matrix construction).  Test infrastructure only:
the HIP library never imports or calls it.

For one slot: Y = A U + eps in C^{n_s}, A the partial-DFT matrix (n_s rows R
of the Q-point DFT, scaled by 1/sqrt(n_s), so every column has unit norm),
U with the Bernoulli-Gaussian prior (1 - rho) delta_0 + rho CN(0, su2).

  scalar channel   r = u + w, w ~ CN(0, nu)
  activity         p(r) = rho phi(r; nu + su2) / ((1 - rho) phi(r; nu) + rho phi(r; nu + su2))
  MMSE denoiser    eta(r) = p(r) su2 / (nu + su2) r
  AMP iteration    R = U_hat + A^H Y_res,  U_hat' = eta(R; nu),
                   Y_res' = Y - A U_hat' + Y_res / n_s * sum_a eta'(R_a; nu)
  evidence         S_a = log p(R_a; nu) after I iterations

Readings where the text leaves a choice:
- nu^(i) = ||Y_res^(i)||^2 / n_s (the estimate the text offers);
- eta' is the complex analogue of the derivative used by complex AMP: for a
  denoiser eta(r) = c(|r|^2) r it is the mean of d Re(eta)/d Re(r) and
  d Im(eta)/d Im(r), which equals c(t) + t c'(t), t = |r|^2;
- the final pseudo-observation is R^(I) = U_hat^(I) + A^H Y_res^(I), with
  nu^(I) from Y_res^(I).
"""
from __future__ import annotations

import numpy as np


def partial_dft(Q: int, rows) -> np.ndarray:
    """A[j, a] = exp(-2 pi i R[j] a / Q) / sqrt(n_s), complex128 [n_s][Q]."""
    rows = np.asarray(rows, dtype=np.int64)
    a = np.arange(Q, dtype=np.int64)
    # the exponent reduced mod Q first, so that large products stay exact
    k = (rows[:, None] * a[None, :]) % Q
    return np.exp(-2j * np.pi * k / Q) / np.sqrt(len(rows))


def log_cn_pdf(r, v: float) -> np.ndarray:
    """log phi(r; 0, v) of the circular complex Gaussian: -log(pi v) - |r|^2 / v."""
    return -np.log(np.pi * v) - np.abs(r) ** 2 / v


def log_activity(r, nu: float, rho: float, su2: float) -> np.ndarray:
    """log p(r) = log Pr(U != 0 | R = r), from the two mixture densities."""
    l1 = np.log(rho) + log_cn_pdf(r, nu + su2)
    l0 = np.log1p(-rho) + log_cn_pdf(r, nu)
    return l1 - np.logaddexp(l0, l1)


def eta_mmse(r, nu: float, rho: float, su2: float) -> np.ndarray:
    """E[U | R = r] under the Bernoulli-Gaussian prior."""
    return np.exp(log_activity(r, nu, rho, su2)) * (su2 / (nu + su2)) * r


def eta_prime(r, nu: float, rho: float, su2: float) -> np.ndarray:
    """c(t) + t c'(t) for eta(r) = c(|r|^2) r (the complex divergence)."""
    p = np.exp(log_activity(r, nu, rho, su2))
    s = su2 / (nu + su2)
    delta = 1.0 / nu - 1.0 / (nu + su2)          # d/dt of the log-odds of activity
    t = np.abs(r) ** 2
    return s * p + t * s * p * (1.0 - p) * delta


def amp_core(Y, A, rho: float, su2: float, iters: int):
    """AMP-MMSE for Y = A U + noise with any sensing matrix A [n_s][Q]:
    returns (R^(I) [Q], nu^(I), U_hat^(I) [Q])."""
    Y = np.asarray(Y, dtype=np.complex128)
    n_s, Q = A.shape
    U = np.zeros(Q, dtype=np.complex128)
    res = Y.copy()
    for _ in range(iters):
        nu = float(np.sum(np.abs(res) ** 2) / n_s)
        R = U + A.conj().T @ res
        U_new = eta_mmse(R, nu, rho, su2)
        onsager = res / n_s * float(np.sum(eta_prime(R, nu, rho, su2)))
        res = Y - A @ U_new + onsager
        U = U_new
    nu = float(np.sum(np.abs(res) ** 2) / n_s)
    R = U + A.conj().T @ res
    return R, nu, U


def amp_slot(y, rows, Q: int, rho: float, su2: float, iters: int):
    """AMP-MMSE on one slot with its partial-DFT matrix: (R^(I) [Q], nu^(I))."""
    y = np.asarray(y, dtype=np.float64)
    Y = y[:, 0] + 1j * y[:, 1] if y.ndim == 2 else y.astype(np.complex128)
    R, nu, _ = amp_core(Y, partial_dft(Q, rows), rho, su2, iters)
    return R, nu


def amp_evidence(y, rows, Q: int, rho: float, su2: float, iters: int) -> np.ndarray:
    """S[a] = log p(R^(I)_a; nu^(I)) for one slot, float64 [Q]."""
    R, nu = amp_slot(y, rows, Q, rho, su2, iters)
    return log_activity(R, nu, rho, su2)


def amp_evidence_batch(y, rows, Q: int, rho, su2, iters: int) -> np.ndarray:
    """Every slot of a batch: y [S][n_s][2], rows [S][n_s], rho / su2 scalars
    or per slot; returns float64 [S][Q]."""
    S = y.shape[0]
    rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), (S,))
    su2 = np.broadcast_to(np.asarray(su2, dtype=np.float64), (S,))
    return np.stack([amp_evidence(y[s], rows[s], Q, float(rho[s]), float(su2[s]), iters) for s in range(S)])
