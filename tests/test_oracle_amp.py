"""Pins of the AMP-MMSE oracle (Appendix, slot-wise AMP-MMSE detector;
sensing-matrix construction) against what the mathematics fixes:
- the partial-DFT matrix against numpy's FFT and its orthogonality;
- the Bernoulli-Gaussian activity posterior and MMSE denoiser against
  two-dimensional quadrature of the prior times the likelihood;
- the sensitivity against finite differences of the denoiser;
- the iteration: with zero iterations R = A^H Y; on an i.i.d. Gaussian
  matrix (AMP's own setting) the pseudo-observation error has the variance
  nu the iteration estimates and the MSE reaches the state-evolution level,
  which a dropped Onsager term visibly misses;
- support recovery on an easy slot.
"""
import numpy as np
import pytest

from oracle import amp as O


def test_partial_dft_is_the_fft_rows_scaled():
    Q, rows = 64, np.array([0, 3, 7, 20, 33, 63])
    F = np.fft.fft(np.eye(Q))                    # F[k, n] = exp(-2 pi i k n / Q)
    A = O.partial_dft(Q, rows)
    np.testing.assert_allclose(A, F[rows] / np.sqrt(len(rows)), atol=1e-12)
    np.testing.assert_allclose(np.sum(np.abs(A) ** 2, axis=0), 1.0, atol=1e-12)
    np.testing.assert_allclose(A @ A.conj().T, Q / len(rows) * np.eye(len(rows)), atol=1e-12)


def _grid(half=9.0, n=601):
    x = np.linspace(-half, half, n)
    U = x[None, :] + 1j * x[:, None]
    return U, (x[1] - x[0]) ** 2


@pytest.mark.parametrize("r", [0.3 + 0.1j, -1.2 + 0.8j, 2.5 - 0.5j])
def test_activity_and_mmse_against_quadrature(r):
    nu, rho, su2 = 0.7, 0.2, 2.0
    U, dA = _grid()
    cn = lambda z, v: np.exp(-np.abs(z) ** 2 / v) / (np.pi * v)
    lik = cn(r - U, nu) * cn(U, su2)             # p(r | u) p(u | active)
    p_act = np.sum(lik) * dA                     # p(r | active) by quadrature
    num = rho * np.sum(U * lik) * dA             # rho * int u p(r|u) p(u) du
    den = (1 - rho) * cn(r, nu) + rho * p_act
    np.testing.assert_allclose(np.exp(O.log_activity(np.array([r]), nu, rho, su2))[0], rho * p_act / den,
                               rtol=1e-6)
    np.testing.assert_allclose(O.eta_mmse(np.array([r]), nu, rho, su2)[0], num / den, rtol=1e-6, atol=1e-9)


def test_sensitivity_is_the_complex_divergence():
    nu, rho, su2, h = 0.5, 0.1, 3.0, 1e-6
    r = np.array([0.2 + 0.3j, -1.5 + 0.4j, 2.0 - 2.2j, 0.01 - 0.02j])
    e = lambda z: O.eta_mmse(z, nu, rho, su2)
    d_re = (e(r + h).real - e(r - h).real) / (2 * h)
    d_im = (e(r + 1j * h).imag - e(r - 1j * h).imag) / (2 * h)
    np.testing.assert_allclose(O.eta_prime(r, nu, rho, su2), 0.5 * (d_re + d_im), rtol=1e-6)


def test_zero_iterations_is_the_backprojection():
    rng = np.random.default_rng(3)
    Q, rows = 64, np.sort(rng.choice(64, 24, replace=False))
    y = rng.standard_normal((24, 2))
    R, nu = O.amp_slot(y, rows, Q, 0.05, 4.0, 0)
    Y = y[:, 0] + 1j * y[:, 1]
    np.testing.assert_allclose(R, O.partial_dft(Q, rows).conj().T @ Y, atol=1e-12)
    assert abs(nu - np.sum(np.abs(Y) ** 2) / 24) < 1e-12


def _iid_problem(seed=1, Q=2000, n_s=1000, rho=0.1, su2=1.0, sig2=0.01):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((n_s, Q)) + 1j * rng.standard_normal((n_s, Q))) / np.sqrt(2 * n_s)
    act = rng.random(Q) < rho
    U = np.where(act, (rng.standard_normal(Q) + 1j * rng.standard_normal(Q)) * np.sqrt(su2 / 2), 0)
    Y = A @ U + (rng.standard_normal(n_s) + 1j * rng.standard_normal(n_s)) * np.sqrt(sig2 / 2)
    return A, U, Y, rho, su2, sig2


def _state_evolution_mse(rho, su2, sig2, delta, iters, rng):
    """Scalar recursion tau2 <- sig2 + mmse(tau2) / delta, mmse by Monte Carlo."""
    M = 400000
    act = rng.random(M) < rho
    U = np.where(act, (rng.standard_normal(M) + 1j * rng.standard_normal(M)) * np.sqrt(su2 / 2), 0)
    W = (rng.standard_normal(M) + 1j * rng.standard_normal(M)) / np.sqrt(2)
    tau2 = sig2 + rho * su2 / delta
    for _ in range(iters):
        mse = np.mean(np.abs(O.eta_mmse(U + np.sqrt(tau2) * W, tau2, rho, su2) - U) ** 2)
        tau2 = sig2 + mse / delta
    return mse


def test_iid_matrix_matches_state_evolution():
    A, U, Y, rho, su2, sig2 = _iid_problem()
    R, nu, Uh = O.amp_core(Y, A, rho, su2, 15)
    ratio = np.mean(np.abs(R - U) ** 2) / nu
    mse = np.mean(np.abs(Uh - U) ** 2)
    se = _state_evolution_mse(rho, su2, sig2, A.shape[0] / A.shape[1], 15, np.random.default_rng(9))
    assert 0.9 < ratio < 1.1, ratio
    assert mse < 1.5 * se, (mse, se)


def test_dropped_onsager_term_fails_the_state_evolution(monkeypatch):
    """A planted mistake (eta' = 0, so no Onsager correction) must not pass."""
    A, U, Y, rho, su2, sig2 = _iid_problem()
    monkeypatch.setattr(O, "eta_prime", lambda r, nu, rho, su2: np.zeros_like(np.abs(r)))
    R, nu, Uh = O.amp_core(Y, A, rho, su2, 15)
    se = _state_evolution_mse(rho, su2, sig2, A.shape[0] / A.shape[1], 15, np.random.default_rng(9))
    assert np.mean(np.abs(Uh - U) ** 2) > 5 * se


def test_easy_slot_support_recovered():
    rng = np.random.default_rng(5)
    Q, n_s = 64, 48
    rows = np.sort(rng.choice(Q, n_s, replace=False))
    U = np.zeros(Q)
    U[[7, 40]] = 6.0
    A = O.partial_dft(Q, rows)
    Y = A @ U + (rng.standard_normal(n_s) + 1j * rng.standard_normal(n_s)) * np.sqrt(0.5)
    S = O.amp_evidence(np.stack([Y.real, Y.imag], -1), rows, Q, 2 / 64, 36.0, 20)
    assert np.all(S[[7, 40]] > -1e-3)
    assert set(np.argsort(S)[-2:]) == {7, 40}
    assert np.all(np.delete(S, [7, 40]) < -2.0)     # activity below 0.14 elsewhere


def test_slot_generator_statistics():
    """The channel the inputs come from: K picks per slot, Y - A U ~ CN(0, 1)."""
    import synth
    sl = synth.make_amp_slots(frames=200, L=24, Q=64, n_s=24, K=2, payload_bits=48, ebn0_db=[2.0, 6.0], seed=7)
    assert np.all(sl.counts.sum(axis=1) == 2)
    A = np.stack([O.partial_dft(64, r) for r in sl.rows[:500]])
    Y = sl.y[:500, :, 0] + 1j * sl.y[:500, :, 1]
    E = Y - np.einsum("sja,sa->sj", A, np.sqrt(sl.p_sym[:500, None]) * sl.counts[:500])
    assert abs(np.mean(np.abs(E) ** 2) - 1.0) < 0.03
    assert abs(sl.p_sym[0] - 48 * 10 ** 0.2 / 24) < 1e-12
    assert np.all(np.diff(np.sort(sl.rows, axis=1), axis=1) > 0)   # distinct rows
