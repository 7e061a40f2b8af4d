"""GPU parity of the slot-wise AMP-MMSE detector (cider_amp_evidence, through
the C ABI) against the FP64 oracle: every evidence value of every slot,
within 1e-4 of max(1, |oracle|).  FP32 run through the same iterations in a
NumPy emulation stays within 2e-6 of FP64 on the workload's slots; the
tolerance leaves room for the kernel's different summation order and
hardware exp/log.
"""
import numpy as np
import pytest

import synth
from oracle.amp import amp_evidence_batch

from gpu_common import lib, rel_err, say, torch_cuda

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _run(y, rows, Q, rho, su2, iters):
    torch = torch_cuda()
    P = lib()
    S, n_s = y.shape[0], y.shape[1]
    yd = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).cuda()
    rd = torch.from_numpy(np.ascontiguousarray(rows, dtype=np.int32)).cuda()
    out = torch.full((max(S, 1), Q), float("nan"), dtype=torch.float32, device="cuda")
    P.cider_amp_evidence(yd, rd, S, n_s, Q, rho, su2, iters, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:S]


@pytest.mark.parametrize("ebn0", [2.0, 6.0])
def test_workload_slots_match_oracle(ebn0):
    sl = synth.make_amp_slots(frames=40, L=24, Q=64, n_s=24, K=2, payload_bits=48, ebn0_db=ebn0, seed=11)
    su2, rho = float(sl.p_sym[0]), 2 / 64
    say(f"AMP Q=64 n_s=24 K=2 Eb/N0={ebn0} dB, {sl.y.shape[0]} slots, 20 iterations")
    S = _run(sl.y, sl.rows, 64, rho, su2, 20)
    ref = amp_evidence_batch(sl.y, sl.rows, 64, rho, su2, 20)
    e = rel_err(S, ref)
    print(f"  max err {e:.2e}")
    assert np.all(np.isfinite(S)) and e <= TOL


@pytest.mark.parametrize("Q,n_s,iters,shared", [(64, 64, 20, False), (64, 1, 5, False), (2, 2, 3, False),
                                                (48, 24, 20, False), (64, 24, 0, True), (64, 24, 1, True),
                                                (37, 13, 7, False)])
def test_edge_shapes_match_oracle(Q, n_s, iters, shared):
    sl = synth.make_amp_slots(frames=3, L=7, Q=Q, n_s=n_s, K=2, payload_bits=12, ebn0_db=4.0, seed=Q + n_s,
                              shared_rows=shared)
    su2, rho = float(sl.p_sym[0]), min(0.5, 2 / Q)
    say(f"AMP edge Q={Q} n_s={n_s} iters={iters} shared_rows={shared}")
    S = _run(sl.y, sl.rows, Q, rho, su2, iters)
    ref = amp_evidence_batch(sl.y, sl.rows, Q, rho, su2, iters)
    assert rel_err(S, ref) <= TOL


def test_rows_are_taken_modulo_q():
    sl = synth.make_amp_slots(frames=2, L=5, Q=64, n_s=24, K=2, payload_bits=48, ebn0_db=4.0, seed=5)
    shifted = sl.rows + 64 * np.where(np.arange(24) % 2 == 0, 3, -2)[None, :]
    say("AMP rows outside [0, Q)")
    a = _run(sl.y, sl.rows, 64, 2 / 64, float(sl.p_sym[0]), 10)
    b = _run(sl.y, shifted.astype(np.int32), 64, 2 / 64, float(sl.p_sym[0]), 10)
    assert np.array_equal(a, b)


def test_no_slots_is_a_no_op():
    assert _run(np.zeros((0, 24, 2), np.float32), np.zeros((0, 24), np.int32), 64, 0.03, 2.0, 20).shape == (0, 64)


@pytest.mark.parametrize("Q", [64, 48])
def test_repeated_rows_match_oracle(Q):
    """Rows drawn with replacement: A has repeated rows (the Q = 64 FFT path
    sums the residual entries that land on the same row)."""
    rng = np.random.default_rng(21)
    S, n_s = 30, 24
    rows = rng.integers(0, Q, size=(S, n_s)).astype(np.int32)
    y = rng.standard_normal((S, n_s, 2)).astype(np.float32) * 2.0
    say(f"AMP repeated rows Q={Q}")
    got = _run(y, rows, Q, 2 / Q, 3.0, 20)
    ref = amp_evidence_batch(y, rows, Q, 2 / Q, 3.0, 20)
    assert rel_err(got, ref) <= TOL
