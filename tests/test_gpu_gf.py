"""GPU parity of the GF(64) check-node update (Q-ary LDPC code over GF(64);
FFT-BP's Walsh-Hadamard check update) against the FP64 oracle, through the
C ABI: every outgoing message of checks of degree 1..32 with random nonzero
coefficients and random input distributions, within the FP32 tolerance;
rows the kernel must skip (empty, or reaching past the edge count) are left
unwritten."""
import numpy as np
import pytest

from oracle import gf

from gpu_common import TOL, say, torch_cuda, lib

pytestmark = pytest.mark.gpu


def _random_check_set(degrees, seed):
    rng = np.random.default_rng(seed)
    row_ptr = np.concatenate([[0], np.cumsum(degrees)]).astype(np.int32)
    E = int(row_ptr[-1])
    coef = rng.integers(1, 64, E).astype(np.uint8)
    p = rng.random((E, 64)) ** 3
    p /= p.sum(axis=1, keepdims=True)
    return row_ptr, coef, p.astype(np.float32)


def test_gf64_check_update_matches_oracle():
    torch = torch_cuda()
    P = lib()
    degrees = [1, 2, 3, 4, 6, 8, 12, 32] * 2
    row_ptr, coef, p = _random_check_set(degrees, 5)
    E, C = len(coef), len(degrees)
    say(f"gf64 check update: {C} checks, {E} edges, degrees {sorted(set(degrees))}")
    out = torch.full((E, 64), -7.0, dtype=torch.float32, device="cuda")
    P.cider_gf64_check_update(torch.from_numpy(p).cuda(), torch.from_numpy(row_ptr).cuda(),
                              torch.from_numpy(coef).cuda(), C, E, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    p64 = p.astype(np.float64)
    worst = 0.0
    for j in range(C):
        e0, e1 = int(row_ptr[j]), int(row_ptr[j + 1])
        for o in range(e0, e1):
            others = [i for i in range(e0, e1) if i != o]
            ref = gf.check_message_wht([p64[i] for i in others], [int(coef[i]) for i in others], int(coef[o]))
            worst = max(worst, float(np.max(np.abs(got[o] - ref))))
    print(f"  max |gpu - oracle| = {worst:.2e}")
    assert worst <= TOL["fp32"]


def test_gf64_malformed_rows_left_unwritten():
    torch = torch_cuda()
    P = lib()
    _, coef, p = _random_check_set([4], 6)
    row_ptr = np.array([0, 2, 2, 5], dtype=np.int32)        # row 1 empty, row 2 reaches past 4 edges
    say("gf64 check update: malformed rows")
    out = torch.full((4, 64), -7.0, dtype=torch.float32, device="cuda")
    P.cider_gf64_check_update(torch.from_numpy(p).cuda(), torch.from_numpy(row_ptr).cuda(),
                              torch.from_numpy(coef).cuda(), 3, 4, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.all(got[2:] == -7.0)
    ref0 = gf.check_message_wht([p[1].astype(np.float64)], [int(coef[1])], int(coef[0]))
    assert np.max(np.abs(got[0] - ref0)) <= TOL["fp32"]
