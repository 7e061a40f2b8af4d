"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and rejects bad arguments before touching a device."""
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cider.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cider_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2605_26580_amd as P
    L = P.abi.lib()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert sorted(P.abi.EXPORTS) == names


def test_opts_defaults():
    import paper_2605_26580_amd as P
    o = P.cider_opts_default()
    assert o.precision == P.CIDER_BF16 and o.schedule == P.CIDER_SCHED_LINEAR and o.first_reveal == 1
    assert o.remask == 0 and o.remask_max_rounds == 2 and abs(o.remask_thr - 0.9) < 1e-7
    assert o.tau == 1.0 and o.eta == 1.0 and o.lam_max == 20.0 and abs(o.lam_min - 1e-6) < 1e-12
    assert o.tau_max == 1.0 and o.tau_min == 1.0 and o.fused_blocks == 1 and o.autotune == 1
    assert not o.qhead and o.qhead_hidden == 0 and o.remask_stages == 3
    assert np.allclose(list(o.remask_phi), [0.96, 0.90, 0.85, 0.0])
    o = P.cider_opts_default(remask_phi=(0.5, 0.25))
    assert np.allclose(list(o.remask_phi), [0.5, 0.25, 0.0, 0.0])


@pytest.mark.parametrize("L,d,h,q", [(2, 64, 4, 2), (4, 128, 8, 2), (6, 256, 8, 2), (8, 384, 12, 2), (4, 128, 4, 64),
                                     (1, 64, 4, 8)])
def test_blob_size_agrees_with_generator(L, d, h, q):
    import paper_2605_26580_amd as P
    cfg = synth.ModelCfg(L, d, h, q=q)
    assert P.cider_weights_blob_floats(P.make_cfg(L, d, h, q=q)) == synth.weights.blob_size(cfg)


def test_bad_q_rejected_on_cpu():
    import paper_2605_26580_amd as P
    assert P.cider_weights_blob_floats(P.make_cfg(2, 64, 4, q=3)) == 0
    assert P.cider_weights_blob_floats(P.make_cfg(2, 64, 4, q=128)) == 0
    with pytest.raises(P.CiderError) as e:                                      # zero coefficient
        P.CodeQ(4, 1, np.array([0, 3]), np.array([0, 1, 2]), np.array([1, 0, 5]), 3)
    assert e.value.status == P.abi.CIDER_EINVAL
    with pytest.raises(P.CiderError):                                           # degree above 16
        P.CodeQ(32, 1, np.array([0, 17]), np.arange(17), np.ones(17), 3)


def test_bad_model_and_code_rejected_on_cpu():
    import paper_2605_26580_amd as P
    assert P.cider_weights_blob_floats(P.make_cfg(2, 96, 4)) == 0          # d not a multiple of 64
    with pytest.raises(P.CiderError) as e:
        P.Weights(P.make_cfg(2, 64, 5), np.zeros(10, np.float32))
    assert e.value.status == P.abi.CIDER_EINVAL
    with pytest.raises(P.CiderError):
        P.Code(8, 2, np.array([0, 3, 9]), np.array([0, 1, 2, 3, 4, 5, 6, 7, 9]))   # index out of range
    with pytest.raises(P.CiderError):
        P.Code(8, 1, np.array([0, 3]), np.array([2, 1, 3]))                      # not ascending
    assert "invalid" in P.cider_strerror(P.abi.CIDER_EINVAL)



def test_amp_arguments_rejected_on_cpu():
    """cider_amp_evidence validates before any device work (no GPU needed)."""
    import paper_2605_26580_amd as P
    bad = [dict(n_s=0), dict(n_s=65), dict(Q=1), dict(Q=65), dict(iters=-1), dict(rho=0.0), dict(rho=1.0),
           dict(su2=0.0), dict(slots=-1)]
    for kw in bad:
        args = dict(slots=4, n_s=24, Q=64, rho=0.03, su2=2.0, iters=20)
        args.update(kw)
        rc = P.abi.lib().cider_amp_evidence(None, None, args["slots"], args["n_s"], args["Q"], args["rho"],
                                            args["su2"], args["iters"], None, None)
        assert rc == -1, kw
    # valid sizes but missing buffers
    assert P.abi.lib().cider_amp_evidence(None, None, 4, 24, 64, 0.03, 2.0, 20, None, None) == -1


def test_gf64_check_update_arguments_rejected_on_cpu():
    """cider_gf64_check_update validates sizes and buffers before any device work."""
    import paper_2605_26580_amd as P
    L = P.abi.lib()
    assert L.cider_gf64_check_update(None, None, None, -1, 0, None, None) == -1
    assert L.cider_gf64_check_update(None, None, None, 0, -1, None, None) == -1
    assert L.cider_gf64_check_update(None, None, None, 1 << 31, 10, None, None) == -1
    assert L.cider_gf64_check_update(None, None, None, 4, 12, None, None) == -1      # null buffers
    assert L.cider_gf64_check_update(None, None, None, 0, 0, None, None) == 0        # nothing to do
