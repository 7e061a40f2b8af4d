"""GPU checks of the protocol-level wrapper (Appendix, protocol-level scaling
by stochastic binning): frames of K_tot users spread over zeta preamble bins,
every decodable bin of several frames decoded in one packed call.

- each decoded bin equals the same bin decoded alone, bit for bit, so the
  per-bin parity of the decoder carries over to the frame;
- row-valid flags equal H x = 0 (mod 2) recomputed from the decoded grid;
- the bins above K_max are erased and no others, and the frame's user
  errors (oracle count over the decoded grids) are at least its overflow users.
"""
import numpy as np
import pytest

import synth
from oracle import protocol as Pr

from gpu_common import code_handle, code_of, lib, prec_id, say, torch_cuda, weights_handle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,d,h", [("fp32", 64, 4), ("bf16", 128, 8)])
def test_frames_decode_as_bins_alone(prec, d, h):
    torch = torch_cuda()
    P = lib()
    K_tot, zeta, K_max, n, T = 40, 8, 8, 64, 8
    cfg = synth.ModelCfg(2, d, h, n_max=64)
    wh, _ = weights_handle(cfg, seed=31 + d)
    code = code_of(n, 1000 + n)
    ch = code_handle(code)
    frames = synth.make_protocol_frames(code, 4, K_tot, zeta, K_max, (2.0, 6.0), seed=21)
    say(f"protocol frames {prec}: 4 frames, K_tot={K_tot}, zeta={zeta}, K_max={K_max}, n={n}, d={d}")
    dev = torch.device("cuda", 0)
    desc = [{"loads": fr.loads, "payload": {chi: (torch.from_numpy(b.y).to(dev), b.sigma2) for chi, b in fr.bins}}
            for fr in frames]
    opts = P.cider_opts_default(precision=prec_id(prec), use_graph=1)
    res = P.decode_frames(desc, ch, n, wh, T, K_max, opts)
    torch.cuda.synchronize()
    H = np.zeros((code.m, code.n), dtype=np.int64)
    for j in range(code.m):
        H[j, code.col_idx[code.row_ptr[j]:code.row_ptr[j + 1]]] = 1
    seen_over = 0
    for fi, (fr, r) in enumerate(zip(frames, res)):
        assert sorted(r["erased"]) == sorted(fr.overflow.tolist())
        assert sorted(r["decoded"]) == sorted(chi for chi, _ in fr.bins)
        seen_over += len(r["erased"])
        grids = {chi: g.cpu().numpy() for chi, (g, _) in r["decoded"].items()}
        for chi, b in fr.bins:
            X = grids[chi]
            V = r["decoded"][chi][1].cpu().numpy()
            assert X.shape == (b.K, n) and X.max() <= 1
            assert np.array_equal(V, ((X.astype(np.int64) @ H.T) % 2 == 0).all(axis=1).astype(np.uint8))
            alone = torch.full((b.K, n), 9, dtype=torch.uint8, device=dev)
            P.cider_decode(desc[fi]["payload"][chi][0], b.sigma2, ch, b.K, n, wh, T, alone,
                           P.cider_opts_default(precision=prec_id(prec)))
            torch.cuda.synchronize()
            assert np.array_equal(alone.cpu().numpy(), X), f"bin {chi} (K={b.K}): frame batch and alone differ"
        sent = {chi: b.codewords for chi, b in fr.bins}
        err = Pr.frame_user_errors(fr.loads, K_max, sent, grids)
        over_users = int(fr.loads[fr.loads > K_max].sum())
        assert over_users <= err <= K_tot
    print(f"  {sum(len(f.bins) for f in frames)} bins decoded, {seen_over} overflow bins erased")
