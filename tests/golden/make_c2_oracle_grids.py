"""Writes c2_oracle_grids.npz: the FP64 oracle's decoded grids for 3072
bins of the c2 workload (K = 4 users, (3,6)-regular binary LDPC n = 128,
Eb/N0 cycling 2/4/6 dB, denoiser L = 4, d = 128, 8 heads, seeded weights,
T = 16, linear schedule, hybrid first-reveal, no remasking), with each
bin's decision gaps.

Only ``oracle`` and the seeded generators in ``synth`` are called.  The gaps
are how far each integer decision of the refinement loop sits from a tie in
float64 (refinement loop and confidence-ranked reveal, method section): the
reveal cut (r-th minus (r+1)-th candidate margin), the argmax of each
revealed site (its margin) and the first-reveal row choice (best minus
second margin of a slot).  An exact zero is a structural tie -- identical
user rows, which carry bit-identical logits in any precision -- and is
counted apart (zero_ties); the gap of such a decision is measured past the
tied group, to the nearest distinct value.  min_rel_gap puts each nonzero gap against
the logits it is made of (a margin difference of two sites over 4 max(1, |L|)
of both sites, an argmax margin over 2 max(1, |L|) of its site): a GPU decode
whose logits are within that relative error, max |dL| / max(1, |L|), of the
oracle's takes every decision the same way.

    python tests/golden/make_c2_oracle_grids.py [--bins 3072] [--workers 8]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle.decode import DecodeOpts, decode_bin  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_oracle_grids.npz")
_ctx = {}


def _setup(nbins: int):
    wl = synth.workload("c2")
    cfg = wl.model
    w = synth.unpack_weights(synth.make_weights(cfg, wl.weight_seed), cfg)
    code = synth.regular_ldpc(wl.n, seed=wl.code_seed)
    bins = synth.make_bins(code, wl.K, nbins, wl.ebn0_db, wl.bin_seed)
    _ctx.update(wl=wl, cfg=cfg, w=w, code=code, bins=bins)


def _one(b: int):
    wl, cfg, bins = _ctx["wl"], _ctx["cfg"], _ctx["bins"]
    r = decode_bin(bins.y[b], float(bins.sigma2[b]), _ctx["code"], wl.K, _ctx["w"], cfg.n_layers, cfg.heads,
                   wl.T, DecodeOpts())
    g = {key: [s["gaps"][key] for s in r.steps] for key in ("cut", "sel", "slot")}
    nz = [v for vals in g.values() for v in vals if 0.0 < v < np.inf]
    ties = sum(s["gaps"]["ties"] for s in r.steps)
    mins = [min([v for v in g[key] if v > 0.0], default=np.inf) for key in ("cut", "sel", "slot")]
    rel = min(s["gaps"][key] for s in r.steps for key in ("rcut", "rsel", "rslot"))
    return r.X, min(nz, default=np.inf), mins, ties, rel


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--bins", type=int, default=3072)
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    from multiprocessing import get_context
    t0 = time.time()
    with get_context("fork").Pool(a.workers, initializer=_setup, initargs=(a.bins,)) as pool:
        res = pool.map(_one, range(a.bins), chunksize=4)
    _setup(a.bins)
    X = np.stack([r[0] for r in res]).astype(np.uint8)
    np.savez_compressed(
        OUT, X_packed=np.packbits(X, axis=-1), shape=np.array(X.shape, dtype=np.int64),
        min_gap=np.array([r[1] for r in res]), min_cut=np.array([r[2][0] for r in res]),
        min_sel=np.array([r[2][1] for r in res]), min_slot=np.array([r[2][2] for r in res]),
        zero_ties=np.array([r[3] for r in res], dtype=np.int32),
        min_rel_gap=np.array([r[4] for r in res]),
        y_sum=np.array([float(np.sum(_ctx["bins"].y, dtype=np.float64))]))
    print(f"wrote {OUT}: {a.bins} bins in {time.time() - t0:.0f} s on {a.workers} workers")


if __name__ == "__main__":
    main()
