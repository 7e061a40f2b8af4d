"""The five synthetic workloads the decoder is exercised on.

c1  K=2, n=32   (3,6)-LDPC, Eb/N0 4 dB, L=2 d=64 h=4, T=8,  16 bins, FP32
c2  K=4, n=128, Eb/N0 {2,4,6} dB, L=4 d=128 h=8, T=16, 256 bins, BF16 vs FP32
c3  K=8, n=256, Eb/N0 5 dB, L=6 d=256 h=8, T=32, 512 bins, remasking on
c4  ragged: 4096 bins, K~U{2..8}, n~U{64,128,256,512}, Eb/N0~U[2,6], L=6 d=256 h=8, T=32
c5  served: Poisson arrivals, K~U{2..16}, n~U{128..1024}, L=8 d=384 h=12, T=32, remasking on
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Optional, Sequence, Tuple

from .weights import ModelCfg


@dataclass(frozen=True)
class Workload:
    name: str
    K: int
    n: int
    model: ModelCfg
    T: int
    batch: int
    ebn0_db: Tuple[float, ...]
    code_seed: int
    weight_seed: int
    bin_seed: int
    remask: bool = False
    remask_thr: float = 0.9
    remask_max_rounds: int = 2
    ragged_K: Optional[Tuple[int, ...]] = None
    ragged_n: Optional[Tuple[int, ...]] = None
    ebn0_range: Optional[Tuple[float, float]] = None
    binning: Optional[Tuple[int, int, int]] = None   # (K_tot, zeta, K_max): batch counts frames


WORKLOADS: Dict[str, Workload] = {
    "c1": Workload("c1", K=2, n=32, model=ModelCfg(2, 64, 4), T=8, batch=16,
                   ebn0_db=(4.0,), code_seed=1032, weight_seed=11, bin_seed=101),
    "c2": Workload("c2", K=4, n=128, model=ModelCfg(4, 128, 8), T=16, batch=256,
                   ebn0_db=(2.0, 4.0, 6.0), code_seed=1128, weight_seed=12, bin_seed=102),
    "c3": Workload("c3", K=8, n=256, model=ModelCfg(6, 256, 8), T=32, batch=512,
                   ebn0_db=(5.0,), code_seed=1256, weight_seed=13, bin_seed=103,
                   remask=True),
    "c4": Workload("c4", K=8, n=512, model=ModelCfg(6, 256, 8), T=32, batch=4096,
                   ebn0_db=(4.0,), code_seed=1000, weight_seed=13, bin_seed=104,
                   ragged_K=tuple(range(2, 9)), ragged_n=(64, 128, 256, 512),
                   ebn0_range=(2.0, 6.0)),
    "c5": Workload("c5", K=16, n=1024, model=ModelCfg(8, 384, 12), T=32, batch=0,
                   ebn0_db=(4.0,), code_seed=1000, weight_seed=15, bin_seed=105,
                   remask=True, ragged_K=tuple(range(2, 17)), ragged_n=(128, 256, 512, 1024),
                   ebn0_range=(2.0, 6.0)),
    # stochastic-binning traffic: frames of K_tot = 100 users over zeta = 25 preamble
    # bins, bank up to K_max = 8 (overflow bins erased); c4's model, n = 256
    "protocol": Workload("protocol", K=8, n=256, model=ModelCfg(6, 256, 8), T=32, batch=160,
                         ebn0_db=(4.0,), code_seed=1256, weight_seed=13, bin_seed=106,
                         ragged_K=tuple(range(1, 9)), ragged_n=(256,), ebn0_range=(2.0, 6.0),
                         binning=(100, 25, 8)),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]
