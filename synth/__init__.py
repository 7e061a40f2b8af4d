"""Seeded synthetic inputs for the CIDER refinement path.

This module produces *data only*: binary regular LDPC parity-check matrices,
codewords, noisy BPSK aggregates and random denoiser weights.  It contains
none of the decoder's arithmetic (no evidence, no denoiser, no parity
messages, no reveal rule), so that the FP64 oracle and the HIP library can
both consume its outputs without sharing any of the method's code.

Every draw goes through ``numpy.random.Generator(PCG64(SeedSequence(seed)))``
so that the same seed yields the same bytes on every machine.
"""
from .code import LdpcCode, regular_ldpc, nullspace_gf2, rank_gf2
from .channel import ebn0_to_sigma2, make_bins, make_ragged_bins, BinBatch, RaggedBin
from .weights import ModelCfg, weight_layout, make_weights, unpack_weights, make_quality_head
from .configs import WORKLOADS, Workload, workload
from .amp import AmpSlots, make_amp_slots, p_sym_of
from .binning import ProtocolFrame, make_protocol_frames
from .qary import QaryCode, QaryFrames, qary_ldpc, make_qary_frames

__all__ = [
    "LdpcCode", "regular_ldpc", "nullspace_gf2", "rank_gf2",
    "ebn0_to_sigma2", "make_bins", "make_ragged_bins", "BinBatch", "RaggedBin",
    "ModelCfg", "weight_layout", "make_weights", "unpack_weights", "make_quality_head",
    "WORKLOADS", "Workload", "workload",
    "AmpSlots", "make_amp_slots", "p_sym_of",
    "ProtocolFrame", "make_protocol_frames",
    "QaryCode", "QaryFrames", "qary_ldpc", "make_qary_frames",
]
