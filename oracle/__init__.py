"""FP64 CPU oracle for the CIDER refinement path -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, deliberately unoptimised NumPy (float64)
statement of what the decoder computes, written from the paper.  It exists
to check the HIP library.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library never does, and the
two share no code (they meet only at the seeded inputs from ``synth``).

Modules
    evidence  -- per-slot evidence S and beliefs p (evidence interface)
    denoiser  -- embedding, Module A, the transformer layers, projection
    parity    -- Module B: soft parity messages fed back as a logit bias
    schedule  -- reveal-count schedules and the confidence-ranked reveal
    decode    -- the refinement loop, final pass and quality-guided remasking
    metrics   -- Hungarian-matched SER/CER and the grid -> message-set rule
    brute     -- brute-force joint MAP and the genie denoiser (tiny codes)
    amp       -- the slot-wise AMP-MMSE detector of the non-binary channel
    quality   -- the PRISM-style quality head and its row confidences
    protocol  -- stochastic binning: bin loads, overflow, frame-level errors
    gf        -- GF(2^m) arithmetic, Pi_alpha and the non-binary check message
    qary      -- the decode over a Q-ary LDPC code (Q-symbol Modules A and B, reveal)

Parity status: every function is pinned by tests under tests/ (closed forms,
brute force, library special cases, invariants) except the end-to-end
decode on random weights, whose free-running output has no value in the
paper to match; there the HIP library is compared with this oracle.
"""
from . import evidence, denoiser, parity, schedule, decode, metrics, brute, amp, quality, protocol, gf, qary  # noqa: F401
from .decode import DecodeOpts, decode_bin  # noqa: F401
