"""Non-binary LDPC codes over GF(2^m) and the frames of the paper's Q-ary
benchmark (Appendix, Q-ary LDPC code; dataset scales over GF(64)).

A code is drawn like the binary ones: a random Tanner-graph connectivity
from the configuration model (column weight dv, row weight dc, no variable
twice in a check), then i.i.d. uniform nonzero coefficients on the edges,
redrawn until H has full row rank over GF(2^m), so that the code has
Q^(n - P) codewords.  Symbol index a is the field element whose coefficient
bits are a's bits (polynomial basis; x^3 + x + 1 for GF(8), x^6 + x + 1 for
GF(64)).

Data only: the field products here build and encode the code; none of the
decoder's arithmetic lives in this module.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .amp import AmpSlots, make_amp_slots

_POLY = {1: 0b11, 2: 0b111, 3: 0b1011, 4: 0b10011, 6: 0b1000011}


def _mul_table(m: int) -> np.ndarray:
    Q = 1 << m
    T = np.zeros((Q, Q), dtype=np.int64)
    for a in range(Q):
        for b in range(Q):
            x, y, r = a, b, 0
            while y:
                if y & 1:
                    r ^= x
                y >>= 1
                x <<= 1
                if x >> m:
                    x ^= _POLY[m]
            T[a, b] = r
    return T


@dataclass
class QaryCode:
    n: int                 # code length (slots)
    m: int                 # number of checks P
    q_bits: int            # Q = 2^q_bits
    row_ptr: np.ndarray    # int32 [m+1] check -> slots (CSR, ascending)
    col_idx: np.ndarray    # int32 [nnz]
    coef: np.ndarray       # uint8 [nnz] nonzero coefficient H[j, l] of each edge
    var_ptr: np.ndarray    # int32 [n+1] slot -> checks (ascending)
    var_idx: np.ndarray    # int32 [nnz]
    H: np.ndarray          # int64 [m][n] dense H over GF(2^q_bits)
    G: np.ndarray          # int64 [k][n] generator: rows span the null space of H
    seed: int

    @property
    def Q(self) -> int:
        return 1 << self.q_bits

    @property
    def k(self) -> int:
        return int(self.G.shape[0])

    def encode(self, info: np.ndarray) -> np.ndarray:
        """info [..., k] symbols -> codewords [..., n] (c = u G over GF(2^m))."""
        T = _mul_table(self.q_bits)
        info = np.asarray(info, dtype=np.int64)
        out = np.zeros(info.shape[:-1] + (self.n,), dtype=np.int64)
        for i in range(self.k):
            out ^= T[info[..., i][..., None], self.G[i]]
        return out.astype(np.uint8)


def _row_reduce(H: np.ndarray, T: np.ndarray, inv: np.ndarray):
    """Reduced row echelon form over GF(2^m); returns (R, pivot columns)."""
    R = H.copy()
    piv = []
    r = 0
    for col in range(R.shape[1]):
        rows = np.nonzero(R[r:, col])[0]
        if rows.size == 0:
            continue
        p = r + rows[0]
        R[[r, p]] = R[[p, r]]
        R[r] = T[inv[R[r, col]], R[r]]
        for i in range(R.shape[0]):
            if i != r and R[i, col]:
                R[i] ^= T[R[i, col], R[r]]
        piv.append(col)
        r += 1
        if r == R.shape[0]:
            break
    return R, piv


def qary_ldpc(n: int, q_bits: int, dv: int = 2, dc: int = 3, seed: int = 0, tries: int = 1000) -> QaryCode:
    """(dv, dc)-regular LDPC code of length n over GF(2^q_bits), full rank."""
    if (n * dv) % dc:
        raise ValueError("n * dv must be a multiple of dc")
    m = n * dv // dc
    Q = 1 << q_bits
    T = _mul_table(q_bits)
    inv = np.zeros(Q, dtype=np.int64)
    for a in range(1, Q):
        inv[a] = int(np.nonzero(T[a] == 1)[0][0])
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    for _ in range(tries):
        sockets = rng.permutation(np.repeat(np.arange(n), dv))
        checks = sockets.reshape(m, dc)
        if any(len(set(row.tolist())) != dc for row in checks):
            continue
        H = np.zeros((m, n), dtype=np.int64)
        for j in range(m):
            for l in checks[j]:
                H[j, l] = int(rng.integers(1, Q))
        R, piv = _row_reduce(H, T, inv)
        if len(piv) < m:
            continue
        free = [c for c in range(n) if c not in piv]
        G = np.zeros((len(free), n), dtype=np.int64)
        for i, f in enumerate(free):
            G[i, f] = 1
            for r, pc in enumerate(piv):
                G[i, pc] = R[r, f]          # x_pc = -sum R[r, f] x_f = sum (char 2)
        row_ptr = np.zeros(m + 1, dtype=np.int32)
        cols, coef = [], []
        for j in range(m):
            nz = np.nonzero(H[j])[0]
            cols += nz.tolist()
            coef += H[j, nz].tolist()
            row_ptr[j + 1] = len(cols)
        col_idx = np.array(cols, dtype=np.int32)
        var_ptr = np.zeros(n + 1, dtype=np.int32)
        vidx = []
        for l in range(n):
            js = np.nonzero(H[:, l])[0]
            vidx += js.tolist()
            var_ptr[l + 1] = len(vidx)
        return QaryCode(n=n, m=m, q_bits=q_bits, row_ptr=row_ptr, col_idx=col_idx,
                        coef=np.array(coef, dtype=np.uint8), var_ptr=var_ptr,
                        var_idx=np.array(vidx, dtype=np.int32), H=H, G=G, seed=seed)
    raise RuntimeError("no full-rank draw")


@dataclass
class QaryFrames:
    codewords: np.ndarray   # uint8 [F][K][n]
    slots: AmpSlots         # F * n slots, frame-major: slot l of frame f is f * n + l


def make_qary_frames(code: QaryCode, K: int, frames: int, n_s: int, ebn0_db, seed: int,
                     sigma2: float = 1.0) -> QaryFrames:
    """Frames of K users, each sending a codeword of K distinct uniform
    messages; slot l carries the K users' symbols of position l through the
    partial-DFT slot channel (make_amp_slots), with the payload of
    (n - P) q_bits bits per message setting the symbol power."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    Q = code.Q
    info = np.zeros((frames, K, code.k), dtype=np.int64)
    for f in range(frames):
        while True:
            u = rng.integers(0, Q, size=(K, code.k))
            if len({row.tobytes() for row in u}) == K:
                break
        info[f] = u
    cw = code.encode(info.reshape(frames * K, code.k)).reshape(frames, K, code.n)
    idx = cw.transpose(0, 2, 1).reshape(frames * code.n, K).astype(np.int64)
    slots = make_amp_slots(frames, code.n, Q, n_s, K, code.k * code.q_bits, ebn0_db, int(rng.integers(0, 2**31 - 1)),
                           sigma2=sigma2, idx=idx)
    return QaryFrames(codewords=cw, slots=slots)
