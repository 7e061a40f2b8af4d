"""Binary regular LDPC codes drawn from the configuration model.

The paper's codes are sparse parity-check codes whose Tanner-graph
connectivity is sampled at random (Appendix, LDPC details, "Construction of
H").  The workloads here use binary codes with column weight 3 and row
weight 6 (rate 1/2).  A draw is rejected when a check would hold the same
variable twice or when H is rank deficient over GF(2), so that exactly
k = n - n/2 information bits remain.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class LdpcCode:
    n: int                 # code length (variables / slots)
    m: int                 # number of checks
    H: np.ndarray          # uint8 [m][n] dense parity-check matrix
    row_ptr: np.ndarray    # int32 [m+1]  check -> variables (CSR, ascending)
    col_idx: np.ndarray    # int32 [nnz]
    var_ptr: np.ndarray    # int32 [n+1]  variable -> checks (transpose, ascending)
    var_idx: np.ndarray    # int32 [nnz]
    G: np.ndarray          # uint8 [k][n] generator (basis of the null space of H)
    seed: int

    @property
    def k(self) -> int:
        return int(self.G.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def encode(self, info: np.ndarray) -> np.ndarray:
        """info uint8 [..., k] -> codeword uint8 [..., n] (c = u G mod 2)."""
        info = np.asarray(info, dtype=np.int64)
        return (info @ self.G.astype(np.int64) % 2).astype(np.uint8)


def rank_gf2(M: np.ndarray) -> int:
    """Rank over GF(2) by Gaussian elimination on a copy."""
    A = (np.asarray(M, dtype=np.uint8) & 1).copy()
    rows, cols = A.shape
    r = 0
    for c in range(cols):
        piv = np.nonzero(A[r:, c])[0]
        if piv.size == 0:
            continue
        p = r + int(piv[0])
        if p != r:
            A[[r, p]] = A[[p, r]]
        hit = np.nonzero(A[:, c])[0]
        hit = hit[hit != r]
        A[hit] ^= A[r]
        r += 1
        if r == rows:
            break
    return r


def nullspace_gf2(H: np.ndarray) -> np.ndarray:
    """Basis (rows) of {c : H c = 0 mod 2} via reduced row echelon form."""
    A = (np.asarray(H, dtype=np.uint8) & 1).copy()
    m, n = A.shape
    pivots = []
    r = 0
    for c in range(n):
        if r == m:
            break
        piv = np.nonzero(A[r:, c])[0]
        if piv.size == 0:
            continue
        p = r + int(piv[0])
        if p != r:
            A[[r, p]] = A[[p, r]]
        hit = np.nonzero(A[:, c])[0]
        hit = hit[hit != r]
        A[hit] ^= A[r]
        pivots.append(c)
        r += 1
    free = [c for c in range(n) if c not in set(pivots)]
    basis = np.zeros((len(free), n), dtype=np.uint8)
    for i, f in enumerate(free):
        basis[i, f] = 1
        for row, pc in enumerate(pivots):
            if A[row, f]:
                basis[i, pc] = 1
    return basis


def _csr(H: np.ndarray):
    m, n = H.shape
    row_ptr = np.zeros(m + 1, dtype=np.int32)
    cols = []
    for j in range(m):
        c = np.nonzero(H[j])[0]
        cols.append(c)
        row_ptr[j + 1] = row_ptr[j] + c.size
    col_idx = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    var_ptr = np.zeros(n + 1, dtype=np.int32)
    rows = []
    for v in range(n):
        r = np.nonzero(H[:, v])[0]
        rows.append(r)
        var_ptr[v + 1] = var_ptr[v] + r.size
    var_idx = np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32)
    return row_ptr, col_idx, var_ptr, var_idx


def regular_ldpc(n: int, dv: int = 3, dc: int = 6, seed: int = 0, max_draws: int = 20000) -> LdpcCode:
    """Seeded (dv, dc)-regular binary LDPC code of length n (configuration model).

    The dv*n variable sockets are permuted at random and dealt to m = dv*n/dc
    checks in groups of dc.  Draws with a repeated variable inside one check, or
    with rank_GF2(H) < m, are rejected and redrawn from the same generator.
    """
    if (dv * n) % dc != 0:
        raise ValueError("dv*n must be a multiple of dc")
    m = dv * n // dc
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    sockets = np.repeat(np.arange(n, dtype=np.int64), dv)
    for _ in range(max_draws):
        perm = rng.permutation(sockets).reshape(m, dc)
        srt = np.sort(perm, axis=1)
        if np.any(srt[:, 1:] == srt[:, :-1]):
            continue
        H = np.zeros((m, n), dtype=np.uint8)
        H[np.repeat(np.arange(m), dc), perm.reshape(-1)] = 1
        if rank_gf2(H) < m:
            continue
        G = nullspace_gf2(H)
        row_ptr, col_idx, var_ptr, var_idx = _csr(H)
        return LdpcCode(n=n, m=m, H=H, row_ptr=row_ptr, col_idx=col_idx,
                        var_ptr=var_ptr, var_idx=var_idx, G=G, seed=seed)
    raise RuntimeError(f"no valid ({dv},{dc}) code of length {n} in {max_draws} draws")
