"""Small test-side helpers: toy codes built from their definitions, brute force."""
from __future__ import annotations

import itertools

import numpy as np

from paper_2305_05286_amd.workload.codes import Code


def code_from_dense(H: np.ndarray, name: str = "toy") -> Code:
    H = np.asarray(H, dtype=np.uint8)
    M, N = H.shape
    row_ptr = np.zeros(M + 1, dtype=np.int32)
    cols = []
    for i in range(M):
        c = np.nonzero(H[i])[0]
        cols.extend(c.tolist())
        row_ptr[i + 1] = len(cols)
    return Code(name=name, M=M, N=N, row_ptr=row_ptr, col_idx=np.asarray(cols, np.int32),
                K=0, info_pos=np.zeros(0, np.int32), encoder="gf2")


def hamming_H(m: int) -> np.ndarray:
    """Parity-check matrix of the (2^m - 1, 2^m - 1 - m) Hamming code: its columns
    are all nonzero binary vectors of length m."""
    n = 2 ** m - 1
    H = np.zeros((m, n), dtype=np.uint8)
    for j in range(n):
        v = j + 1
        for i in range(m):
            H[i, j] = (v >> i) & 1
    return H


def random_tree_H(n_target: int, seed: int) -> np.ndarray:
    """Random cycle-free Tanner graph: each new check joins one existing variable
    and 1..3 new variables."""
    rng = np.random.default_rng(seed)
    rows = []
    nvar = 1
    while nvar < n_target:
        anchor = int(rng.integers(0, nvar))
        k = int(min(rng.integers(1, 4), n_target - nvar))
        rows.append([anchor] + list(range(nvar, nvar + k)))
        nvar += k
    H = np.zeros((len(rows), nvar), dtype=np.uint8)
    for i, r in enumerate(rows):
        H[i, r] = 1
    return H


def all_codewords(H: np.ndarray) -> np.ndarray:
    M, N = H.shape
    assert N <= 20
    words = np.array(list(itertools.product([0, 1], repeat=N)), dtype=np.uint8)
    syn = (words.astype(np.int64) @ H.T.astype(np.int64)) & 1
    return words[(syn == 0).all(axis=1)]


def brute_force_map_llr(H: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Exact bitwise posterior LLR: log sum_{c_v=0} e^{W(c)} - log sum_{c_v=1} e^{W(c)},
    W(c) = sum_u (1 - 2 c_u) L_u / 2, over the codewords c of H."""
    C = all_codewords(H)
    W = ((1.0 - 2.0 * C) * L[None, :]).sum(axis=1) / 2.0
    out = np.empty(H.shape[1])
    for v in range(H.shape[1]):
        w0 = W[C[:, v] == 0]
        w1 = W[C[:, v] == 1]
        out[v] = np.logaddexp.reduce(w0) - np.logaddexp.reduce(w1)
    return out


def brute_force_max_marginal(H: np.ndarray, L: np.ndarray) -> np.ndarray:
    """max_{c_v=0} W(c) - max_{c_v=1} W(c) over the codewords of H."""
    C = all_codewords(H)
    W = ((1.0 - 2.0 * C) * L[None, :]).sum(axis=1) / 2.0
    return np.array([W[C[:, v] == 0].max() - W[C[:, v] == 1].max() for v in range(H.shape[1])])


def ml_codeword(H: np.ndarray, L: np.ndarray) -> np.ndarray:
    C = all_codewords(H)
    corr = ((1.0 - 2.0 * C) * L[None, :]).sum(axis=1)
    return C[int(np.argmax(corr))]


def syndrome(code: Code, bits: np.ndarray) -> np.ndarray:
    """H x^T mod 2 per frame, shape [B, M]."""
    bits = np.asarray(bits, dtype=np.uint8)
    rows = np.repeat(np.arange(code.M), np.diff(code.row_ptr))
    B = bits.shape[0]
    out = np.zeros((B, code.M), dtype=np.uint8)
    g = bits[:, code.col_idx]
    for i in range(code.M):
        out[:, i] = np.bitwise_xor.reduce(g[:, code.row_ptr[i]:code.row_ptr[i + 1]], axis=1)
    return out
