"""Seeded LDPC code construction and encoders (workload inputs only).

This module builds the parity-check matrices the decoders run on and encodes
random information words into codewords.  It holds none of the decoding
arithmetic: it is shared, as an input generator, by the tests, the benchmark
and the oracle checks.

Conventions
-----------
* A code is an M x N binary parity-check matrix H stored as CSR
  (``row_ptr`` int32[M+1], ``col_idx`` int32[E], ascending within each row).
  Check-node c_i is row i, variable-node v is column v (paper Sec. II).
* Quasi-cyclic (QC) codes carry a base matrix of shifts ``shifts[mb][nb]``:
  -1 is a Z x Z zero block, s in [0, Z) is the identity cyclically shifted so
  that row k of the block has its one in column (k + s) mod Z.
* Codewords satisfy H c^T = 0 over GF(2).  Every encoder here is systematic:
  ``info_pos`` lists the codeword positions that carry the information bits.
"""
from __future__ import annotations

import json
from dataclasses import dataclass, field
from pathlib import Path
from typing import Optional

import numpy as np

__all__ = [
    "Code",
    "qc_to_csr",
    "socket_regular_code",
    "qc_pattern_dualdiag",
    "qc_pattern_staircase",
    "draw_qc_shifts",
    "make_qc_code",
    "load_code",
    "save_code",
    "encode",
    "gf2_rank",
    "has_4cycle",
]


@dataclass
class Code:
    """A binary LDPC code: CSR parity-check matrix plus encoder metadata."""

    name: str
    M: int
    N: int
    row_ptr: np.ndarray  # int32[M+1]
    col_idx: np.ndarray  # int32[E]
    K: int
    info_pos: np.ndarray  # int32[K]; codeword positions of the info bits
    encoder: str  # "qc_dualdiag" | "qc_staircase" | "gf2"
    seed: int = 0
    Z: int = 0
    shifts: Optional[np.ndarray] = None  # int32[mb][nb] for QC codes
    meta: dict = field(default_factory=dict)
    # GF(2) systematic generator data for encoder == "gf2" (built lazily)
    _gf2: Optional[tuple] = None

    @property
    def E(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def rate(self) -> float:
        return self.K / self.N

    @property
    def is_qc(self) -> bool:
        return self.shifts is not None

    def dense(self) -> np.ndarray:
        H = np.zeros((self.M, self.N), dtype=np.uint8)
        for i in range(self.M):
            H[i, self.col_idx[self.row_ptr[i]:self.row_ptr[i + 1]]] = 1
        return H

    def row_degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def col_degrees(self) -> np.ndarray:
        return np.bincount(self.col_idx, minlength=self.N)


# ---------------------------------------------------------------------------
# CSR helpers
# ---------------------------------------------------------------------------

def _csr_from_rows(rows: list[list[int]]) -> tuple[np.ndarray, np.ndarray]:
    row_ptr = np.zeros(len(rows) + 1, dtype=np.int32)
    cols: list[int] = []
    for i, r in enumerate(rows):
        rs = sorted(r)
        cols.extend(rs)
        row_ptr[i + 1] = len(cols)
    return row_ptr, np.asarray(cols, dtype=np.int32)


def qc_to_csr(shifts: np.ndarray, Z: int) -> tuple[np.ndarray, np.ndarray]:
    """Lift a QC base matrix to CSR.  Rows of block-row r are r*Z + k."""
    mb, nb = shifts.shape
    rows = []
    for r in range(mb):
        for k in range(Z):
            rows.append([b * Z + (k + int(shifts[r, b])) % Z
                         for b in range(nb) if shifts[r, b] >= 0])
    return _csr_from_rows(rows)


def has_4cycle(row_ptr: np.ndarray, col_idx: np.ndarray) -> bool:
    """True if two distinct rows share two or more columns."""
    M = len(row_ptr) - 1
    seen: dict[tuple[int, int], int] = {}
    for i in range(M):
        cols = col_idx[row_ptr[i]:row_ptr[i + 1]]
        for a in range(len(cols)):
            for b in range(a + 1, len(cols)):
                key = (int(cols[a]), int(cols[b]))
                if key in seen and seen[key] != i:
                    return True
                seen[key] = i
    return False


# ---------------------------------------------------------------------------
# GF(2) linear algebra (bit-packed rows)
# ---------------------------------------------------------------------------

def _pack_rows(H: np.ndarray) -> np.ndarray:
    return np.packbits(H.astype(np.uint8), axis=1, bitorder="little")


def gf2_rank(H: np.ndarray) -> int:
    A = _pack_rows(H).copy()
    M, N = H.shape
    rank = 0
    for col in range(N):
        byte, bit = divmod(col, 8)
        rows = np.nonzero((A[rank:, byte] >> bit) & 1)[0]
        if rows.size == 0:
            continue
        p = rank + rows[0]
        if p != rank:
            A[[rank, p]] = A[[p, rank]]
        hit = np.nonzero((A[:, byte] >> bit) & 1)[0]
        hit = hit[hit != rank]
        A[hit] ^= A[rank]
        rank += 1
        if rank == M:
            break
    return rank


def _gf2_systematic(H: np.ndarray):
    """Reduced row echelon form of H over GF(2) (rows packed 64 bits to a word).

    Returns (pivot_cols, info_cols, P) where, for a codeword c,
    c[pivot_cols] = P @ c[info_cols] (mod 2), P shape (rank, K).
    """
    M, N = H.shape
    W = (N + 63) // 64
    A = np.zeros((M, W * 8), dtype=np.uint8)
    A[:, :(N + 7) // 8] = _pack_rows(H)
    A = A.view("<u8")
    pivots = []
    r = 0
    for col in range(N):
        word, bit = divmod(col, 64)
        b = np.uint64(bit)
        rows = np.nonzero((A[r:, word] >> b) & np.uint64(1))[0]
        if rows.size == 0:
            continue
        p = r + rows[0]
        if p != r:
            A[[r, p]] = A[[p, r]]
        hit = np.nonzero((A[:, word] >> b) & np.uint64(1))[0]
        hit = hit[hit != r]
        A[hit] ^= A[r]
        pivots.append(col)
        r += 1
        if r == M:
            break
    pivots = np.asarray(pivots, dtype=np.int32)
    info = np.setdiff1d(np.arange(N, dtype=np.int32), pivots)
    R = np.unpackbits(A[:len(pivots)].view(np.uint8), axis=1, bitorder="little")[:, :N]
    P = R[:, info]
    return pivots, info, P


# ---------------------------------------------------------------------------
# Regular codes from random sockets (edge by edge, 4-cycles rejected)
# ---------------------------------------------------------------------------

def socket_regular_code(n: int, dv: int, dc: int, seed: int, *,
                        name: str = "", full_rank: bool = True,
                        max_attempts: int = 1000) -> Code:
    """(dv, dc)-regular code drawn from random edge sockets.

    Edges are placed one at a time: a variable socket is matched to a random
    free check socket, and a placement is rejected when it would create a
    double edge or a 4-cycle (two checks sharing two variables).  A dead end
    restarts the attempt; an attempt whose H is rank-deficient is also
    rejected when ``full_rank`` is set, so that K = N - M.
    """
    assert (n * dv) % dc == 0
    m = n * dv // dc
    ss = np.random.SeedSequence([seed, n, dv, dc])
    for attempt, child in enumerate(ss.spawn(max_attempts)):
        rng = np.random.default_rng(child)
        var_nb: list[set[int]] = [set() for _ in range(n)]
        chk_nb: list[set[int]] = [set() for _ in range(m)]
        free = np.full(m, dc, dtype=np.int64)
        order = np.repeat(np.arange(n), dv)
        rng.shuffle(order)
        ok = True
        for v in order:
            cand = np.nonzero(free > 0)[0]
            rng.shuffle(cand)
            placed = False
            for c in cand:
                c = int(c)
                if c in var_nb[v]:
                    continue
                # 4-cycle: another check c2 of v already shares a variable with c
                if any(chk_nb[c] & chk_nb[c2] for c2 in var_nb[v]):
                    continue
                var_nb[v].add(c)
                chk_nb[c].add(int(v))
                free[c] -= 1
                placed = True
                break
            if not placed:
                ok = False
                break
        if not ok:
            continue
        rows = [sorted(chk_nb[c]) for c in range(m)]
        row_ptr, col_idx = _csr_from_rows(rows)
        code = Code(name=name or f"reg{dv}{dc}_n{n}", M=m, N=n, row_ptr=row_ptr,
                    col_idx=col_idx, K=0, info_pos=np.zeros(0, np.int32),
                    encoder="gf2", seed=seed, meta={"attempt": attempt})
        H = code.dense()
        rk = gf2_rank(H)
        if full_rank and rk != m:
            continue
        piv, info, P = _gf2_systematic(H)
        code.K = n - len(piv)
        code.info_pos = info.astype(np.int32)
        code._gf2 = (piv, info, P)
        return code
    raise RuntimeError("socket construction failed")


# ---------------------------------------------------------------------------
# QC codes
# ---------------------------------------------------------------------------

def qc_pattern_dualdiag(mb: int, info_weights: list[int], seed: int) -> np.ndarray:
    """Base pattern with a dual-diagonal parity part whose first column has weight 3.

    Layout: ``len(info_weights)`` information block-columns followed by mb
    parity block-columns.  Parity column 0 has ones in rows 0, mb//2 and
    mb-1; parity column j >= 1 has ones in rows j-1 and j.  Returns a
    0/1 array (mb, nb); the information rows are chosen at random with row
    degrees kept as even as possible.
    """
    kb = len(info_weights)
    nb = kb + mb
    pat = np.zeros((mb, nb), dtype=np.int8)
    pat[[0, mb // 2, mb - 1], kb] = 1
    for j in range(1, mb):
        pat[j - 1, kb + j] = 1
        pat[j, kb + j] = 1
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5a7]))
    order = np.argsort(-np.asarray(info_weights), kind="stable")
    for b in order:
        w = info_weights[b]
        deg = pat.sum(axis=1).astype(float) + rng.random(mb) * 0.5
        rows = np.argsort(deg, kind="stable")[:w]
        pat[rows, b] = 1
    return pat


def qc_pattern_staircase(mb: int, info_weights: list[int], seed: int) -> np.ndarray:
    """Base pattern with a strict lower dual-diagonal parity part.

    Parity column j has ones in rows j and j+1; the last parity column has a
    single one (row mb-1), so it is a degree-1 variable column.
    """
    kb = len(info_weights)
    nb = kb + mb
    pat = np.zeros((mb, nb), dtype=np.int8)
    for j in range(mb):
        pat[j, kb + j] = 1
        if j + 1 < mb:
            pat[j + 1, kb + j] = 1
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5c3]))
    order = np.argsort(-np.asarray(info_weights), kind="stable")
    for b in order:
        w = info_weights[b]
        deg = pat.sum(axis=1).astype(float) + rng.random(mb) * 0.5
        rows = np.argsort(deg, kind="stable")[:w]
        pat[rows, b] = 1
    return pat


def _base_4cycle_ok(sh: np.ndarray, Z: int, r: int, b: int) -> bool:
    """No lifted 4-cycle through base entry (r, b) with the already set shifts."""
    mb, nb = sh.shape
    s = sh[r, b]
    for r2 in range(mb):
        if r2 == r or sh[r2, b] < 0:
            continue
        for b2 in range(nb):
            if b2 == b or sh[r, b2] < 0 or sh[r2, b2] < 0:
                continue
            if (s - sh[r, b2] + sh[r2, b2] - sh[r2, b]) % Z == 0:
                return False
    return True


def draw_qc_shifts(pattern: np.ndarray, Z: int, seed: int, fixed: Optional[dict] = None,
                   max_tries: int = 2000) -> np.ndarray:
    """Draw circulant shifts U[0, Z) for a base pattern, rejecting base 4-cycles.

    ``fixed`` maps (r, b) -> shift for entries whose shift the encoder needs.
    Entries are filled column by column; a shift creating a lifted 4-cycle
    with the shifts already set is redrawn.
    """
    mb, nb = pattern.shape
    rng = np.random.default_rng(np.random.SeedSequence([seed, Z, 0xc1c]))
    for _ in range(50):
        sh = np.full((mb, nb), -1, dtype=np.int64)
        if fixed:
            for (r, b), s in fixed.items():
                sh[r, b] = s
        ok = True
        for b in range(nb):
            for r in range(mb):
                if pattern[r, b] == 0 or sh[r, b] >= 0:
                    continue
                for _t in range(max_tries):
                    sh[r, b] = rng.integers(0, Z)
                    if _base_4cycle_ok(sh, Z, r, b):
                        break
                else:
                    ok = False
                    break
            if not ok:
                break
        if ok:
            # fixed entries must also be free of 4-cycles with the drawn ones
            if all(_base_4cycle_ok(sh, Z, r, b) for r in range(mb) for b in range(nb) if sh[r, b] >= 0):
                return sh.astype(np.int32)
    raise RuntimeError("could not draw 4-cycle-free shifts")


def make_qc_code(name: str, pattern: np.ndarray, Z: int, seed: int, kind: str) -> Code:
    """QC code from a base pattern; ``kind`` selects the parity structure/encoder."""
    mb, nb = pattern.shape
    kb = nb - mb
    fixed = {}
    if kind == "qc_dualdiag":
        sigma = int(np.random.default_rng(np.random.SeedSequence([seed, 0xd1a])).integers(1, Z))
        fixed[(0, kb)] = sigma
        fixed[(mb // 2, kb)] = 0
        fixed[(mb - 1, kb)] = sigma
        for j in range(1, mb):
            fixed[(j - 1, kb + j)] = 0
            fixed[(j, kb + j)] = 0
    elif kind == "qc_staircase":
        for j in range(mb):
            fixed[(j, kb + j)] = 0
            if j + 1 < mb:
                fixed[(j + 1, kb + j)] = 0
    elif kind != "gf2":
        raise ValueError(kind)
    shifts = draw_qc_shifts(pattern, Z, seed, fixed)
    row_ptr, col_idx = qc_to_csr(shifts, Z)
    code = Code(name=name, M=mb * Z, N=nb * Z, row_ptr=row_ptr, col_idx=col_idx,
                K=kb * Z, info_pos=np.arange(kb * Z, dtype=np.int32), encoder=kind,
                seed=seed, Z=Z, shifts=shifts)
    if kind == "gf2":
        piv, info, P = _gf2_systematic(code.dense())
        code.K = code.N - len(piv)
        code.info_pos = info.astype(np.int32)
        code._gf2 = (piv, info, P)
    return code


# ---------------------------------------------------------------------------
# Encoders
# ---------------------------------------------------------------------------

def _roll_blocks(x: np.ndarray, s: int) -> np.ndarray:
    """Multiply Z-blocks by a shifted identity: out[k] = x[(k + s) mod Z]."""
    return np.roll(x, -s, axis=-1)


def _qc_lambda(code: Code, info: np.ndarray) -> np.ndarray:
    """lam[r] = sum over info block-columns b of P^{s_rb} u_b, shape (B, mb, Z)."""
    sh = code.shifts
    mb, nb = sh.shape
    kb = nb - mb
    Z = code.Z
    B = info.shape[0]
    u = info.reshape(B, kb, Z)
    lam = np.zeros((B, mb, Z), dtype=np.uint8)
    for r in range(mb):
        for b in range(kb):
            if sh[r, b] >= 0:
                lam[:, r] ^= _roll_blocks(u[:, b], int(sh[r, b]))
    return lam


def encode(code: Code, info: np.ndarray) -> np.ndarray:
    """Encode info words (B, K) uint8 into codewords (B, N) uint8."""
    info = np.asarray(info, dtype=np.uint8)
    B = info.shape[0]
    if code.encoder == "gf2":
        if code._gf2 is None:
            code._gf2 = _gf2_systematic(code.dense())
        piv, inf, P = code._gf2
        c = np.zeros((B, code.N), dtype=np.uint8)
        c[:, inf] = info
        # parity = P @ info (mod 2), via float matmul on 0/1 values
        par = (info.astype(np.float32) @ P.T.astype(np.float32))
        c[:, piv] = (np.rint(par).astype(np.int64) & 1).astype(np.uint8)
        return c
    sh = code.shifts
    mb, nb = sh.shape
    kb = nb - mb
    Z = code.Z
    lam = _qc_lambda(code, info)
    p = np.zeros((B, mb, Z), dtype=np.uint8)
    if code.encoder == "qc_dualdiag":
        sigma = int(sh[0, kb])
        p0 = np.bitwise_xor.reduce(lam, axis=1)
        p[:, 0] = p0
        sp0 = _roll_blocks(p0, sigma)
        p[:, 1] = lam[:, 0] ^ sp0
        for r in range(1, mb - 1):
            p[:, r + 1] = lam[:, r] ^ p[:, r] ^ (p0 if r == mb // 2 else 0)
    elif code.encoder == "qc_staircase":
        p[:, 0] = lam[:, 0]
        for r in range(1, mb):
            p[:, r] = lam[:, r] ^ p[:, r - 1]
    else:
        raise ValueError(code.encoder)
    return np.concatenate([info, p.reshape(B, mb * Z)], axis=1)


# ---------------------------------------------------------------------------
# Frozen artefacts
# ---------------------------------------------------------------------------

def save_code(code: Code, path: Path) -> None:
    d = {
        "name": code.name, "M": code.M, "N": code.N, "K": code.K,
        "encoder": code.encoder, "seed": code.seed, "Z": code.Z,
        "meta": code.meta,
    }
    if code.is_qc:
        d["shifts"] = code.shifts.tolist()
    else:
        d["row_ptr"] = code.row_ptr.tolist()
        d["col_idx"] = code.col_idx.tolist()
    Path(path).write_text(json.dumps(d, separators=(",", ":")) + "\n")


def load_code(path) -> Code:
    d = json.loads(Path(path).read_text())
    if "shifts" in d:
        shifts = np.asarray(d["shifts"], dtype=np.int32)
        row_ptr, col_idx = qc_to_csr(shifts, d["Z"])
        mb, nb = shifts.shape
        code = Code(name=d["name"], M=d["M"], N=d["N"], row_ptr=row_ptr, col_idx=col_idx,
                    K=d["K"], info_pos=np.arange(d["K"], dtype=np.int32),
                    encoder=d["encoder"], seed=d["seed"], Z=d["Z"], shifts=shifts,
                    meta=d.get("meta", {}))
        if code.encoder == "gf2":
            piv, info, P = _gf2_systematic(code.dense())
            code.info_pos = info.astype(np.int32)
            code._gf2 = (piv, info, P)
        return code
    row_ptr = np.asarray(d["row_ptr"], dtype=np.int32)
    col_idx = np.asarray(d["col_idx"], dtype=np.int32)
    code = Code(name=d["name"], M=d["M"], N=d["N"], row_ptr=row_ptr, col_idx=col_idx,
                K=d["K"], info_pos=np.zeros(0, np.int32), encoder=d["encoder"],
                seed=d["seed"], meta=d.get("meta", {}))
    piv, info, P = _gf2_systematic(code.dense())
    code.info_pos = info.astype(np.int32)
    code._gf2 = (piv, info, P)
    return code
