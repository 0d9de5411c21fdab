"""PEG-constructed LDPC codes with the paper's degree distributions (Sec. V).

The paper simulates rate-1/2 codes built by progressive edge growth: a (3,6)-
regular code and an irregular code with edge-perspective distributions

    lambda(x) = 0.45 x + 0.3708 x^2 + 0.0307 x^3 + 0.1485 x^11
    rho(x)    = 0.5467 x^4 + 0.4533 x^5

at lengths 2048 and 8192.  The matrices themselves are not published; these are
seeded constructions of the same kind.  Node degrees follow from lambda: the
fraction of variables of degree i is (lambda_i / i) / sum_j (lambda_j / j),
rounded to whole nodes by largest remainder.  Check degrees are concentrated
(every check gets floor(E/M) or ceil(E/M) edges), which for these lengths is
the two-degree rho above up to the rounding of lambda.

The construction itself is in ``peg.c`` (compiled with gcc on first use).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

from .codes import Code, _csr_from_rows, _gf2_systematic, gf2_rank

HERE = Path(__file__).resolve().parent
SRC = HERE / "peg.c"
LIB = HERE / "libpeg.so"

# edge-perspective variable degree distribution of the paper's irregular code
LAMBDA_IRREGULAR = {2: 0.45, 3: 0.3708, 4: 0.0307, 12: 0.1485}
RHO_IRREGULAR = {5: 0.5467, 6: 0.4533}

_lib = None


def build(force: bool = False) -> Path:
    """Compile peg.c with gcc (when missing, stale, or forced)."""
    if force or not LIB.exists() or LIB.stat().st_mtime < SRC.stat().st_mtime:
        tmp = LIB.with_suffix(f".so.tmp{os.getpid()}")
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-o", str(tmp), str(SRC)])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(str(LIB))
        lib.peg_build.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p]
        lib.peg_build.restype = ctypes.c_int
        _lib = lib
    return _lib


def node_degrees(n: int, lam: dict) -> np.ndarray:
    """Variable degrees (ascending) for n nodes from an edge-perspective lambda."""
    degs = sorted(lam)
    w = np.array([lam[d] / d for d in degs])
    exact = n * w / w.sum()
    cnt = np.floor(exact).astype(np.int64)
    short = n - int(cnt.sum())
    for i in np.argsort(-(exact - cnt), kind="stable")[:short]:
        cnt[i] += 1
    return np.repeat(np.array(degs, dtype=np.int32), cnt)


def peg_edges(vdeg: np.ndarray, M: int, seed: int) -> list[list[int]]:
    """Check lists per variable from the PEG construction (check degrees concentrated)."""
    vdeg = np.ascontiguousarray(vdeg, dtype=np.int32)
    E = int(vdeg.sum())
    lo, n_hi = E // M, E % M
    out = np.empty(E, dtype=np.int32)
    rc = _load().peg_build(len(vdeg), M, vdeg.ctypes.data, lo, n_hi, seed, out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"PEG construction failed ({rc})")
    off = np.concatenate([[0], np.cumsum(vdeg)])
    return [out[off[v]:off[v + 1]].tolist() for v in range(len(vdeg))]


def peg_code(name: str, n: int, lam: dict, seed: int, rate: float = 0.5) -> Code:
    """A PEG code of length n: variable degrees from lam, M = n (1 - rate) checks."""
    M = int(round(n * (1.0 - rate)))
    vdeg = node_degrees(n, lam)
    var_checks = peg_edges(vdeg, M, seed)
    rows: list[list[int]] = [[] for _ in range(M)]
    for v, cs in enumerate(var_checks):
        for c in cs:
            rows[c].append(v)
    row_ptr, col_idx = _csr_from_rows(rows)
    code = Code(name=name, M=M, N=n, row_ptr=row_ptr, col_idx=col_idx, K=0,
                info_pos=np.zeros(0, np.int32), encoder="gf2", seed=seed,
                meta={"construction": "peg", "lambda": {str(k): v for k, v in lam.items()}})
    piv, info, P = _gf2_systematic(code.dense())
    code.K = n - len(piv)
    code.info_pos = info.astype(np.int32)
    code._gf2 = (piv, info, P)
    return code


def girth(code: Code, limit: int = 12) -> int:
    """Length of the shortest cycle of the Tanner graph (a value above limit means none shorter).

    Breadth-first search from every variable over the bipartite graph; a
    non-tree edge met at depth d from a root closes a cycle of length <= 2 d.
    """
    N, M = code.N, code.M
    rp, ci = code.row_ptr, code.col_idx
    cols = [[] for _ in range(N)]
    for i in range(M):
        for e in range(rp[i], rp[i + 1]):
            cols[ci[e]].append(i)
    best = limit + 2
    for root in range(N):
        # node ids: variables 0..N-1, checks N..N+M-1
        dist = {root: 0}
        parent = {root: -1}
        frontier = [root]
        d = 0
        while frontier and 2 * (d + 1) < best:
            nxt = []
            for u in frontier:
                nbrs = [N + c for c in cols[u]] if u < N else list(ci[rp[u - N]:rp[u - N + 1]])
                for w in nbrs:
                    w = int(w)
                    if w == parent[u]:
                        continue
                    if w in dist:
                        best = min(best, dist[u] + dist[w] + 1)
                        continue
                    dist[w] = d + 1
                    parent[w] = u
                    nxt.append(w)
            frontier = nxt
            d += 1
    return best


__all__ = ["LAMBDA_IRREGULAR", "RHO_IRREGULAR", "build", "node_degrees", "peg_edges", "peg_code", "girth",
           "gf2_rank"]
