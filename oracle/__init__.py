"""FP64 CPU oracle for CBP decoding and the BP schedules it is compared with.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; the product library never calls
it.  It shares no code with the GPU path (its only input from elsewhere is the
seeded workload: code matrices and float32 channel LLRs).

The arithmetic lives in ``cbp_oracle.c`` (plain C, FP64, OpenMP over frames);
this module compiles it with gcc on first use and wraps it with ctypes.
Every function follows the paper (Guan & Liang, arXiv 2305.05286):

* ``phi``, ``psi_plus``, ``psi_minus``: Sec. II-A eq. (equ_s2e5); Sec. IV-B
  eqs. (equ_s4e6), (equ_s4e13) with the absolute value of App. A (equ_ae8).
* ``decode(..., algo="cbp")``: Sec. IV-C Steps 1-3.
* ``algo="lbp"``: layered BP, Sec. II-B with the check rule (equ_s2e4).
* ``algo="fbp"``: flooding BP, Sec. II-A.
* ``algo="lbp_nms" | "fbp_nms"``: the same schedules with the normalized
  min-sum check rule (alpha * sign * min of the other clamped |Q|).
* ``algo="cbp_nms"``: CBP with the min-sum B2V/C2B of Sec. IV-D.
* the default decision of ``cbp`` / ``cbp_nms`` (``hd_mode=0``, Step 3: from
  the V2C phase of each variable's last visit) and both stopping rules
  (syndrome; Step 2(3) with ``stop_rule=1``) are pinned against a layered BP
  trajectory recorded row by row in ``tests/test_oracle_decision_pins.py``.
* ``unrolled``: a fixed number of CBP sweeps whose B2V outputs are scaled and
  offset by per-sweep, per-column weights (the differentiable decoder), with
  the flushed soft output.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "cbp_oracle.c"
LIB = HERE / "liborcbp.so"

ALGOS = {"cbp": 0, "lbp": 1, "fbp": 2, "lbp_nms": 3, "fbp_nms": 4, "cbp_nms": 5}
LMAX = 20.0
ALPHA = 0.75

_lib = None


def build(force: bool = False) -> Path:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not LIB.exists() or LIB.stat().st_mtime < SRC.stat().st_mtime:
        tmp = LIB.with_suffix(f".so.tmp{os.getpid()}")
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-Wall", "-o", str(tmp), str(SRC), "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(str(LIB))
        d, i, ll, p = ctypes.c_double, ctypes.c_int, ctypes.c_longlong, ctypes.c_void_p
        lib.orc_phi.restype = d
        lib.orc_phi.argtypes = [d]
        lib.orc_phiq.restype = d
        lib.orc_phiq.argtypes = [d, d]
        lib.orc_psi_plus.restype = d
        lib.orc_psi_plus.argtypes = [d, d, d]
        lib.orc_psi_minus.restype = d
        lib.orc_psi_minus.argtypes = [d, d, d]
        lib.orc_max_threads.restype = i
        lib.orc_max_threads.argtypes = []
        lib.orc_decode.restype = i
        lib.orc_decode.argtypes = [i, i, i, p, p, p, ll, i, d, d, i, i, p, p,
                                   i, ll, p, p, p, p, p, i]
        lib.orc_unrolled.restype = i
        lib.orc_unrolled.argtypes = [i, i, p, p, p, i, i, p, p, p, ll, d, p, i]
        _lib = lib
    return _lib


def phi(x: float) -> float:
    return _load().orc_phi(float(x))


def phiq(y: float, lmax: float = LMAX) -> float:
    return _load().orc_phiq(float(y), float(lmax))


def psi_plus(x: float, y: float, lmax: float = LMAX) -> float:
    return _load().orc_psi_plus(float(x), float(y), float(lmax))


def psi_minus(x: float, y: float, lmax: float = LMAX) -> float:
    return _load().orc_psi_minus(float(x), float(y), float(lmax))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def decode(code, llr, max_iter: int, algo: str = "cbp", *, lmax: float = LMAX,
           alpha: float = ALPHA, hd_mode: int = 0, stop_rule: int = 0,
           dump_sweep: int = 0, ndump: int = 0, opcounts: bool = False,
           nthreads: int = 0):
    """Decode float32 LLRs [B, N].  Returns dict with ``bits`` uint8 [B, N],
    ``iters`` int32 [B] and, when requested, ``Q``, ``R``, ``Om``, ``Lam``
    dumps (float64, NaN where a frame stopped before ``dump_sweep``) and
    ``ops`` int64 [max_iter, 3] (B2V, V2C, C2B per sweep of frame 0)."""
    lib = _load()
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    if llr.ndim != 2 or llr.shape[1] != code.N:
        raise ValueError("llr must be [B, N]")
    B = llr.shape[0]
    row_ptr = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(code.col_idx, dtype=np.int32)
    bits = np.zeros((B, code.N), dtype=np.uint8)
    iters = np.zeros(B, dtype=np.int32)
    out = {"bits": bits, "iters": iters}
    dq = dr = dom = dlam = None
    if dump_sweep > 0 and ndump > 0:
        ndump = min(ndump, B)
        dq = np.full((ndump, code.N), np.nan)
        dr = np.full((ndump, code.E), np.nan)
        dom = np.full((ndump, code.M), np.nan)
        dlam = np.full((ndump, code.N), np.nan)
        out.update(Q=dq, R=dr, Om=dom, Lam=dlam)
    ops = np.zeros((max(max_iter, 1), 3), dtype=np.int64) if opcounts else None
    if ops is not None:
        out["ops"] = ops
    rc = lib.orc_decode(ALGOS[algo], code.M, code.N, _ptr(row_ptr), _ptr(col_idx), _ptr(llr),
                        B, int(max_iter), float(lmax), float(alpha), int(hd_mode),
                        int(stop_rule), _ptr(bits), _ptr(iters), int(dump_sweep),
                        int(ndump if dq is not None else 0), _ptr(dq), _ptr(dr), _ptr(dom),
                        _ptr(dlam), _ptr(ops), int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_decode failed ({rc})")
    return out


def unrolled(code, llr, w, beta, *, grp=None, lmax: float = LMAX, nthreads: int = 0):
    """T = len(w) sweeps of CBP with weighted B2V outputs; returns the soft output
    float64 [B, N].  w, beta: [T, G]; grp: int [N] weight group of each variable
    (default: the base block-column v // Z of a QC code)."""
    lib = _load()
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    if llr.ndim != 2 or llr.shape[1] != code.N:
        raise ValueError("llr must be [B, N]")
    w = np.ascontiguousarray(w, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    if w.ndim != 2 or beta.shape != w.shape:
        raise ValueError("w and beta must be [T, G]")
    T, G = w.shape
    if grp is None:
        grp = np.arange(code.N) // code.Z
    grp = np.ascontiguousarray(grp, dtype=np.int32)
    row_ptr = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(code.col_idx, dtype=np.int32)
    out = np.zeros(llr.shape, dtype=np.float64)
    rc = lib.orc_unrolled(code.M, code.N, _ptr(row_ptr), _ptr(col_idx), _ptr(grp), G, T, _ptr(w),
                          _ptr(beta), _ptr(llr), llr.shape[0], float(lmax), _ptr(out), int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_unrolled failed ({rc})")
    return out
