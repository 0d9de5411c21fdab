"""Mixed-code workload: QC codes of five rates and five lifting sizes in one batch.

Each frame draws its code uniformly from the family and its Eb/N0 uniformly from
[0, 4] dB; frames are packed back to back (frame f's N LLRs start at offset[f]).

Family: one base pattern per rate, lifted at every Z in ``Z_VALUES``.

  rate  base (mb x nb)  information block-columns
  1/3   16 x 24          8
  1/2   12 x 24         12
  2/3    8 x 24         16
  5/6    4 x 24         20
  8/9    3 x 27         24

The parity part is the strict lower dual-diagonal (staircase) used for the
n=26112 code, so every code has a linear-time encoder; information
block-columns have weight 3 or 4 (at most mb).  Shifts are U[0, Z) with lifted
4-cycles rejected where the lifting size leaves room for it (small Z with dense
high-rate bases cannot avoid them all; such draws keep the last candidate).
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from .codes import Code, _base_4cycle_ok, encode, qc_pattern_staircase, qc_to_csr

RATES = (("1/3", 16, 24), ("1/2", 12, 24), ("2/3", 8, 24), ("5/6", 4, 24), ("8/9", 3, 27))
Z_VALUES = (16, 32, 64, 128, 384)

__all__ = ["RATES", "Z_VALUES", "mixed_family", "make_mixed_batch"]


def _info_weights(mb: int, kb: int) -> list[int]:
    return [min(mb, 4 if i % 3 == 0 else 3) for i in range(kb)]


def _draw_shifts(pattern: np.ndarray, Z: int, seed: int, max_tries: int = 64) -> np.ndarray:
    mb, nb = pattern.shape
    kb = nb - mb
    rng = np.random.default_rng(np.random.SeedSequence([seed, Z, 0x313]))
    sh = np.full((mb, nb), -1, dtype=np.int64)
    for j in range(mb):  # staircase parity part: identity blocks
        sh[j, kb + j] = 0
        if j + 1 < mb:
            sh[j + 1, kb + j] = 0
    for b in range(kb):
        for r in range(mb):
            if pattern[r, b] == 0:
                continue
            for _ in range(max_tries):
                sh[r, b] = rng.integers(0, Z)
                if _base_4cycle_ok(sh, Z, r, b):
                    break
    return sh.astype(np.int32)


@lru_cache(maxsize=None)
def mixed_family(z_values: tuple = Z_VALUES, rates: tuple = RATES) -> tuple:
    """The family's codes (rate-major, then Z), deterministic from fixed seeds."""
    codes = []
    for ri, (rname, mb, nb) in enumerate(rates):
        kb = nb - mb
        pat = qc_pattern_staircase(mb, _info_weights(mb, kb), seed=100 + ri)
        for Z in z_values:
            sh = _draw_shifts(pat, Z, seed=100 + ri)
            row_ptr, col_idx = qc_to_csr(sh, Z)
            codes.append(Code(name=f"mix_r{rname.replace('/', '_')}_z{Z}", M=mb * Z, N=nb * Z,
                              row_ptr=row_ptr, col_idx=col_idx, K=kb * Z,
                              info_pos=np.arange(kb * Z, dtype=np.int32), encoder="qc_staircase",
                              seed=100 + ri, Z=Z, shifts=sh))
    return tuple(codes)


def make_mixed_batch(codes, n_frames: int, key=(0,), ebn0_range=(0.0, 4.0), *,
                     return_codewords: bool = True) -> dict:
    """A packed mixed batch.

    Returns a dict with ``code`` int32[B] (index into ``codes``), ``offset``
    int64[B], ``ebn0`` float64[B], ``llr`` float32[total] and, if asked,
    ``codeword`` uint8[total].  Frame f uses BPSK over AWGN at its own Eb/N0
    (sigma^2 = 1 / (2 R 10^(Eb/N0 / 10)), L = 2y / sigma^2 in float64 rounded
    to float32 once, as for the single-code workload).
    """
    key = tuple(int(k) for k in key)
    rng = np.random.default_rng(np.random.SeedSequence([*key, 0xa11]))
    cidx = rng.integers(0, len(codes), size=n_frames).astype(np.int32)
    ebn0 = rng.uniform(ebn0_range[0], ebn0_range[1], size=n_frames)
    lens = np.array([codes[c].N for c in cidx], dtype=np.int64)
    offset = np.zeros(n_frames, dtype=np.int64)
    if n_frames:
        offset[1:] = np.cumsum(lens)[:-1]
    total = int(lens.sum())
    llr = np.empty(total, dtype=np.float32)
    cw = np.empty(total, dtype=np.uint8) if return_codewords else None
    for c, code in enumerate(codes):
        fr = np.nonzero(cidx == c)[0]
        if fr.size == 0:
            continue
        ri = np.random.default_rng(np.random.SeedSequence([*key, c, 0]))
        rn = np.random.default_rng(np.random.SeedSequence([*key, c, 1]))
        info = ri.integers(0, 2, size=(fr.size, code.K), dtype=np.uint8)
        noise = rn.standard_normal((fr.size, code.N), dtype=np.float32)
        x = encode(code, info)
        s2 = 1.0 / (2.0 * code.rate * 10.0 ** (ebn0[fr] / 10.0))
        y = (1.0 - 2.0 * x.astype(np.float64)) + np.sqrt(s2)[:, None] * noise.astype(np.float64)
        vals = ((2.0 / s2)[:, None] * y).astype(np.float32)
        idx = offset[fr][:, None] + np.arange(code.N)[None, :]
        llr[idx] = vals
        if cw is not None:
            cw[idx] = x
    out = {"code": cidx, "offset": offset, "ebn0": ebn0, "llr": llr}
    if cw is not None:
        out["codeword"] = cw
    return out
