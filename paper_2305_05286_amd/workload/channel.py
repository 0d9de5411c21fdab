"""Seeded BPSK / AWGN workload: random information words to FP32 channel LLRs.

The channel model is the paper's simulation setup (Sec. V: BPSK over AWGN);
the prior LLR is the log-likelihood ratio of Sec. IV Step 1 (the latest V2C
message is initialised to ln Pr(y|x=0)/Pr(y|x=1)).  Fixed here because the
paper leaves them open:

* mapping bit 0 -> +1, bit 1 -> -1, so L > 0 favours bit 0;
* noise variance sigma^2 = 1 / (2 R 10^(Eb/N0 / 10)) with R = K/N;
* L = 2 y / sigma^2, computed in float64 and rounded to float32 once; every
  decoder (GPU kernels and the oracle) consumes this same float32 array.

Randomness: frames are generated in chunks of ``CHUNK`` frames; chunk j of a
stream keyed by ``key`` uses ``SeedSequence([*key, j, 0])`` for the info bits
and ``SeedSequence([*key, j, 1])`` for the noise, so any prefix of a batch is
reproducible on its own.
"""
from __future__ import annotations

import numpy as np

from .codes import Code, encode

CHUNK = 8192

__all__ = ["CHUNK", "sigma2_for", "make_frames", "noiseless_llrs"]


def sigma2_for(code: Code, ebn0_db: float) -> float:
    return 1.0 / (2.0 * code.rate * 10.0 ** (ebn0_db / 10.0))


def make_frames(code: Code, ebn0_db: float, n_frames: int, key=(0,), *,
                start: int = 0, return_codewords: bool = True):
    """Return (llr float32[B,N], codeword uint8[B,N] or None).

    Frames [start, start + n_frames) of the stream ``key``; ``start`` must be a
    multiple of ``CHUNK`` so that a prefix sample equals the full batch's prefix.
    """
    if start % CHUNK:
        raise ValueError("start must be a multiple of CHUNK")
    key = tuple(int(k) for k in key)
    s2 = sigma2_for(code, ebn0_db)
    sigma = np.sqrt(s2)
    llr = np.empty((n_frames, code.N), dtype=np.float32)
    cw = np.empty((n_frames, code.N), dtype=np.uint8) if return_codewords else None
    done = 0
    chunk = start // CHUNK
    while done < n_frames:
        nb = min(CHUNK, n_frames - done)
        ri = np.random.default_rng(np.random.SeedSequence([*key, chunk, 0]))
        rn = np.random.default_rng(np.random.SeedSequence([*key, chunk, 1]))
        info = ri.integers(0, 2, size=(CHUNK, code.K), dtype=np.uint8)[:nb]
        noise = rn.standard_normal((CHUNK, code.N), dtype=np.float32)[:nb]
        c = encode(code, info)
        y = (1.0 - 2.0 * c.astype(np.float64)) + sigma * noise.astype(np.float64)
        llr[done:done + nb] = (2.0 / s2) * y
        if cw is not None:
            cw[done:done + nb] = c
        done += nb
        chunk += 1
    return llr, cw


def noiseless_llrs(code: Code, n_frames: int, amplitude: float, seed: int = 0):
    """LLRs (1 - 2c) * amplitude for random codewords c (no noise)."""
    rng = np.random.default_rng(seed)
    info = rng.integers(0, 2, size=(n_frames, code.K), dtype=np.uint8)
    c = encode(code, info)
    return ((1.0 - 2.0 * c.astype(np.float32)) * np.float32(amplitude)).astype(np.float32), c
