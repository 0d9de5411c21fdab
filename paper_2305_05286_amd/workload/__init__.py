"""Seeded input generators: LDPC codes, encoders and BPSK/AWGN channel LLRs."""
from .codes import (Code, encode, gf2_rank, has_4cycle, load_code, make_qc_code,
                    qc_pattern_dualdiag, qc_pattern_staircase, qc_to_csr, save_code,
                    socket_regular_code)
from .channel import CHUNK, make_frames, noiseless_llrs, sigma2_for
from .registry import get_code, CODE_NAMES
from .mixed import RATES, Z_VALUES, make_mixed_batch, mixed_family

__all__ = [
    "Code", "encode", "gf2_rank", "has_4cycle", "load_code", "make_qc_code",
    "qc_pattern_dualdiag", "qc_pattern_staircase", "qc_to_csr", "save_code",
    "socket_regular_code", "CHUNK", "make_frames", "noiseless_llrs", "sigma2_for",
    "get_code", "CODE_NAMES", "RATES", "Z_VALUES", "make_mixed_batch", "mixed_family",
]
