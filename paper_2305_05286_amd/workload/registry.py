"""Named workload codes, frozen as JSON artefacts next to this file.

``python -m paper_2305_05286_amd.workload.registry`` regenerates every artefact
from its seed; the artefacts are committed so that every consumer reads the
same matrices without re-running the (slow, seeded) constructions.

Codes (sizes of the synthetic workloads that stand in for the paper's
rate-1/2 PEG codes, which are not published):

* ``reg36_n96``   (3,6)-regular, N=96, M=48, random sockets, no 4-cycles.
* ``qc2304``      QC, 12x24 base, Z=96, N=2304, rate 1/2, column weights 2..6,
                  dual-diagonal parity part with a weight-3 first column.
* ``qc26112``     QC, 46x68 base, Z=384, N=26112, rate 22/68, strict lower
                  dual-diagonal parity part (last column has weight 1),
                  22 information columns of seeded weight 3..8.
* ``qc2304_alt``  the ``qc2304`` base pattern with independently drawn shifts.
* ``qc_t16``      QC, 4x8 base, Z=16 (small test code, four frames per wave).
* ``qc_t64s``     QC, 4x8 base, Z=64, staircase parity (weight-1 column).
* ``peg_reg36_n2048``, ``peg_reg36_n8192``  (3,6)-regular PEG codes, rate 1/2.
* ``peg_irr_n2048``, ``peg_irr_n8192``      PEG codes with the paper's irregular
                  lambda(x), rho(x) (Sec. V), rate 1/2.
"""
from __future__ import annotations

from functools import lru_cache
from pathlib import Path

import numpy as np

from .codes import (Code, load_code, make_qc_code, qc_pattern_dualdiag,
                    qc_pattern_staircase, save_code, socket_regular_code)
from .peg import LAMBDA_IRREGULAR, peg_code

CODEBOOK = Path(__file__).resolve().parent / "codebook"

QC2304_INFO_WEIGHTS = [6, 6, 6, 5, 5, 4, 4, 3, 3, 3, 3, 3]


def _qc26112_info_weights(seed: int) -> list[int]:
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x2611]))
    return [int(w) for w in rng.integers(3, 9, size=22)]


def _build(name: str) -> Code:
    if name == "reg36_n96":
        return socket_regular_code(96, 3, 6, seed=1, name=name)
    if name == "qc2304":
        pat = qc_pattern_dualdiag(12, QC2304_INFO_WEIGHTS, seed=2)
        return make_qc_code(name, pat, 96, seed=2, kind="qc_dualdiag")
    if name == "qc2304_alt":
        pat = qc_pattern_dualdiag(12, QC2304_INFO_WEIGHTS, seed=2)
        return make_qc_code(name, pat, 96, seed=20, kind="qc_dualdiag")
    if name == "qc26112":
        pat = qc_pattern_staircase(46, _qc26112_info_weights(3), seed=3)
        return make_qc_code(name, pat, 384, seed=3, kind="qc_staircase")
    if name == "qc_t16":
        pat = qc_pattern_dualdiag(4, [3, 3, 2, 2], seed=4)
        return make_qc_code(name, pat, 16, seed=4, kind="qc_dualdiag")
    if name == "qc_t64s":
        pat = qc_pattern_staircase(4, [3, 3, 3, 2], seed=5)
        return make_qc_code(name, pat, 64, seed=5, kind="qc_staircase")
    if name.startswith("peg_"):
        _, kind, length = name.split("_")
        n = int(length[1:])
        lam = {3: 1.0} if kind == "reg36" else LAMBDA_IRREGULAR
        return peg_code(name, n, lam, seed=n + (0 if kind == "reg36" else 1))
    raise KeyError(name)


PEG_CODE_NAMES = ("peg_reg36_n2048", "peg_irr_n2048", "peg_reg36_n8192", "peg_irr_n8192")
CODE_NAMES = ("reg36_n96", "qc2304", "qc2304_alt", "qc26112", "qc_t16", "qc_t64s") + PEG_CODE_NAMES


@lru_cache(maxsize=None)
def get_code(name: str) -> Code:
    """Load a named code from its frozen artefact (built on first use if absent)."""
    path = CODEBOOK / f"{name}.json"
    if not path.exists():
        CODEBOOK.mkdir(exist_ok=True)
        save_code(_build(name), path)
    return load_code(path)


def regenerate(names=CODE_NAMES) -> None:
    CODEBOOK.mkdir(exist_ok=True)
    for n in names:
        code = _build(n)
        save_code(code, CODEBOOK / f"{n}.json")
        print(f"{n}: M={code.M} N={code.N} K={code.K} E={code.E}")


if __name__ == "__main__":
    regenerate()
