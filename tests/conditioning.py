"""Which frames sit at a tipping point that FP32 arithmetic can move, judged by
the FP64 oracle alone (test infrastructure).

A frame is ill-conditioned when the oracle's result (decisions or sweep count)
changes under any of these input perturbations:

* every LLR moved one float32 ulp up, or one ulp down;
* every LLR scaled by 1 + DELTA or 1 - DELTA with the sign drawn at random per
  LLR (DRAWS draws).  DELTA = 2e-6 is the relative error the FP32 kernels'
  arithmetic puts on a message in one update: two evaluations of their
  check-rule approximation, each within 8.3e-7 relative of the exact function
  (checked on the host against the closed form), plus a few float32 roundings.

Such a frame can be decided differently by any FP32 decoder that follows the
method exactly, so it is excused from frame-exact parity; every other frame,
converged or not, is held to it.  The perturbations are oracle inputs derived
from the channel LLRs only, never from a GPU output.
"""
from __future__ import annotations

import numpy as np

import oracle

DELTA = 2e-6
DRAWS = 2


def changed(code, o, llr, max_iter, algo, **kw):
    p = oracle.decode(code, llr, max_iter, algo, **kw)
    return (p["iters"] != o["iters"]) | (p["bits"] != o["bits"]).any(axis=1)


def ill_ulp(code, o, llr, max_iter, algo, **kw):
    ill = np.zeros(len(llr), dtype=bool)
    for d in (np.inf, -np.inf):
        ill |= changed(code, o, np.nextafter(llr, np.float32(d)), max_iter, algo, **kw)
    return ill


def ill_delta(code, o, llr, max_iter, algo, **kw):
    ill = np.zeros(len(llr), dtype=bool)
    for k in range(DRAWS):
        u = np.random.default_rng([7, k]).choice([-1.0, 1.0], size=llr.shape)
        ill |= changed(code, o, (llr.astype(np.float64) * (1.0 + DELTA * u)).astype(np.float32),
                       max_iter, algo, **kw)
    return ill


def ill_conditioned(code, llr, max_iter, algo, o=None, **kw):
    """(ill_ulp, ill_delta) masks of the frames `llr` for the oracle run `o`
    (computed if not given) of the same frames and options."""
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    if o is None:
        o = oracle.decode(code, llr, max_iter, algo, **kw)
    return ill_ulp(code, o, llr, max_iter, algo, **kw), ill_delta(code, o, llr, max_iter, algo, **kw)
