"""Write the FP64 oracle's results on the benchmark's own frames, for the GPU
parity tests at full sweep size (the oracle needs tens of CPU-minutes for
them, so they are computed once here and stored).

Calls only ``oracle`` and the seeded input generators.  For every frame of
every (code, decoder, Eb/N0) entry it stores:

* ``iters``: the oracle's sweep count;
* ``cwok``: whether the oracle's decisions equal the transmitted codeword,
  and for the frames where they do not, ``hash``: an 8-byte BLAKE2b digest of
  the decisions (np.packbits of the row);
* ``ill``: whether the oracle's result (decisions or sweep count) changes
  when every LLR moves by one float32 ulp up, or one ulp down;
* ``illd``: whether it changes when every LLR is scaled by 1 +- DELTA with
  random signs (tests/conditioning.py states DELTA and its derivation).
A frame flagged by either sits at a tipping point that the FP32 kernels'
own error can move, so it is excused from frame-exact parity (the decision
is the oracle's, never the GPU's).

Frames: the benchmark's streams (prefixes are reproducible on their own):
the n = 2304 code, key (2024, round(100 * Eb/N0)), the first 16384 frames
(CBP, layered NMS) or 4096 (CBP-NMS, flooding NMS) at 1.0 ... 2.5 dB, at most
50 sweeps; the n = 26112 code, key (2027, round(100 * Eb/N0)), the first 512
frames at 0.5 ... 1.5 dB, at most 25 sweeps, and the last 128 frames of the
benchmark's 4096-frame batch at 1.0 dB, which the streamed kernel decodes in
refilled slots.

    python tests/golden/make_parity_tables.py [qc2304|qc26112 ...]
"""
from __future__ import annotations

import hashlib
import sys
import time
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
ROOT = HERE.parents[1]
for p in (ROOT, HERE.parent):
    if str(p) not in sys.path:
        sys.path.insert(0, str(p))

import oracle  # noqa: E402
from conditioning import ill_delta, ill_ulp  # noqa: E402
from paper_2305_05286_amd.workload import get_code, make_frames  # noqa: E402

SNRS_2304 = [1.0, 1.25, 1.5, 1.75, 2.0, 2.25, 2.5]
SNRS_26112 = [0.5, 0.75, 1.0, 1.25, 1.5]

# (code, entry name, decoder, Eb/N0, key, first frame, frames, max_iter)
ENTRIES = (
    [("qc2304", f"{a}_{round(100 * s)}", a, s, (2024, round(100 * s)), 0, n, 50)
     for a, n in (("cbp", 16384), ("lbp_nms", 16384), ("cbp_nms", 4096), ("fbp_nms", 4096))
     for s in SNRS_2304]
    + [("qc26112", f"{a}_{round(100 * s)}", a, s, (2027, round(100 * s)), 0, 512, 25)
       for a in ("cbp", "lbp_nms", "fbp_nms", "cbp_nms") for s in SNRS_26112]
    + [("qc26112", f"refill_{a}_100", a, 1.0, (2027, 100), 4096 - 128, 128, 25)
       for a in ("cbp", "lbp_nms")]
)


def digest(bits: np.ndarray) -> np.ndarray:
    """8-byte BLAKE2b of each packed row, as uint64."""
    pk = np.packbits(bits, axis=1)
    return np.array([int.from_bytes(hashlib.blake2b(r.tobytes(), digest_size=8).digest(), "little")
                     for r in pk], dtype=np.uint64)


def frames(code, snr, key, first, n):
    llr, cw = make_frames(code, snr, first + n, key=key)
    return llr[first:], cw[first:]


def entry(code, algo, snr, key, first, n, max_iter, only_delta=False):
    llr, cw = frames(code, snr, key, first, n)
    o = oracle.decode(code, llr, max_iter, algo)
    illd = ill_delta(code, o, llr, max_iter, algo)
    if only_delta:
        return {"illd": np.packbits(illd)}
    ill = ill_ulp(code, o, llr, max_iter, algo)
    cwok = (o["bits"] == cw).all(axis=1)
    return {"iters": o["iters"].astype(np.uint8), "cwok": np.packbits(cwok), "ill": np.packbits(ill),
            "illd": np.packbits(illd), "hash": digest(o["bits"][~cwok])}


def oracle_source_digest() -> str:
    return hashlib.sha256(oracle.SRC.read_bytes()).hexdigest()


def main(names) -> None:
    for cname in names:
        out = HERE / f"parity_{cname}.npz"
        store = dict(np.load(out)) if out.exists() else {}
        if str(store.get("oracle_sha256", "")) != oracle_source_digest():
            store = {}
        code = get_code(cname)
        for c, name, algo, snr, key, first, n, mi in ENTRIES:
            if c != cname or f"{name}/illd" in store:
                continue
            t0 = time.time()
            e = entry(code, algo, snr, key, first, n, mi, only_delta=f"{name}/iters" in store)
            for k, v in e.items():
                store[f"{name}/{k}"] = v
            store[f"{name}/meta"] = np.array([snr, key[0], key[1], first, n, mi], dtype=np.float64)
            store["oracle_sha256"] = np.array(oracle_source_digest())
            np.savez_compressed(out, **store)
            ill = np.unpackbits(store[f"{name}/ill"])[:n].astype(bool)
            illd = np.unpackbits(store[f"{name}/illd"])[:n].astype(bool)
            it = store[f"{name}/iters"]
            print(f"{cname} {name}: {n} frames in {time.time() - t0:.0f}s, mean sweeps "
                  f"{it.mean():.2f}, failed {(it >= mi).mean():.4f}, "
                  f"ill-conditioned: one ulp {ill.mean():.4f}, +-DELTA {illd.mean():.4f}, "
                  f"either {(ill | illd).mean():.4f}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["qc2304", "qc26112"])
