"""Error rates and convergence of CBP, LBP and FBP on the PEG codes (Sec. V, Figs. 6-9).

    python -m paper_2305_05286_amd.peg_study --out results.json

For each PEG code (regular (3,6) and the paper's irregular lambda/rho, lengths
2048 and 8192, rate 1/2) and each Eb/N0 point, frames are decoded with at most
200 sweeps by

* ``cbp``        CBP (Sec. IV-C), stopping on a zero syndrome after a sweep;
* ``cbp_paper``  CBP with the paper's stopping rule (Step 2(3));
* ``lbp``        layered BP with the log-tanh check rule (Sec. II-B);
* ``fbp``        flooding BP with the log-tanh check rule (Sec. II-A);
* ``cbp_nms``    CBP with the normalized min-sum rule of Sec. IV-D (``--alpha``,
                 default 0.75; the paper's Figs. 10-12), on request,

all through the library's CSR kernels (frames staged in LDS where a frame fits
and the options allow, else one frame per lane; the two agree bit for bit;
the paper's stopping rule runs one frame per lane).  A point stops after ``--errors``
frame errors or ``--max-frames`` frames.  Frames: BPSK over AWGN (bit 0 -> +1,
L = 2 y / sigma^2, sigma^2 = 1 / (2 R Eb/N0)), codewords drawn from a pool of
seeded random codewords, fresh noise drawn on the GPU for every batch.  The
decoders' error probability does not depend on the codeword sent (BP and CBP
are symmetric in it), so a pool stands in for fresh codewords.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

DECODERS = {"cbp": ("cbp", {}), "cbp_paper": ("cbp", {"stop_rule": 1}),
            "lbp": ("lbp", {}), "fbp": ("fbp", {}), "cbp_nms": ("cbp_nms", {})}
DEFAULT_DECODERS = ("cbp", "cbp_paper", "lbp", "fbp")
CODES = ("peg_reg36_n2048", "peg_irr_n2048", "peg_reg36_n8192", "peg_irr_n8192")
SNRS = (1.2, 1.4, 1.6, 1.8, 2.0, 2.2)


def run_point(handle, pool, rate, ebn0, algo, kw, max_iter, batch, max_frames, target_errors, gen):
    import torch
    from . import cbp
    n_fr = n_fe = n_be = 0
    it_sum = 0
    t0 = time.perf_counter()
    s2 = 1.0 / (2.0 * rate * 10.0 ** (ebn0 / 10.0))
    while n_fr < max_frames and n_fe < target_errors:
        b = min(batch, max_frames - n_fr)
        idx = torch.randint(0, pool.shape[0], (b,), device=pool.device, generator=gen)
        c = pool[idx]
        y = (1.0 - 2.0 * c.float()) + (s2 ** 0.5) * torch.randn(c.shape, device=pool.device, generator=gen)
        llr = ((2.0 / s2) * y).contiguous()
        # the CSR kernels: frames staged in LDS where a frame fits and the options
        # allow (bit-identical to the one-frame-per-lane kernel), else one per lane
        bits, iters = cbp.decode(handle, llr, max_iter, algo, kernel="auto", **kw)
        err = bits != c
        fe = err.any(dim=1)
        n_fe += int(fe.sum())
        n_be += int(err.sum())
        it_sum += int(iters.sum())
        n_fr += b
    torch.cuda.synchronize()
    return {"frames": n_fr, "frame_errors": n_fe, "fer": n_fe / n_fr, "ber": n_be / (n_fr * pool.shape[1]),
            "mean_iters": it_sum / n_fr, "seconds": time.perf_counter() - t0}


def study(codes=CODES, snrs=SNRS, decoders=DEFAULT_DECODERS, max_iter=200, batch=131072,
          max_frames=1 << 18, target_errors=100, pool_size=4096, seed=0, alpha=0.75, log=print):
    import torch
    from . import cbp
    from .workload import encode, get_code
    out = {"max_iter": max_iter, "target_errors": target_errors, "max_frames": max_frames, "alpha": alpha,
           "points": []}
    for name in codes:
        code = get_code(name)
        handle = cbp.Code.from_workload(code)
        rng = np.random.default_rng(np.random.SeedSequence([seed, code.N, code.E]))
        cw = encode(code, rng.integers(0, 2, size=(pool_size, code.K), dtype=np.uint8))
        pool = torch.from_numpy(cw).cuda()
        for ebn0 in snrs:
            for dname in decoders:
                algo, kw = DECODERS[dname]
                if algo.endswith("nms"):
                    kw = dict(kw, alpha=alpha)
                gen = torch.Generator(device="cuda")
                gen.manual_seed(int(seed * 1_000_003 + code.N * 101 + round(ebn0 * 100)))
                r = run_point(handle, pool, code.rate, ebn0, algo, kw, max_iter, batch, max_frames,
                              target_errors, gen)
                r.update({"code": name, "ebn0_db": ebn0, "decoder": dname})
                out["points"].append(r)
                log(f"[peg] {name} {ebn0:.2f} dB {dname:9s}: FER {r['fer']:.3e} ({r['frame_errors']}/"
                    f"{r['frames']}), BER {r['ber']:.3e}, mean sweeps {r['mean_iters']:.2f} "
                    f"[{r['seconds']:.1f} s]")
    return out


def table(res) -> str:
    """Markdown: per code, FER and mean sweeps per decoder and Eb/N0."""
    lines = []
    codes = list(dict.fromkeys(p["code"] for p in res["points"]))
    decs = list(dict.fromkeys(p["decoder"] for p in res["points"]))
    for name in codes:
        pts = [p for p in res["points"] if p["code"] == name]
        snrs = sorted(set(p["ebn0_db"] for p in pts))
        lines.append(f"\n{name} (FER / mean sweeps, max {res['max_iter']})\n")
        lines.append("| Eb/N0 | " + " | ".join(decs) + " |")
        lines.append("|---" * (len(decs) + 1) + "|")
        for s in snrs:
            row = [f"{s:.1f}"]
            for d in decs:
                p = next(q for q in pts if q["ebn0_db"] == s and q["decoder"] == d)
                fer = f"{p['fer']:.2e}" if p["frame_errors"] else f"<{1 / p['frames']:.0e}"
                row.append(f"{fer} / {p['mean_iters']:.1f}")
            lines.append("| " + " | ".join(row) + " |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--codes", default=",".join(CODES))
    ap.add_argument("--snrs", default=",".join(str(s) for s in SNRS))
    ap.add_argument("--decoders", default=",".join(DEFAULT_DECODERS))
    ap.add_argument("--max-iter", type=int, default=200)
    ap.add_argument("--batch", type=int, default=131072)
    ap.add_argument("--max-frames", type=int, default=1 << 18)
    ap.add_argument("--errors", type=int, default=100)
    ap.add_argument("--alpha", type=float, default=0.75, help="normalization of the min-sum decoders")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    res = study(a.codes.split(","), [float(s) for s in a.snrs.split(",")], a.decoders.split(","),
                a.max_iter, a.batch, a.max_frames, a.errors, alpha=a.alpha,
                log=lambda m: (print(m), sys.stdout.flush()))
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
    print(table(res))


if __name__ == "__main__":
    main()
