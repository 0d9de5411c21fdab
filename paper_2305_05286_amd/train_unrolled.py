"""Training of the unrolled, weighted CBP decoder (per-sweep, per-column B2V scale and offset).

    python -m paper_2305_05286_amd.train_unrolled --steps 2000 --sweeps 10 --batch 8192

Each step draws a fresh batch on the GPU: codewords sampled from a pool of seeded random
codewords of the n=2304 QC code, BPSK over AWGN at a per-frame Eb/N0 uniform in
[1.5, 2.5] dB (L = 2y / sigma^2), and takes one Adam step on the mean binary cross-entropy
between the soft output and the transmitted bits (o > 0 favours bit 0).  The decoder's
forward and backward passes are the library's kernels (cbp_unrolled_forward / _backward).
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def gpu_batch(pool, rate: float, batch: int, snr_lo: float, snr_hi: float, gen):
    """Fresh frames on the GPU: (llr float32 [B, N], codewords float32 [B, N])."""
    import torch
    idx = torch.randint(0, pool.shape[0], (batch,), device=pool.device, generator=gen)
    c = pool[idx]
    ebn0 = snr_lo + (snr_hi - snr_lo) * torch.rand(batch, 1, device=pool.device, generator=gen)
    s2 = 1.0 / (2.0 * rate * 10.0 ** (ebn0 / 10.0))
    y = (1.0 - 2.0 * c) + torch.sqrt(s2) * torch.randn(c.shape, device=pool.device, generator=gen)
    return (2.0 / s2) * y, c


def evaluate(model, llr, cw):
    import torch
    with torch.no_grad():
        o = model(llr)
        bce = torch.nn.functional.binary_cross_entropy_with_logits(-o, cw).item()
        err = ((o < 0).float() != cw)
        return {"bce": bce, "ber": err.float().mean().item(), "fer": err.any(dim=1).float().mean().item()}


def train(code_name: str = "qc2304", sweeps: int = 10, steps: int = 2000, batch: int = 8192,
          snr=(1.5, 2.5), lr: float = 1e-2, seed: int = 0, pool_size: int = 32768, log_every: int = 100,
          log=print):
    import torch
    from . import cbp
    from .workload import get_code, make_frames

    code = get_code(code_name)
    handle = cbp.Code.from_workload(code)
    _, cw = make_frames(code, 2.0, pool_size, key=(7001, seed))
    pool = torch.from_numpy(cw.astype(np.float32)).cuda()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    vgen = torch.Generator(device="cuda")
    vgen.manual_seed(seed + 1000)
    vl, vc = gpu_batch(pool, code.rate, batch, snr[0], snr[1], vgen)

    model = cbp.unrolled_module(handle, sweeps).cuda()
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    hist = {"step": [], "train_bce": [], "val": []}
    base = evaluate(model, vl, vc)  # w = 1, beta = 0: plain CBP with `sweeps` sweeps
    log(f"[train] {code_name}, {sweeps} sweeps, batch {batch}, Eb/N0 U[{snr[0]}, {snr[1]}] dB: "
        f"plain CBP validation {base}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(1, steps + 1):
        llr, c = gpu_batch(pool, code.rate, batch, snr[0], snr[1], gen)
        o = model(llr)
        loss = torch.nn.functional.binary_cross_entropy_with_logits(-o, c)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        if step % log_every == 0 or step == steps:
            v = evaluate(model, vl, vc)
            hist["step"].append(step)
            hist["train_bce"].append(loss.item())
            hist["val"].append(v)
            log(f"[train] step {step}: train BCE {loss.item():.5f}, validation {v}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    final = evaluate(model, vl, vc)
    return {"code": code_name, "sweeps": sweeps, "batch": batch, "steps": steps, "lr": lr,
            "snr_db": list(snr), "seconds": dt, "steps_per_s": steps / dt,
            "frames_per_s": steps * batch / dt, "untrained": base, "trained": final,
            "w": model.w.detach().cpu().numpy().tolist(), "beta": model.beta.detach().cpu().numpy().tolist(),
            "history": hist}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--code", default="qc2304")
    ap.add_argument("--sweeps", type=int, default=10)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None, help="write the result (weights, history) as JSON")
    a = ap.parse_args()
    res = train(a.code, a.sweeps, a.steps, a.batch, lr=a.lr, seed=a.seed)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(res, fh)
    print(json.dumps({k: v for k, v in res.items() if k not in ("w", "beta", "history")}))


if __name__ == "__main__":
    main()
