"""Frame parity on the benchmark's own frames at full sweep size, against the
FP64 oracle's stored results (tests/golden/parity_*.npz, written by
tests/golden/make_parity_tables.py, which calls only the oracle).

* n = 2304 code, register-resident kernel: the first 16384 frames of every
  Eb/N0 point of the benchmark's sweep (1.0 ... 2.5 dB, at most 50 sweeps) for
  CBP and layered NMS, the first 4096 for CBP-NMS and flooding NMS.
* n = 26112 code, streamed kernel: the first 512 frames of every point of its
  sweep (0.5 ... 1.5 dB, at most 25 sweeps), and the last 128 frames of the
  4096-frame batch at 1.0 dB, which slots decode after refilling.

Bar: decisions and sweep count identical on >= 99.9% of the frames that the
oracle finds well-conditioned (at least one differing frame allowed per point) (tests/conditioning.py: its result survives one
ulp of every LLR and random relative perturbations at the FP32 kernels' own
message error), converged or not; the ill-conditioned share is reported and
bounded (log-tanh CBP: at most 4% of a point's frames), and the bar holds
on the converged frames alone as well.
"""
import hashlib
import sys
from pathlib import Path

import numpy as np
import pytest

from paper_2305_05286_amd import cbp
from paper_2305_05286_amd.workload import get_code, make_frames

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = Path(__file__).resolve().parent / "golden"
PARITY = 0.999
# Bound on the ill-conditioned share of a point.  Log-tanh CBP: 2.5% of the
# frames at 1.0 dB on the n = 2304 code.  The min-sum decoders: at 1.0 dB half
# of their frames never converge, and the FP64 result of most of those moves
# under one ulp of the input (43% of layered NMS's frames), so their bar holds
# on the remaining frames.
ILL_BOUND = {"cbp": 0.04, "lbp_nms": 0.6, "cbp_nms": 0.6, "fbp_nms": 0.6}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def tables(cname):
    return dict(np.load(GOLDEN / f"parity_{cname}.npz"))


def digest_rows(bits):
    pk = np.packbits(bits, axis=1)
    return np.array([int.from_bytes(hashlib.blake2b(r.tobytes(), digest_size=8).digest(), "little")
                     for r in pk], dtype=np.uint64)


def compare(T, name, gb, gi, cw):
    """Per-frame equality of the GPU result with the stored oracle result."""
    n = int(T[f"{name}/meta"][4])
    mi = int(T[f"{name}/meta"][5])
    oi = T[f"{name}/iters"].astype(np.int32)
    cwok = np.unpackbits(T[f"{name}/cwok"])[:n].astype(bool)
    ill = np.unpackbits(T[f"{name}/ill"])[:n].astype(bool) | np.unpackbits(T[f"{name}/illd"])[:n].astype(bool)
    assert gb.shape[0] == n and gi.shape[0] == n
    same = gi == oi
    same[cwok] &= (gb[cwok] == cw[cwok]).all(axis=1)
    rest = np.nonzero(~cwok)[0]
    same[rest] &= digest_rows(gb[rest]) == T[f"{name}/hash"]
    return same, ill, oi < mi


def check(label, algo, same, ill, conv):
    well = ~ill
    p_all, p_well = same.mean(), same[well].mean()
    say(f"    {label}: frames equal {p_all:.5f}; ill-conditioned {ill.mean():.4f}; equal on well-conditioned "
        f"{p_well:.5f} (converged {same[well & conv].mean() if (well & conv).any() else 1:.5f}, "
        f"failed {same[well & ~conv].mean() if (well & ~conv).any() else 1:.5f}); "
        f"{int((~same).sum())} differ, {int((~same & ill).sum())} of them ill-conditioned")
    assert ill.mean() <= ILL_BOUND[algo], (label, ill.mean())
    assert (~same & well).sum() <= allowed(well.sum()), (label, p_well)
    assert (~same & well & conv).sum() <= allowed((well & conv).sum()), label


def allowed(n):
    """Differing frames the bar allows among n: 0.1% of them, and at least one
    (a point of 512 frames cannot resolve 99.9%: one frame is 0.2%)."""
    return max(1, int((1.0 - PARITY) * n))


SNRS_2304 = [1.0, 1.25, 1.5, 1.75, 2.0, 2.25, 2.5]


@pytest.mark.parametrize("snr", SNRS_2304)
def test_qc2304_register_kernel_full_sweep(snr):
    T = tables("qc2304")
    code = get_code("qc2304")
    h = cbp.Code.from_workload(code)
    c = round(100 * snr)
    n = int(T[f"cbp_{c}/meta"][4])
    llr, cw = make_frames(code, snr, n, key=(2024, c))
    t = torch.from_numpy(llr).cuda()
    for algo in ("cbp", "lbp_nms", "cbp_nms", "fbp_nms"):
        name = f"{algo}_{c}"
        m = int(T[f"{name}/meta"][4])
        say(f"[gpu] qc2304 {algo} qc_reg {snr} dB, {m} frames")
        gb, gi = cbp.decode(h, t[:m], 50, algo, kernel="qc_reg")
        torch.cuda.synchronize()
        same, ill, conv = compare(T, name, gb.cpu().numpy(), gi.cpu().numpy(), cw[:m])
        check(f"qc2304 {algo} {snr} dB", algo, same, ill, conv)


@pytest.mark.parametrize("snr", [0.5, 0.75, 1.0, 1.25, 1.5])
def test_qc26112_streamed_kernel_sweep(snr):
    T = tables("qc26112")
    code = get_code("qc26112")
    h = cbp.Code.from_workload(code)
    c = round(100 * snr)
    llr, cw = make_frames(code, snr, 512, key=(2027, c))
    t = torch.from_numpy(llr).cuda()
    for algo in ("cbp", "lbp_nms", "fbp_nms", "cbp_nms"):
        say(f"[gpu] qc26112 {algo} qc_stream {snr} dB, 512 frames")
        gb, gi = cbp.decode(h, t, 25, algo, kernel="qc_stream")
        torch.cuda.synchronize()
        same, ill, conv = compare(T, f"{algo}_{c}", gb.cpu().numpy(), gi.cpu().numpy(), cw)
        check(f"qc26112 {algo} {snr} dB", algo, same, ill, conv)


def test_qc26112_refilled_slots_full_batch():
    """4096 frames in one launch (1280 slots in flight at most): the last 128
    frames are decoded by slots that took them from the frame counter after
    finishing earlier frames."""
    T = tables("qc26112")
    code = get_code("qc26112")
    h = cbp.Code.from_workload(code)
    llr, cw = make_frames(code, 1.0, 4096, key=(2027, 100))
    t = torch.from_numpy(llr).cuda()
    for algo in ("cbp", "lbp_nms"):
        say(f"[gpu] qc26112 {algo} qc_stream 1.0 dB, 4096 frames, last 128 against the oracle")
        gb, gi = cbp.decode(h, t, 25, algo, kernel="qc_stream")
        torch.cuda.synchronize()
        same, ill, conv = compare(T, f"refill_{algo}_100", gb[-128:].cpu().numpy(), gi[-128:].cpu().numpy(),
                                  cw[-128:])
        check(f"qc26112 {algo} refilled slots", algo, same, ill, conv)
