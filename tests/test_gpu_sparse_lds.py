"""The LDS-staged CSR kernel (CBP_KERNEL_SPARSE_LDS).

Frames with their whole state in LDS, each sweep run level by level with the edges of a
level on separate threads.  Its per-edge arithmetic and fold order are those of the
one-frame-per-lane kernel, so decisions and sweep counts must equal that kernel's bit for
bit, for CBP and the layered and flooding BP baselines with both check rules, the syndrome
stop and fixed sweeps, ragged and tiny batches (fewer frames than workgroups), weight-one
columns and the long (200-sweep) runs of the PEG codes; and through the lane kernel's own
parity, the FP64 oracle's.
"""
import sys

import numpy as np
import pytest

import oracle
from conditioning import ill_conditioned
from paper_2305_05286_amd import cbp
from paper_2305_05286_amd.workload import get_code, make_frames

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(c, t, max_iter, algo, kernel, **kw):
    b, i = cbp.decode(c, t, max_iter, algo, kernel=kernel, **kw)
    torch.cuda.synchronize()
    return b.cpu().numpy(), i.cpu().numpy()


# (code, Eb/N0, frames, max_iter): a (3,6) code of 96 bits (eight frames per workgroup), a QC
# code with a weight-one column on the CSR path, and the irregular and regular PEG codes
CODES = [("reg36_n96", 1.5, 3001, 40), ("qc_t64s", 1.5, 1999, 40), ("peg_irr_n2048", 1.25, 4099, 200),
         ("peg_reg36_n2048", 1.5, 2500, 200), ("peg_irr_n8192", 1.5, 700, 200)]


@pytest.mark.parametrize("name,ebn0,frames,max_iter", CODES)
@pytest.mark.parametrize("algo", ["cbp", "cbp_nms", "lbp", "fbp", "lbp_nms", "fbp_nms"])
def test_equals_lane_kernel(name, ebn0, frames, max_iter, algo):
    code = get_code(name)
    c = cbp.Code.from_workload(code)
    assert c.has_kernel("sparse_lds")
    # every case fits, flooding BP at n = 8192 included (157 KB: the BP kernels keep one
    # level's fold states and decide from the posterior's sign)
    assert cbp.workspace_size(c, algo, 1, kernel="sparse_lds") > 0
    llr, _ = make_frames(code, ebn0, frames, key=(43,))
    t = torch.from_numpy(llr).cuda()
    say(f"[gpu] sparse_lds {name} {algo} {frames} frames")
    rb, ri = run(c, t, max_iter, algo, "sparse")
    lb, li = run(c, t, max_iter, algo, "sparse_lds")
    assert (ri > 3).sum() > frames // 50  # frames that outlive the first sweeps
    assert np.array_equal(li, ri)
    assert np.array_equal(lb, rb)
    # fixed sweeps: every frame runs them all
    say(f"[gpu]   fixed sweeps")
    fb, fi = run(c, t, 7, algo, "sparse", stop_rule=2)
    gb, gi = run(c, t, 7, algo, "sparse_lds", stop_rule=2)
    assert (gi == 7).all() and np.array_equal(gi, fi) and np.array_equal(gb, fb)


@pytest.mark.parametrize("frames", [1, 2, 5, 300])
def test_small_batches_and_auto(frames):
    """Fewer frames than CUs (one frame per workgroup), and AUTO's pick for a CSR code."""
    code = get_code("peg_irr_n2048")
    c = cbp.Code.from_workload(code)
    llr, _ = make_frames(code, 1.5, frames, key=(44,))
    t = torch.from_numpy(llr).cuda()
    say(f"[gpu] sparse_lds {frames} frames")
    rb, ri = run(c, t, 100, "cbp", "sparse")
    for k in ("sparse_lds", "auto"):
        lb, li = run(c, t, 100, "cbp", k)
        assert np.array_equal(li, ri) and np.array_equal(lb, rb), k


def test_edge_cases():
    code = get_code("reg36_n96")
    c = cbp.Code.from_workload(code)
    llr, cw = make_frames(code, 2.0, 257, key=(45,))
    t = torch.from_numpy(llr).cuda()
    say("[gpu] sparse_lds edge cases")
    # max_iter 0: the channel decisions, no sweep
    b, i = run(c, t, 0, "cbp", "sparse_lds")
    assert (i == 0).all() and np.array_equal(b, (llr < 0).astype(np.uint8))
    # noiseless input stops before the first sweep
    clean = torch.from_numpy(np.where(cw == 0, 4.0, -4.0).astype(np.float32)).cuda()
    b, i = run(c, clean, 50, "cbp", "sparse_lds")
    assert (i == 0).all() and np.array_equal(b, cw.astype(np.uint8))
    # all-zero LLRs: x = 0 is a codeword
    z = torch.zeros((9, code.N), dtype=torch.float32, device="cuda")
    b, i = run(c, z, 50, "cbp", "sparse_lds")
    assert (i == 0).all() and not b.any()
    # empty batch
    e = torch.zeros((0, code.N), dtype=torch.float32, device="cuda")
    b, i = run(c, e, 50, "cbp", "sparse_lds")
    assert b.shape == (0, code.N) and i.shape == (0,)


def test_against_oracle():
    """The first frames of a PEG batch against the FP64 oracle: every frame that differs must be
    one the oracle alone finds ill-conditioned, and at least 99.9% of the frames (at least one
    excepted) must be equal."""
    code = get_code("peg_irr_n2048")
    c = cbp.Code.from_workload(code)
    n, mi = 400, 40
    llr, _ = make_frames(code, 1.75, 2048, key=(46,))
    t = torch.from_numpy(llr).cuda()
    say("[gpu] sparse_lds vs oracle")
    gb, gi = run(c, t, mi, "cbp", "sparse_lds")
    o = oracle.decode(code, llr[:n], mi, "cbp")
    same = (o["iters"] == gi[:n]) & (o["bits"] == gb[:n]).all(axis=1)
    bad = np.flatnonzero(~same)
    if bad.size:
        sub = {"bits": o["bits"][bad], "iters": o["iters"][bad]}
        iu, idl = ill_conditioned(code, llr[bad], mi, "cbp", o=sub)
        assert (iu | idl).all(), bad[~(iu | idl)]
    assert bad.size <= max(1, int(0.001 * n))
