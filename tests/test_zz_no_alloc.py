"""cbp_decode_static: the decoders with the library's static device scratch as
workspace (nothing allocated), against the allocating entry points on the same
inputs.  Same kernels, and the results of the persistent kernels do not depend
on how many frames are in flight, so decisions and sweep counts must be equal
bit for bit; each case makes two calls in a row, the second on a smaller batch,
so stale scratch contents from the first call would show.
"""
import sys

import numpy as np
import pytest

from paper_2305_05286_amd import cbp
from paper_2305_05286_amd.workload import get_code, make_frames

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    # (code, algo, kernel, Eb/N0, first batch, second batch, max_iter)
    ("qc2304", "cbp", "qc_reg", 1.75, 4096, 1000, 50),
    ("qc2304", "lbp_nms", "qc_reg", 1.75, 4096, 999, 50),
    ("qc2304", "cbp", "qc_stream", 1.75, 3000, 500, 50),
    ("qc26112", "cbp", "qc_stream", 1.0, 512, 100, 25),
    ("qc26112", "fbp_nms", "qc_stream", 1.25, 300, 77, 25),
    ("reg36_n96", "cbp", "sparse", 2.0, 5000, 300, 30),
    ("peg_irr_n2048", "lbp", "sparse", 1.5, 1500, 100, 60),
    ("peg_irr_n2048", "cbp_nms", "sparse", 1.5, 1500, 65, 60),
]


@pytest.mark.parametrize("name,algo,kernel,ebn0,b1,b2,max_iter", CASES,
                         ids=[f"{c[0]}-{c[1]}-{c[2]}" for c in CASES])
def test_static_matches_allocating_entry(name, algo, kernel, ebn0, b1, b2, max_iter):
    code = get_code(name)
    c = cbp.Code.from_workload(code)
    llr, _ = make_frames(code, ebn0, b1, key=(61,))
    t = torch.from_numpy(llr).cuda()
    for B in (b1, b2):
        say(f"[gpu] static scratch {name} {algo} {kernel} batch {B}")
        rb, ri = cbp.decode(c, t[:B], max_iter, algo, kernel=kernel)
        sb, si = cbp.decode_static(c, t[:B], max_iter, algo, kernel=kernel)
        torch.cuda.synchronize()
        rb, ri, sb, si = rb.cpu().numpy(), ri.cpu().numpy(), sb.cpu().numpy(), si.cpu().numpy()
        say(f"    mean sweeps {ri.mean():.3f}, frames equal {((rb == sb).all(1) & (ri == si)).mean():.5f}")
        assert np.array_equal(si, ri)
        assert np.array_equal(sb, rb)


def test_static_errors_and_validation():
    code = get_code("qc2304")
    llr, _ = make_frames(code, 2.0, 64, key=(62,))
    t = torch.from_numpy(llr).cuda()
    # a fresh handle has no device tables yet: refused rather than allocated
    c = cbp.Code.from_workload(code)
    say("[gpu] static scratch: tables not built")
    with pytest.raises(cbp.CbpError) as ei:
        cbp.decode_static(c, t, 20)
    assert ei.value.status == -2 and "device tables" in str(ei.value)
    ok = cbp.cbp_syndrome(c, (t < 0).to(torch.uint8))     # builds them
    torch.cuda.synchronize()
    assert ok.shape == (64,)
    # input check through the scratch word
    bad = t.clone()
    bad[5, 17] = float("nan")
    say("[gpu] static scratch: validate")
    with pytest.raises(cbp.CbpError) as ei:
        cbp.decode_static(c, bad, 20, validate=True)
    assert ei.value.status == -1 and "frame 5" in str(ei.value)
    rb, ri = cbp.decode(c, t, 20)
    sb, si = cbp.decode_static(c, t, 20, validate=True)
    torch.cuda.synchronize()
    assert torch.equal(rb, sb) and torch.equal(ri, si)
    # a code whose smallest unit of work exceeds the scratch: 64 frames of the
    # n = 26112 code on the sparse kernel need more than 64 MiB
    big = get_code("qc26112")
    cb = cbp.Code.from_workload(big)
    lb, _ = make_frames(big, 1.0, 4, key=(63,))
    tb = torch.from_numpy(lb).cuda()
    cbp.cbp_syndrome(cb, (tb < 0).to(torch.uint8))
    torch.cuda.synchronize()
    say("[gpu] static scratch: over the limit")
    with pytest.raises(cbp.CbpError) as ei:
        cbp.decode_static(cb, tb, 5, kernel="sparse")
    assert ei.value.status == -2 and "static scratch" in str(ei.value)
    # bad decoder index through the raw entry point
    assert cbp.lib().cbp_decode_static(c.handle, 7, None, None, None, 1, 1, None, None) == -1
