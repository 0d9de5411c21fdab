"""Unrolled differentiable CBP (cbp_unrolled_*) through the C ABI.

Forward: against the FP64 oracle's weighted unrolled CBP, and (unit weights) against the
streamed decoder's flushed posterior.  Backward: the hand-written adjoint against FP64
central finite differences of the oracle's forward; determinism; a short training run.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2305_05286_amd import cbp
from paper_2305_05286_amd.workload import get_code, make_frames

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def z72_code():
    """A QC code whose frame (Z = 72 lanes) does not fill whole waves."""
    from paper_2305_05286_amd.workload import make_qc_code, qc_pattern_dualdiag
    return make_qc_code("qc_t72", qc_pattern_dualdiag(4, [3, 3, 2, 2], seed=4), 72, seed=9, kind="qc_dualdiag")


def gpu_forward(code_w, llr, w, beta):
    c = cbp.Code.from_workload(code_w)
    t = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
    wt = torch.tensor(w, dtype=torch.float32, device="cuda")
    bt = torch.tensor(beta, dtype=torch.float32, device="cuda")
    out = cbp.unrolled_cbp(c, t, wt, bt, w.shape[0])
    torch.cuda.synchronize()
    return out.cpu().numpy()


def bce64(o, c):
    """mean over bits of c * softplus(o) + (1 - c) * softplus(-o)  (o > 0 favours bit 0)"""
    return float(np.mean(c * np.logaddexp(0.0, o) + (1 - c) * np.logaddexp(0.0, -o)))


@pytest.mark.parametrize("name", ["qc_t64s", "qc2304", "qc_t72"])
def test_unit_weights_equal_streamed_flushed_posterior(name):
    code = get_code(name) if name != "qc_t72" else z72_code()
    T = 5
    llr, _ = make_frames(code, 1.75, 64, key=(51,))
    nb = code.N // code.Z
    say(f"[gpu] unrolled unit weights {name}")
    o = gpu_forward(code, llr, np.ones((T, nb)), np.zeros((T, nb)))
    c = cbp.Code.from_workload(code)
    t = torch.from_numpy(llr).cuda()
    _, _, dump = cbp.cbp_decode(c, t, T, kernel="qc_stream", stop_rule=2, dump_sweep=T, dump_frames=64)
    lam = dump["lam"].cpu().numpy()
    say(f"    identical {np.mean(o == lam):.5f}, max rel {np.max(np.abs(o - lam) / np.maximum(np.abs(lam), 1)):.2e}")
    assert np.max(np.abs(o - lam) / np.maximum(np.abs(lam), 1)) <= 1e-6


@pytest.mark.parametrize("name", ["qc_t64s", "qc2304"])
def test_forward_matches_fp64_oracle(name):
    code = get_code(name)
    T, nb = 6, code.N // code.Z
    rng = np.random.default_rng(52)
    w = rng.uniform(0.6, 1.4, size=(T, nb))
    beta = rng.uniform(0.0, 0.4, size=(T, nb))
    llr, _ = make_frames(code, 2.0, 64, key=(52,))
    say(f"[gpu] unrolled forward vs oracle {name}")
    o = gpu_forward(code, llr, w.astype(np.float32), beta.astype(np.float32))
    ref = oracle.unrolled(code, llr, w.astype(np.float32).astype(np.float64),
                          beta.astype(np.float32).astype(np.float64))
    err = np.abs(o - ref) / np.maximum(np.abs(ref), 1.0)
    say(f"    max rel {err.max():.2e}, within 1e-4: {np.mean(err <= 1e-4):.5f}")
    # every soft output within the FP32 message bar of FP64
    assert err.max() <= 1e-4


@pytest.mark.parametrize("name", ["qc_t16", "qc_t72"])
def test_gradients_match_fp64_finite_differences(name):
    code = get_code(name) if name != "qc_t72" else z72_code()
    T, nb = 3, code.N // code.Z
    rng = np.random.default_rng(53)
    w = rng.uniform(0.7, 1.3, size=(T, nb)).astype(np.float32).astype(np.float64)
    beta = rng.uniform(0.01, 0.1, size=(T, nb)).astype(np.float32).astype(np.float64)
    llr, cw = make_frames(code, 2.0, 4, key=(53,))
    cwf = cw.astype(np.float64)

    # GPU: loss in torch (FP64 on the soft output), gradients through the adjoint kernel
    c = cbp.Code.from_workload(code)
    lt = torch.from_numpy(llr).cuda().requires_grad_(True)
    wt = torch.tensor(w, dtype=torch.float32, device="cuda", requires_grad=True)
    bt = torch.tensor(beta, dtype=torch.float32, device="cuda", requires_grad=True)
    o = cbp.unrolled_cbp(c, lt, wt, bt, T)
    ct = torch.from_numpy(cwf).cuda()
    od = o.double()
    loss = (ct * torch.nn.functional.softplus(od) + (1 - ct) * torch.nn.functional.softplus(-od)).mean()
    loss.backward()
    gw, gb, gl = wt.grad.cpu().numpy(), bt.grad.cpu().numpy(), lt.grad.cpu().numpy()

    # FP64 central differences of the oracle's forward
    def L(w_, b_, llr_=llr):
        return bce64(oracle.unrolled(code, llr_, w_, b_), cwf)
    h = 1e-5
    fw, fb = np.zeros_like(w), np.zeros_like(beta)
    for t in range(T):
        for b in range(nb):
            e = np.zeros_like(w)
            e[t, b] = h
            fw[t, b] = (L(w + e, beta) - L(w - e, beta)) / (2 * h)
            fb[t, b] = (L(w, beta + e) - L(w, beta - e)) / (2 * h)
    hl = 2.0 ** -10  # exactly representable perturbation of the float32 LLRs
    idx = [(f, v) for f in range(4) for v in rng.choice(code.N, size=4, replace=False)]
    fl = []
    for f, v in idx:
        lp, lm = llr.copy(), llr.copy()
        lp[f, v] += hl
        lm[f, v] -= hl
        fl.append((L(w, beta, lp) - L(w, beta, lm)) / (2 * hl))
    gl_s = np.array([gl[f, v] for f, v in idx])
    fl = np.array(fl)

    def rel(a, b):
        return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
    say(f"[gpu] unrolled gradients: rel err w {rel(gw, fw):.2e}, beta {rel(gb, fb):.2e}, "
        f"llr {rel(gl_s, fl):.2e}; |dL/dw| {np.abs(fw).max():.3e}")
    assert rel(gw, fw) < 1e-3
    assert rel(gb, fb) < 1e-3
    assert rel(gl_s, fl) < 1e-3
    for g, f in ((gw, fw), (gb, fb), (gl_s, fl)):
        assert np.all(np.abs(g - f) <= 1e-3 * np.abs(f).max() + 1e-3 * np.abs(f))


def test_gradients_at_the_training_size():
    """The configuration the decoder is trained in: the n = 2304 code, 10
    unrolled sweeps.  FP64 central differences of the oracle's forward at 24
    sampled (sweep, block-column) weights and offsets, spread over all ten
    sweeps, and 12 sampled LLRs, on 3 frames at 1.25 dB (cross-entropy 0.04;
    at 1.75 dB these frames decode with a loss of 5e-10, where the gradients
    are of order 1e-10 and measure saturation rather than the adjoint)."""
    code = get_code("qc2304")
    T, nb = 10, code.N // code.Z
    rng = np.random.default_rng(57)
    w = rng.uniform(0.7, 1.3, size=(T, nb)).astype(np.float32).astype(np.float64)
    beta = rng.uniform(0.01, 0.1, size=(T, nb)).astype(np.float32).astype(np.float64)
    llr, cw = make_frames(code, 1.25, 3, key=(57,))
    cwf = cw.astype(np.float64)
    c = cbp.Code.from_workload(code)
    lt = torch.from_numpy(llr).cuda().requires_grad_(True)
    wt = torch.tensor(w, dtype=torch.float32, device="cuda", requires_grad=True)
    bt = torch.tensor(beta, dtype=torch.float32, device="cuda", requires_grad=True)
    o = cbp.unrolled_cbp(c, lt, wt, bt, T)
    ct = torch.from_numpy(cwf).cuda()
    od = o.double()
    loss = (ct * torch.nn.functional.softplus(od) + (1 - ct) * torch.nn.functional.softplus(-od)).mean()
    loss.backward()
    gw, gb, gl = wt.grad.cpu().numpy(), bt.grad.cpu().numpy(), lt.grad.cpu().numpy()

    def L(w_, b_, llr_=llr):
        return bce64(oracle.unrolled(code, llr_, w_, b_), cwf)
    pairs = [(t, int(b)) for t in range(T) for b in rng.choice(nb, size=2, replace=False)][:20]
    pairs += [(T - 1, int(b)) for b in rng.choice(nb, size=4, replace=False)]
    # The loss is piecewise smooth (clamps, the ReLU of the offset); over ten
    # sweeps a step of 1e-5 can straddle a kink (two of these weights read
    # 0.2% off at 1e-5 and agree to 6 digits at 1e-6), so the steps are small.
    h = 1e-6
    fw, fb, sw, sb = [], [], [], []
    for t, b in pairs:
        e = np.zeros_like(w)
        e[t, b] = h
        fw.append((L(w + e, beta) - L(w - e, beta)) / (2 * h))
        fb.append((L(w, beta + e) - L(w, beta - e)) / (2 * h))
        sw.append(gw[t, b])
        sb.append(gb[t, b])
    hl = 2.0 ** -14  # exactly representable move of the float32 LLRs
    fl, sl = [], []
    for f in range(3):
        for v in rng.choice(code.N, size=4, replace=False):
            lp, lm = llr.copy(), llr.copy()
            lp[f, v] += hl
            lm[f, v] -= hl
            fl.append((L(w, beta, lp) - L(w, beta, lm)) / (2 * hl))
            sl.append(gl[f, v])
    fw, fb, fl, sw, sb, sl = map(np.array, (fw, fb, fl, sw, sb, sl))

    def rel(a, b):
        return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
    say(f"[gpu] unrolled gradients at T=10 on n=2304: rel err w {rel(sw, fw):.2e}, beta {rel(sb, fb):.2e}, "
        f"llr {rel(sl, fl):.2e}; |dL/dw| max {np.abs(fw).max():.3e}, sweeps with nonzero dL/dw "
        f"{sorted({t for (t, _), g in zip(pairs, fw) if g != 0})}")
    assert np.abs(fw).max() > 0 and np.abs(fl).max() > 0
    assert rel(sw, fw) < 1e-3
    assert rel(sb, fb) < 1e-3
    assert rel(sl, fl) < 1e-3


def test_backward_is_deterministic():
    code = get_code("qc2304")
    T, nb = 4, code.N // code.Z
    llr, cw = make_frames(code, 2.0, 300, key=(54,))
    c = cbp.Code.from_workload(code)
    lt = torch.from_numpy(llr).cuda()
    ct = torch.from_numpy(cw.astype(np.float32)).cuda()
    grads = []
    for _ in range(2):
        wt = torch.full((T, nb), 0.9, device="cuda", requires_grad=True)
        bt = torch.full((T, nb), 0.05, device="cuda", requires_grad=True)
        o = cbp.unrolled_cbp(c, lt, wt, bt, T)
        loss = torch.nn.functional.binary_cross_entropy_with_logits(-o, ct)
        loss.backward()
        grads.append((wt.grad.clone(), bt.grad.clone()))
    assert torch.equal(grads[0][0], grads[1][0]) and torch.equal(grads[0][1], grads[1][1])
    assert torch.isfinite(grads[0][0]).all() and grads[0][0].abs().sum() > 0


def test_second_backward_is_refused():
    """The backward pass recomputes in place on the checkpoints, so it runs once per forward."""
    code = get_code("qc_t16")
    c = cbp.Code.from_workload(code)
    llr, cw = make_frames(code, 2.0, 8, key=(56,))
    wt = torch.ones((3, code.N // code.Z), device="cuda", requires_grad=True)
    bt = torch.zeros((3, code.N // code.Z), device="cuda", requires_grad=True)
    o = cbp.unrolled_cbp(c, torch.from_numpy(llr).cuda(), wt, bt, 3)
    loss = o.square().mean()
    loss.backward(retain_graph=True)
    g1 = wt.grad.clone()
    with pytest.raises(RuntimeError, match="consumes"):
        loss.backward()
    # a fresh forward gives the same gradients again
    wt.grad = None
    o = cbp.unrolled_cbp(c, torch.from_numpy(llr).cuda(), wt, bt, 3)
    o.square().mean().backward()
    assert torch.equal(wt.grad, g1)


def test_training_lowers_the_loss():
    code = get_code("qc2304")
    c = cbp.Code.from_workload(code)
    model = cbp.unrolled_module(c, 5).cuda()
    opt = torch.optim.Adam(model.parameters(), lr=2e-2)
    vl, vc = make_frames(code, 1.75, 1024, key=(55, 0))
    vl, vc = torch.from_numpy(vl).cuda(), torch.from_numpy(vc.astype(np.float32)).cuda()

    def val():
        with torch.no_grad():
            return torch.nn.functional.binary_cross_entropy_with_logits(-model(vl), vc).item()
    before = val()
    for step in range(12):
        tl, tc = make_frames(code, 1.75, 1024, key=(55, 1 + step))
        o = model(torch.from_numpy(tl).cuda())
        loss = torch.nn.functional.binary_cross_entropy_with_logits(-o, torch.from_numpy(tc.astype(np.float32)).cuda())
        opt.zero_grad()
        loss.backward()
        opt.step()
    after = val()
    say(f"[gpu] unrolled training: validation BCE {before:.5f} -> {after:.5f}")
    assert after < before


def test_errors_and_empty_batch():
    c = cbp.Code.from_workload(get_code("reg36_n96"))
    with pytest.raises(cbp.CbpError):
        cbp.unrolled_workspace_size(c, 3, 10)
    q = cbp.Code.from_workload(get_code("qc_t16"))
    with pytest.raises(cbp.CbpError):
        cbp.unrolled_workspace_size(q, 0, 10)
    assert cbp.unrolled_workspace_size(q, 3, 0) == 0
