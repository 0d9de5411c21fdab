"""Pins of the oracle's default hard decision, its stopping rules and the sweep
indexing of the unrolled decoder's weights, against references written here.

The reference for CBP's decisions is a textbook layered BP (tanh form of the
check rule, rows in index order) that shares nothing with the oracle's
check-belief recursion.  Sec. IV-B derives CBP from layered BP (eqs. equ_s4e9,
equ_s4e10, equ_s4e14, equ_s4e20): when row c_i visits v, the posterior
Lambda = Q_v + R_new(c_j -> v) that CBP forms in its V2C phase is the layered
posterior of v as left by v's previous row c_j, i.e. layered BP's posterior of
v just before row c_i reads it (the channel LLR before v's first row).  So:

* Step 3's decision (x_v from the V2C phase of v's last visit in the sweep)
  is layered BP's posterior of v just before v's last row of that sweep;
* the syndrome test runs on those decisions ([L < 0] before the first sweep);
* Step 2(3)'s run counter advances on a row whose new V2C messages have a
  positive sign product (that is the sign of Omega_ci, eq. equ_s4e21) and
  whose V2C-phase decisions flip no bit, and resets otherwise; M such rows in
  a row, across sweep boundaries, stop the decoder right after the last one.

The trajectory reference below records exactly those quantities, and the
tests require the oracle's bits and iteration counts to equal them.
"""
import numpy as np
import pytest

import oracle
from paper_2305_05286_amd.workload import get_code, make_frames

from helpers import code_from_dense, hamming_H

LMAX = oracle.LMAX
A = oracle.phi(LMAX)


def _sign(x):
    return np.where(x >= 0, 1.0, -1.0)


def lbp_trajectory_decisions(code, llr, max_iter, stop, rule="tanh", alpha=0.75):
    """Textbook layered BP over a batch of frames, returning the decisions, the
    sweep counts and the rows processed that CBP's default decision rule and
    stopping rule `stop` ("syndrome" or "paper") must give.

    Check rule "tanh": R(c -> v) = 2 atanh(prod over the row's other edges of
    tanh(q_w / 2)), the V2C magnitudes |q| clamped to [phi(LMAX), LMAX];
    "nms": alpha * prod of the other signs * min of the other min(|q_w|, LMAX)
    (the layered form of Sec. IV-D's min-sum CBP).  Rows in index order,
    q = Lambda - R(c, v) and Lambda = q + R_new (Sec. II-B)."""
    B, N = llr.shape
    M = code.M
    rp, ci = code.row_ptr, code.col_idx
    lam = llr.astype(np.float64).copy()
    R = np.zeros((B, code.E))
    x = (llr < 0).astype(np.uint8)           # [L < 0]
    out_bits = np.zeros((B, N), np.uint8)
    out_it = np.full(B, -1, np.int32)
    out_rows = np.zeros(B, np.int64)

    def syndrome_zero(bits):
        ok = np.ones(B, bool)
        for i in range(M):
            ok &= (np.bitwise_xor.reduce(bits[:, ci[rp[i]:rp[i + 1]]], axis=1) == 0)
        return ok

    if stop == "syndrome":
        z = syndrome_zero(x)
        out_bits[z] = x[z]
        out_it[z] = 0
    run = np.zeros(B, np.int64)
    for t in range(1, max_iter + 1):
        for i in range(M):
            e = np.arange(rp[i], rp[i + 1])
            vs = ci[e]
            before = lam[:, vs]                  # layered posterior before row i reads it
            nx = (before < 0).astype(np.uint8)   # the V2C-phase decision at this visit
            flip = (nx != x[:, vs]).any(axis=1)
            x[:, vs] = nx
            q = before - R[:, e]
            d = len(e)
            rn = np.empty((B, d))
            if rule == "tanh":
                qc = _sign(q) * np.clip(np.abs(q), A, LMAX)
                th = np.tanh(qc / 2.0)
                for k in range(d):
                    p = np.ones(B)
                    for m in range(d):
                        if m != k:
                            p = p * th[:, m]
                    rn[:, k] = 2.0 * np.arctanh(p)
            else:
                mag = np.minimum(np.abs(q), LMAX)
                for k in range(d):
                    others = [m for m in range(d) if m != k]
                    rn[:, k] = (alpha * np.prod(_sign(q[:, others]), axis=1)
                                * np.min(mag[:, others], axis=1))
            lam[:, vs] = q + rn
            R[:, e] = rn
            if stop == "paper":
                good = (np.prod(_sign(q), axis=1) > 0) & ~flip
                run = np.where(good, run + 1, 0)
                hit = (run >= M) & (out_it < 0)
                out_bits[hit] = x[hit]
                out_it[hit] = t
                out_rows[hit] = (t - 1) * M + i + 1
        if stop == "syndrome":
            z = syndrome_zero(x) & (out_it < 0)
            out_bits[z] = x[z]
            out_it[z] = t
            out_rows[z] = t * M
    rest = out_it < 0
    out_bits[rest] = x[rest]
    out_it[rest] = max_iter
    out_rows[rest] = max_iter * M
    return out_bits, out_it, out_rows


def _hamming_with_redundant_row():
    H = hamming_H(4)
    return code_from_dense(np.vstack([H, H[0] ^ H[2]]), name="hamming15_red")


CODES = [("reg36_n96", 1.5, 400, 30), ("reg36_n96", 2.5, 400, 30),
         ("qc_t64s", 1.5, 200, 30), ("qc_t16", 1.0, 300, 20), ("hamming15", 3.0, 400, 20)]


def _code(name):
    return _hamming_with_redundant_row() if name == "hamming15" else get_code(name)


def _frames(code, snr, B, key):
    if code.name == "hamming15_red":
        rng = np.random.default_rng(key)
        s2 = 1.0 / (2.0 * (11 / 15) * 10 ** (snr / 10))
        # all-zero codeword; BP is symmetric in the codeword (pinned elsewhere)
        return ((2.0 / s2) * (1.0 + np.sqrt(s2) * rng.normal(size=(B, code.N)))).astype(np.float32)
    llr, _ = make_frames(code, snr, B, key=key)
    return llr


@pytest.mark.parametrize("name,snr,B,max_iter", CODES, ids=[f"{c[0]}-{c[1]}" for c in CODES])
def test_default_decision_and_syndrome_stop_equal_layered_trajectory(name, snr, B, max_iter):
    """hd_mode 0 (Step 3's V2C-phase decision) with the syndrome stop."""
    code = _code(name)
    llr = _frames(code, snr, B, (71, int(snr * 100)))
    ref_bits, ref_it, _ = lbp_trajectory_decisions(code, llr, max_iter, "syndrome")
    o = oracle.decode(code, llr, max_iter, "cbp", hd_mode=0, stop_rule=0)
    assert np.array_equal(o["iters"], ref_it)
    assert np.array_equal(o["bits"], ref_bits)
    # the pin has teeth: some frames need several sweeps, and the V2C-phase
    # decisions differ from the flushed (layered) posterior's somewhere
    assert (ref_it >= 2).sum() >= 10
    flushed = oracle.decode(code, llr, max_iter, "cbp", hd_mode=1, stop_rule=0)
    assert not (np.array_equal(flushed["iters"], ref_it) and np.array_equal(flushed["bits"], ref_bits))


@pytest.mark.parametrize("name,snr,B,max_iter", CODES, ids=[f"{c[0]}-{c[1]}" for c in CODES])
def test_paper_stop_rule_equals_run_counter_on_layered_trajectory(name, snr, B, max_iter):
    """stop_rule 1 (Step 2(3), eq. equ_s4e24, N read as M) with hd_mode 0."""
    code = _code(name)
    llr = _frames(code, snr, B, (72, int(snr * 100)))
    ref_bits, ref_it, ref_rows = lbp_trajectory_decisions(code, llr, max_iter, "paper")
    o = oracle.decode(code, llr, max_iter, "cbp", hd_mode=0, stop_rule=1)
    assert np.array_equal(o["iters"], ref_it)
    assert np.array_equal(o["bits"], ref_bits)
    col_deg = np.bincount(code.col_idx, minlength=code.N)
    if col_deg.min() >= 2:
        assert (ref_it < max_iter).sum() >= B // 4      # the rule does stop frames
    # (with degree-1 columns the rule may stop nothing: such a variable's V2C
    # message is its channel LLR, since Q = Lambda - R with R the message just
    # stored, so a wrong channel sign can hold its row's Omega below zero; on
    # qc_t64s, with 64 such columns, no frame stops within 30 sweeps)
    # the run needs M rows, so no frame stops within its first sweep's rows
    # before the last one, and no stop comes without a full sweep of rows
    assert (ref_rows[ref_it < max_iter] >= code.M).all()


def test_paper_stop_rule_mid_sweep_stop_is_exercised():
    """The stopping row can fall inside a sweep; then the decisions are the ones
    right after it (later rows of that sweep have not run) and the sweep it
    falls in is counted.  The pins above cover such frames: check that they do
    occur, and that their decisions differ from the ones at the end of the
    sweep on some frame."""
    code = get_code("reg36_n96")
    llr = _frames(code, 1.5, 400, (73, 150))
    ref_bits, ref_it, ref_rows = lbp_trajectory_decisions(code, llr, 30, "paper")
    o = oracle.decode(code, llr, 30, "cbp", stop_rule=1)
    assert np.array_equal(o["iters"], ref_it) and np.array_equal(o["bits"], ref_bits)
    mid = (ref_it < 30) & (ref_rows % code.M != 0)
    assert mid.sum() >= 20
    assert (ref_it[mid] == (ref_rows[mid] + code.M - 1) // code.M).all()


@pytest.mark.parametrize("stop", ["syndrome", "paper"])
@pytest.mark.parametrize("name,snr", [("reg36_n96", 2.0), ("qc_t16", 1.5)])
def test_min_sum_cbp_decisions_equal_layered_min_sum_trajectory(name, snr, stop):
    """The min-sum CBP (Sec. IV-D, eqs. equ_s4e18xx / equ_s4e21xx) with its
    default decision and either stopping rule, against layered normalized
    min-sum followed row by row.  Min and sign are exact, so the two must agree
    bit for bit."""
    code = get_code(name)
    llr = _frames(code, snr, 300, (74, int(snr * 100)))
    ref_bits, ref_it, _ = lbp_trajectory_decisions(code, llr, 30, stop, rule="nms", alpha=0.75)
    o = oracle.decode(code, llr, 30, "cbp_nms", alpha=0.75, stop_rule=0 if stop == "syndrome" else 1)
    assert np.array_equal(o["iters"], ref_it) and np.array_equal(o["bits"], ref_bits)
    assert (ref_it >= 2).sum() >= 10 and (ref_it < 30).sum() >= 50


# ---- unrolled decoder: which sweep's weights reach the output -------------------

def _f(w, b, x):
    """The weighted B2V message sgn(x) max(w |x| - b, 0)."""
    return np.sign(x) * np.maximum(w * np.abs(x) - b, 0.0)


def test_unrolled_first_sweep_weights_reach_output_closed_form():
    """Three degree-2 checks sharing variable v0: rows {v0, v1}, {v0, v2}, {v0, v3}.
    A degree-2 check passes the other input unchanged (2 atanh(tanh(y/2)) = y), so
    two sweeps can be followed by hand (each variable its own weight group g):

      sweep 1, row 2 stores R(c1 -> v0) = f_1,0(L2)
      sweep 2, row 0 forms Q_v0 = L0 + R(c1 -> v0) + R(c2 -> v0) with
               R(c2 -> v0) = f_2,0(L3) stored at that visit
      output   o_v1 = L1 + f_2,1(L0 + f_1,0(L2) + f_2,0(L3))
               o_v0 = L0 + f_2,0(L1) + f_2,0(L2) + f_2,0(L3)
               o_v2 = L2 + f_2,2(L0 + f_2,0(L1) + f_2,0(L3))
               o_v3 = L3 + f_2,3(L0 + f_2,0(L1) + f_2,0(L2))

    with f_t,g(x) = sgn(x) max(w_t[g] |x| - beta_t[g], 0), w_t and beta_t the
    weights of sweep t (rows t - 1 of the arrays).  o_v1 carries the first
    sweep's weight of v0's group, so a slip between sweep t's weights and sweep
    t - 1's changes it.  All magnitudes stay inside [phi(LMAX), LMAX]."""
    H = np.array([[1, 1, 0, 0], [1, 0, 1, 0], [1, 0, 0, 1]], np.uint8)
    code = code_from_dense(H)
    rng = np.random.default_rng(44)
    llr = (rng.choice([-1, 1], size=(40, 4)) * rng.uniform(0.5, 4.0, size=(40, 4))).astype(np.float32)
    w = np.array([[0.6, 1.1, 0.9, 1.3], [1.4, 0.7, 1.2, 0.8]])
    beta = np.array([[0.1, 0.05, 0.2, 0.0], [0.3, 0.15, 0.0, 0.25]])
    o = oracle.unrolled(code, llr, w, beta, grp=np.arange(4))
    L = llr.astype(np.float64)
    f = lambda t, g, x: _f(w[t, g], beta[t, g], x)
    e1 = L[:, 1] + f(1, 1, L[:, 0] + f(0, 0, L[:, 2]) + f(1, 0, L[:, 3]))
    e0 = L[:, 0] + f(1, 0, L[:, 1]) + f(1, 0, L[:, 2]) + f(1, 0, L[:, 3])
    e2 = L[:, 2] + f(1, 2, L[:, 0] + f(1, 0, L[:, 1]) + f(1, 0, L[:, 3]))
    e3 = L[:, 3] + f(1, 3, L[:, 0] + f(1, 0, L[:, 1]) + f(1, 0, L[:, 2]))
    for got, exp in zip(o.T, (e0, e1, e2, e3)):
        assert np.allclose(got, exp, rtol=1e-9, atol=1e-9)
    # the same expression with the second sweep's weight in place of the first differs
    slip = L[:, 1] + f(1, 1, L[:, 0] + f(1, 0, L[:, 2]) + f(1, 0, L[:, 3]))
    assert np.abs(slip - e1).max() > 0.1
