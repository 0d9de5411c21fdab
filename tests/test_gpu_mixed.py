"""Mixed-code batches (cbp_mix_*) through the C ABI.

Frames of several QC codes (five rates, several lifting sizes, per-frame Eb/N0) are
decoded in one persistent launch.  Checked against the FP64 oracle per code, against
the single-code streamed decoder (bit-identical: same kernel arithmetic), and for the
plan's schedule, autotuner, malformed frames and HIP graph replays.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2305_05286_amd import cbp
from paper_2305_05286_amd.workload import make_mixed_batch, mixed_family

from helpers import syndrome

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PARITY = 0.999


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_family():
    return [c for c in mixed_family() if c.Z in (16, 32, 64)]


def to_dev(b):
    return (torch.from_numpy(b["llr"]).cuda(), torch.from_numpy(b["code"]).cuda(),
            torch.from_numpy(b["offset"]).cuda())


def frame_bits(bits, b, codes, f):
    o = b["offset"][f]
    return bits[o:o + codes[b["code"][f]].N]


def split_by_code(b, codes, arr=None):
    """{code index: (frame ids, [n, N] array of that code's frames from arr (default llr))}"""
    arr = b["llr"] if arr is None else arr
    out = {}
    for c, code in enumerate(codes):
        fr = np.nonzero(b["code"] == c)[0]
        if fr.size:
            idx = b["offset"][fr][:, None] + np.arange(code.N)[None, :]
            out[c] = (fr, arr[idx])
    return out


@pytest.mark.parametrize("algo", ["cbp", "cbp_nms", "lbp_nms", "fbp_nms"])
def test_mixed_matches_oracle(algo):
    codes = small_family()
    b = make_mixed_batch(codes, 900, key=(31, 1))
    mix = cbp.Mix([cbp.Code.from_workload(c) for c in codes])
    say(f"[gpu] mixed {algo}: {len(codes)} codes, 900 frames, schedule {mix.schedule}")
    bits, iters = mix.decode(*to_dev(b), 20, algo)
    torch.cuda.synchronize()
    bits, iters = bits.cpu().numpy(), iters.cpu().numpy()
    same_it, same_bits, conv_n, n = 0, 0, 0, 0
    for c, (fr, llr) in split_by_code(b, codes).items():
        o = oracle.decode(codes[c], llr, 20, algo)
        gb = np.stack([frame_bits(bits, b, codes, f) for f in fr])
        gi = iters[fr]
        conv = o["iters"] < 20
        same_it += (gi == o["iters"]).sum()
        same_bits += ((gb == o["bits"]).all(1) & conv).sum()
        conv_n += conv.sum()
        n += fr.size
        stopped = gi < 20
        assert (syndrome(codes[c], gb[stopped]) == 0).all()
    say(f"    iterations equal {same_it / n:.4f}, decisions equal on decoded frames "
        f"{same_bits / max(conv_n, 1):.4f} ({conv_n} of {n} decoded)")
    assert same_it / n >= PARITY
    assert same_bits / max(conv_n, 1) >= PARITY


def test_mixed_equals_single_code_decoder():
    """Every frame of a mixed batch decodes exactly as in a one-code streamed launch."""
    codes = list(mixed_family())
    b = make_mixed_batch(codes, 1500, key=(31, 2))
    handles = [cbp.Code.from_workload(c) for c in codes]
    mix = cbp.Mix(handles)
    say(f"[gpu] mixed vs single-code: {len(codes)} codes, 1500 frames, schedule {mix.schedule}")
    bits, iters = mix.decode(*to_dev(b), 25, "cbp")
    torch.cuda.synchronize()
    bits, iters = bits.cpu().numpy(), iters.cpu().numpy()
    for c, (fr, llr) in split_by_code(b, codes).items():
        sb, si = cbp.cbp_decode(handles[c], torch.from_numpy(np.ascontiguousarray(llr)).cuda(), 25,
                                kernel="qc_stream")
        torch.cuda.synchronize()
        gb = np.stack([frame_bits(bits, b, codes, f) for f in fr])
        assert (iters[fr] == si.cpu().numpy()).all(), codes[c].name
        assert (gb == sb.cpu().numpy()).all(), codes[c].name


@pytest.mark.parametrize("algo", ["cbp", "cbp_nms", "lbp_nms", "fbp_nms"])
def test_mixed_lds_part_equals_streamed(algo):
    """With lds_groups_per_cu > 0 the codes whose frame fits half a CU's LDS are decoded staged
    in LDS on a second stream beside the streamed launch; with 0 every code streams.  Both give
    the same decisions and sweep counts bit for bit, and so does a graph replay of the split
    launch."""
    codes = list(mixed_family())
    b = make_mixed_batch(codes, 3000, key=(31, 3))
    mix = cbp.Mix([cbp.Code.from_workload(c) for c in codes])
    lanes, groups = mix.schedule[:2]
    say(f"[gpu] mixed {algo}: LDS part against all streamed")
    mix.schedule = (lanes, 3, 0)
    sbits, siters = mix.decode(*to_dev(b), 25, algo)
    torch.cuda.synchronize()
    for lg in (1, 2):
        mix.schedule = (lanes, 3, lg)
        bits, iters = mix.decode(*to_dev(b), 25, algo)
        torch.cuda.synchronize()
        assert np.array_equal(iters.cpu().numpy(), siters.cpu().numpy()), lg
        assert np.array_equal(bits.cpu().numpy(), sbits.cpu().numpy()), lg
    # captured: the fork to the second stream and the join are part of the graph
    mix.schedule = (lanes, 3, 1)
    llr, fc, fo = to_dev(b)
    gbits = torch.full_like(bits, 7)
    giters = torch.full_like(iters, -7)
    g, _, _ = mix.graph(llr, fc, fo, 25, algo, out=(gbits, giters))
    for rep in range(3):
        gbits.fill_(7)
        giters.fill_(-7)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(giters.cpu().numpy(), siters.cpu().numpy()), rep
        assert np.array_equal(gbits.cpu().numpy(), sbits.cpu().numpy()), rep


@pytest.mark.parametrize("subset", ["all_fit", "none_fit"])
def test_mixed_lds_part_subsets_and_small_batches(subset):
    """Plans whose codes all fit the LDS-staged part (the streamed launch then finds every queue
    exhausted) or none do (no side launch), batches of 1, 2 and 5 frames (fewer than the
    workgroups), malformed frames and an empty batch: the same results with and without the
    LDS-staged part."""
    codes = [c for c in mixed_family() if (c.Z <= 128) == (subset == "all_fit")]
    mix = cbp.Mix([cbp.Code.from_workload(c) for c in codes])
    lanes = mix.schedule[0]
    for n in (1, 2, 5, 700):
        b = make_mixed_batch(codes, n, key=(31, 6, n))
        for algo in ("cbp", "lbp_nms", "fbp_nms"):
            say(f"[gpu] mixed LDS part, {subset}: {algo}, {n} frames")
            mix.schedule = (lanes, 2, 0)
            sbits, siters = mix.decode(*to_dev(b), 25, algo)
            torch.cuda.synchronize()
            for lg in (1, 2):
                mix.schedule = (lanes, 2, lg)
                bits, iters = mix.decode(*to_dev(b), 25, algo)
                torch.cuda.synchronize()
                assert np.array_equal(iters.cpu().numpy(), siters.cpu().numpy()), (n, algo, lg)
                assert np.array_equal(bits.cpu().numpy(), sbits.cpu().numpy()), (n, algo, lg)
    # malformed frames are rejected before either launch sees a queue
    b = make_mixed_batch(codes, 300, key=(31, 7))
    llr, fc, fo = to_dev(b)
    fc[4] = -1
    fo[77] = llr.numel() - 3
    out = {}
    for lg in (0, 2):
        say(f"[gpu] mixed LDS part, {subset}: malformed frames, lds_groups_per_cu {lg}")
        mix.schedule = (lanes, 2, lg)
        bits = torch.full((llr.numel(),), 7, dtype=torch.uint8, device="cuda")
        iters = torch.zeros(300, dtype=torch.int32, device="cuda")
        mix.decode(llr, fc, fo, 25, "cbp", out=(bits, iters))
        torch.cuda.synchronize()
        out[lg] = (bits.cpu().numpy(), iters.cpu().numpy())
        assert out[lg][1][4] == -1 and out[lg][1][77] == -1
        assert (np.delete(out[lg][1], [4, 77]) >= 0).all()
    assert np.array_equal(out[0][0], out[2][0]) and np.array_equal(out[0][1], out[2][1])
    # empty batch
    e32 = torch.empty(0, dtype=torch.int32, device="cuda")
    e64 = torch.empty(0, dtype=torch.int64, device="cuda")
    _, iters = mix.decode(torch.zeros(16, dtype=torch.float32, device="cuda"), e32, e64, 10, "cbp",
                          workspace=torch.empty(0, dtype=torch.uint8, device="cuda"))
    assert iters.numel() == 0


def test_mixed_two_streams_share_the_plan():
    """Two decodes with one plan on two streams at once, the LDS-staged part on: both use the
    plan's side stream and fork / join events, taking turns on them, and each gives the result
    of a decode on its own."""
    codes = list(mixed_family())
    mix = cbp.Mix([cbp.Code.from_workload(c) for c in codes])
    mix.schedule = (mix.schedule[0], 2, 2)
    ba, bb = make_mixed_batch(codes, 2000, key=(31, 8)), make_mixed_batch(codes, 1500, key=(31, 9))
    da, db = to_dev(ba), to_dev(bb)
    say("[gpu] mixed: one plan on two streams")
    ref_a = mix.decode(*da, 25, "cbp")
    ref_b = mix.decode(*db, 25, "cbp")
    out_a = (torch.empty_like(ref_a[0]), torch.empty_like(ref_a[1]))
    out_b = (torch.empty_like(ref_b[0]), torch.empty_like(ref_b[1]))
    wa = torch.empty(mix.workspace_size(2000, "cbp"), dtype=torch.uint8, device="cuda")
    wb = torch.empty(mix.workspace_size(1500, "cbp"), dtype=torch.uint8, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(3):
        for o in (out_a, out_b):
            o[0].fill_(7)
            o[1].fill_(-7)
        torch.cuda.synchronize()
        mix.decode(*da, 25, "cbp", workspace=wa, out=out_a, stream=s1)
        mix.decode(*db, 25, "cbp", workspace=wb, out=out_b, stream=s2)
        torch.cuda.synchronize()
        assert torch.equal(out_a[0], ref_a[0]) and torch.equal(out_a[1], ref_a[1]), rep
        assert torch.equal(out_b[0], ref_b[0]) and torch.equal(out_b[1], ref_b[1]), rep


def test_mixed_malformed_frames_are_skipped():
    codes = small_family()[:4]
    b = make_mixed_batch(codes, 200, key=(31, 3))
    llr, fc, fo = to_dev(b)
    bad_code = [3, 50]
    bad_off = [10, 120]
    fc[bad_code[0]] = -1
    fc[bad_code[1]] = len(codes)
    fo[bad_off[0]] = llr.numel() - 10          # runs past the end
    fo[bad_off[1]] = -5
    mix = cbp.Mix([cbp.Code.from_workload(c) for c in codes])
    bits = torch.full((llr.numel(),), 7, dtype=torch.uint8, device="cuda")
    iters = torch.zeros(200, dtype=torch.int32, device="cuda")
    say("[gpu] mixed malformed frames")
    mix.decode(llr, fc, fo, 20, "cbp", out=(bits, iters))
    torch.cuda.synchronize()
    it = iters.cpu().numpy()
    for f in bad_code + bad_off:
        assert it[f] == -1
    good = np.setdiff1d(np.arange(200), bad_code + bad_off)
    assert (it[good] >= 0).all()
    # a frame whose code index is invalid leaves its bytes untouched
    bb = bits.cpu().numpy()
    o = b["offset"][bad_code[0]]
    assert (bb[o:o + codes[b["code"][bad_code[0]]].N] == 7).all()


def test_mixed_schedules_tuner_and_graph_replays():
    codes = list(mixed_family())
    mix = cbp.Mix([cbp.Code.from_workload(c) for c in codes])
    lanes0, g0, l0 = mix.schedule
    assert lanes0 % 384 == 0 and g0 == 0 and l0 == 0
    b = make_mixed_batch(codes, 3000, key=(31, 4))
    llr, fc, fo = to_dev(b)
    say("[gpu] mixed schedules")
    ref_bits, ref_iters = mix.decode(llr, fc, fo, 25, "cbp")
    for sched in [(lanes0, 1), (2 * lanes0, 0), (lanes0, 2), (lanes0, 2, 1), (lanes0, 3, 2)]:
        mix.schedule = sched
        bb, ii = mix.decode(llr, fc, fo, 25, "cbp")
        assert torch.equal(bb, ref_bits) and torch.equal(ii, ref_iters), sched
    with pytest.raises(cbp.CbpError):
        mix.schedule = (lanes0 + 16, 0)       # not a multiple of every Z
    say("[gpu] mixed autotuner")
    best, ms = mix.tune(llr, fc, fo, 25, "cbp")
    assert mix.schedule == best and best[0] % lanes0 == 0 and best[1] >= 1 and ms > 0
    bb, ii = mix.decode(llr, fc, fo, 25, "cbp")
    assert torch.equal(bb, ref_bits) and torch.equal(ii, ref_iters)

    say("[gpu] mixed graph replays")
    llr_g, fc_g, fo_g = llr.clone(), fc.clone(), fo.clone()
    graph, gbits, giters = mix.graph(llr_g, fc_g, fo_g, 25, "cbp")
    for rep in range(4):
        # refill the captured input in place: the same frames at another SNR
        llr_g.copy_(llr * (0.7 + 0.15 * rep))
        graph.launch()
        torch.cuda.synchronize()
        eb, ei = mix.decode(llr_g, fc_g, fo_g, 25, "cbp")   # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(gbits, eb) and torch.equal(giters, ei), rep


def test_mixed_validate_option():
    """opts.validate on a mixed batch: a NaN is reported by its flat index; a graph cannot
    capture the scan (CBP_EUNSUPPORTED); finite inputs decode as without it."""
    codes = small_family()[:3]
    b = make_mixed_batch(codes, 120, key=(31, 5))
    llr, fc, fo = to_dev(b)
    mix = cbp.Mix([cbp.Code.from_workload(c) for c in codes])
    say("[gpu] mixed validate")
    rb, ri = mix.decode(llr, fc, fo, 20, "cbp")
    vb, vi = mix.decode(llr, fc, fo, 20, "cbp", validate=True)
    assert torch.equal(rb, vb) and torch.equal(ri, vi)
    pos = int(b["offset"][40]) + 3
    bad = llr.clone()
    bad[pos] = float("inf")
    with pytest.raises(cbp.CbpError) as ei:
        mix.decode(bad, fc, fo, 20, "cbp", validate=True)
    assert ei.value.status == cbp.CBP_EINVAL and f"element {pos} is" in str(ei.value)
    with pytest.raises(cbp.CbpError) as ei:
        mix.graph(llr.clone(), fc.clone(), fo.clone(), 20, "cbp", validate=True)
    assert ei.value.status == cbp.CBP_EUNSUPPORTED


def test_mixed_empty_batch():
    codes = small_family()[:2]
    mix = cbp.Mix([cbp.Code.from_workload(c) for c in codes])
    e32 = torch.empty(0, dtype=torch.int32, device="cuda")
    e64 = torch.empty(0, dtype=torch.int64, device="cuda")
    llr = torch.zeros(16, dtype=torch.float32, device="cuda")
    bits, iters = mix.decode(llr, e32, e64, 10, "cbp", workspace=torch.empty(0, dtype=torch.uint8, device="cuda"))
    assert iters.numel() == 0


def test_mixed_full_size_sampled():
    """The 65536-frame workload the benchmark times, sampled frames against the oracle."""
    codes = list(mixed_family())
    b = make_mixed_batch(codes, 65536, key=(2026, 7), return_codewords=False)
    mix = cbp.Mix([cbp.Code.from_workload(c) for c in codes])
    say(f"[gpu] mixed full size: 65536 frames, {b['llr'].size} LLRs")
    bits, iters = mix.decode(*to_dev(b), 25, "cbp")
    torch.cuda.synchronize()
    bits, iters = bits.cpu().numpy(), iters.cpu().numpy()
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(65536, size=400, replace=False))
    agree_it, agree_bits, dec = 0, 0, 0
    for f in sample:
        code = codes[b["code"][f]]
        llr = b["llr"][b["offset"][f]:b["offset"][f] + code.N][None, :]
        o = oracle.decode(code, llr, 25, "cbp")
        agree_it += int(o["iters"][0] == iters[f])
        if o["iters"][0] < 25:
            dec += 1
            agree_bits += int((o["bits"][0] == frame_bits(bits, b, codes, f)).all())
    say(f"    sampled 400: iterations equal {agree_it}, decisions equal {agree_bits} of {dec} decoded")
    assert agree_it >= 399 and agree_bits >= dec - 1
