"""The C ABI without a GPU: the library loads, exports what include/cbp.h
declares, and its host-side validation returns the documented errors."""
import contextlib
import ctypes
import os
import re
from pathlib import Path

import numpy as np
import pytest

from paper_2305_05286_amd import cbp
from paper_2305_05286_amd.workload import get_code

ROOT = Path(__file__).resolve().parents[1]


@pytest.fixture(scope="module")
def L():
    if not cbp.LIB_PATH.exists():
        from paper_2305_05286_amd.build import build
        build(verbose=False)
    return cbp.lib()


def declared_functions():
    text = (ROOT / "include" / "cbp.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)))


def test_exports_every_declared_function(L):
    names = declared_functions()
    assert len(names) >= 12
    assert set(names) == set(cbp.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_opts_defaults_and_layout(L):
    o = cbp.Opts()
    L.cbp_opts_default(ctypes.byref(o))
    assert (o.stop_rule, o.hd_mode, o.kernel, o.dump_sweep) == (0, 0, 0, 0)
    assert o.lmax == 20.0 and o.alpha == 0.75
    # 8 x 4-byte fields, int64, 6 pointer-sized fields (C natural alignment)
    assert ctypes.sizeof(cbp.Opts) == 88 and cbp.Opts.dump_frames.offset == 32
    assert o.check_rule == 0 and o.validate == 0 and cbp.Opts.validate.offset == 28


def test_strerror_and_version(L):
    assert L.cbp_strerror(0) == b"ok"
    assert L.cbp_strerror(-1) == b"invalid argument"
    assert L.cbp_strerror(-2) == b"unsupported"
    assert cbp.version() >= 100


def test_code_handles(L):
    c = cbp.Code.from_workload(get_code("qc2304"))
    assert (c.M, c.N, c.E, c.Z) == (1152, 2304, 7296, 96)
    assert c.has_kernel("qc_reg") and c.has_kernel("sparse")
    c1 = cbp.Code.from_workload(get_code("reg36_n96"))
    assert (c1.M, c1.N, c1.E, c1.Z) == (48, 96, 288, 0)
    assert not c1.has_kernel("qc_reg")
    # same base pattern, other shifts: still the compiled pattern
    c2 = cbp.Code.from_workload(get_code("qc2304_alt"))
    assert c2.has_kernel("qc_reg")
    # a base pattern that is not compiled in
    c3 = cbp.Code.from_workload(get_code("qc26112"))
    assert not c3.has_kernel("qc_reg") and c3.has_kernel("qc_stream")
    assert not c1.has_kernel("qc_stream")
    # frame state in LDS within 160 KiB: CBP 4N + 4E + 8M + N bytes (rounded); the BP
    # decoders 4N + 4E + 8 x (rows of the largest level), flooding 4N more
    assert c.has_kernel("sparse_lds") and c1.has_kernel("sparse_lds") and not c3.has_kernel("sparse_lds")
    for algo in ("cbp", "lbp", "fbp", "lbp_nms", "fbp_nms"):
        with pytest.raises(cbp.CbpError) as e:
            cbp.workspace_size(c3, algo, 1, kernel="sparse_lds")
        assert e.value.status == cbp.CBP_EUNSUPPORTED
    # n = 8192 PEG: flooding BP (4N + 4E + 8 x 258 + 4N = 156,496 bytes) fits as well
    peg = cbp.Code.from_workload(get_code("peg_irr_n8192"))
    for algo in ("cbp", "lbp", "fbp"):
        assert cbp.workspace_size(peg, algo, 1, kernel="sparse_lds") == 256


@pytest.mark.parametrize("rp,ci,why", [
    ([0, 1, 3], [0, 1, 2], "degree"),          # row of degree 1
    ([0, 2, 4], [1, 0, 1, 2], "ascending"),    # not ascending
    ([0, 2, 4], [0, 1, 1, 5], "range"),        # column out of range
    ([0, 2, 4], [0, 1, 0, 1], "no edge"),      # column 2 unused
])
def test_csr_validation(L, rp, ci, why):
    with pytest.raises(cbp.CbpError) as ei:
        cbp.Code.from_csr(2, 3, rp, ci)
    assert ei.value.status == cbp.CBP_EINVAL


def test_qc_validation(L):
    with pytest.raises(cbp.CbpError):
        cbp.Code.from_qc(np.array([[0, 5], [1, -2]]), 4)  # -2 and 5 out of range
    h = ctypes.c_void_p()
    assert L.cbp_code_from_qc(0, 2, 4, None, ctypes.byref(h)) == cbp.CBP_EINVAL


def test_decode_argument_errors_without_gpu(L):
    c = cbp.Code.from_workload(get_code("reg36_n96"))
    o = cbp.Opts()
    L.cbp_opts_default(ctypes.byref(o))
    # NULL code
    assert L.cbp_decode(None, None, None, None, 10, 4, None, None) == cbp.CBP_EINVAL
    # batch == 0 is a no-op even with NULL buffers
    assert L.cbp_decode(c.handle, None, None, None, 10, 0, None, None) == cbp.CBP_OK
    # negative sizes
    assert L.cbp_decode(c.handle, None, None, None, -1, 0, None, None) == cbp.CBP_EINVAL
    assert L.lbp_nms_decode(c.handle, None, None, None, 5, -3, None, None) == cbp.CBP_EINVAL
    # NULL buffers with frames
    assert L.fbp_nms_decode(c.handle, None, None, None, 5, 8, None, None) == cbp.CBP_EINVAL
    # option errors are reported before any device work
    fake = ctypes.c_void_p(16)
    o.stop_rule = 1       # the paper's rule is defined for CBP only
    assert L.lbp_nms_decode(c.handle, fake, fake, fake, 5, 8, ctypes.byref(o), None) == cbp.CBP_EINVAL
    o.hd_mode = 1         # ... and with flushed decisions needs the sparse kernel
    q = cbp.Code.from_workload(get_code("qc2304"))
    assert L.cbp_decode(q.handle, fake, fake, fake, 5, 8, ctypes.byref(o), None) == cbp.CBP_EUNSUPPORTED
    o.hd_mode = 0
    o.stop_rule = 3
    assert L.cbp_decode(c.handle, fake, fake, fake, 5, 8, ctypes.byref(o), None) == cbp.CBP_EINVAL
    o.stop_rule = 0
    o.kernel = cbp.KERNELS["qc_reg"]
    assert L.cbp_decode(c.handle, fake, fake, fake, 5, 8, ctypes.byref(o), None) == cbp.CBP_EUNSUPPORTED
    assert b"register-resident" in L.cbp_last_error()
    # the LDS-staged kernel: cbp_decode only, syndrome stop or fixed sweeps,
    # Step-3 decisions, no dumps, and a frame that fits a CU's LDS
    o.kernel = cbp.KERNELS["sparse_lds"]
    for field, val in (("stop_rule", 1), ("hd_mode", 1), ("dump_sweep", 2)):
        setattr(o, field, val)
        o.dump_frames = 1
        assert L.cbp_decode(c.handle, fake, fake, fake, 5, 8, ctypes.byref(o), None) == cbp.CBP_EUNSUPPORTED
        assert b"LDS-staged" in L.cbp_last_error()
        setattr(o, field, 0)
    o.dump_frames = 0
    big = cbp.Code.from_workload(get_code("qc26112"))  # 0.4 MB of state per frame
    assert not big.has_kernel("sparse_lds")
    assert L.cbp_decode(big.handle, fake, fake, fake, 5, 8, ctypes.byref(o), None) == cbp.CBP_EUNSUPPORTED
    o.kernel = 0
    o.lmax = -1.0
    assert L.cbp_decode(c.handle, fake, fake, fake, 5, 8, ctypes.byref(o), None) == cbp.CBP_EINVAL
    o.lmax = 20.0
    o.hd_mode = 1
    assert L.lbp_nms_decode(c.handle, fake, fake, fake, 5, 8, ctypes.byref(o), None) == cbp.CBP_EINVAL
    o.hd_mode = 0
    o.workspace = 4096 + 8  # a caller workspace must be 256-byte aligned
    o.workspace_bytes = 1 << 30
    assert L.lbp_decode(c.handle, fake, fake, fake, 5, 8, ctypes.byref(o), None) == cbp.CBP_EINVAL
    assert b"aligned" in L.cbp_last_error()
    o.workspace = None
    assert L.cbp_syndrome(None, None, None, 3, None) == cbp.CBP_EINVAL


@contextlib.contextmanager
def env(**kw):
    old = {k: os.environ.get(k) for k in kw}
    os.environ.update(kw)
    try:
        yield
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("name", ["reg36_n96", "qc2304", "qc26112", "peg_reg36_n2048", "peg_irr_n8192"])
def test_row_levels(L, name):
    """Row levels: a permutation of the rows; rows of one level share no variable; rows with a
    common variable keep their index order; each row sits one level above the highest earlier
    row it shares a variable with (checked from the columns' row lists)."""
    code = get_code(name)
    nlev, ptr, rows = cbp.Code.from_workload(code).levels()
    assert ptr[0] == 0 and ptr[-1] == code.M and (np.diff(ptr) > 0).all()
    assert np.array_equal(np.sort(rows), np.arange(code.M))
    level = np.empty(code.M, np.int64)
    for l in range(nlev):
        rl = rows[ptr[l]:ptr[l + 1]]
        assert (np.diff(rl) > 0).all()
        level[rl] = l
        cols = np.concatenate([code.col_idx[code.row_ptr[i]:code.row_ptr[i + 1]] for i in rl])
        assert len(np.unique(cols)) == len(cols), f"level {l} has rows sharing a variable"
    col_rows = [[] for _ in range(code.N)]
    for i in range(code.M):
        for v in code.col_idx[code.row_ptr[i]:code.row_ptr[i + 1]]:
            col_rows[v].append(i)
    for i in range(code.M):
        earlier = {k for v in code.col_idx[code.row_ptr[i]:code.row_ptr[i + 1]] for k in col_rows[v] if k < i}
        assert level[i] == (1 + max(level[k] for k in earlier) if earlier else 0)


def test_workspace_sizes(L):
    c = cbp.Code.from_workload(get_code("reg36_n96"))
    n = cbp.workspace_size(c, "cbp", 2000, kernel="sparse")
    S = 2048  # frames padded to whole waves
    assert n >= (96 + 288 + 2 * 48) * 4 * S + 96 * S  # Q, R, check-beliefs (float2), decisions
    assert cbp.workspace_size(c, "cbp", 0) == 0
    # frame state in LDS: only the frame counter in device memory (the
    # default for a code without a QC layout whose frame fits a CU's LDS)
    assert cbp.workspace_size(c, "cbp", 2000) == cbp.workspace_size(c, "cbp", 2000, kernel="sparse_lds") == 256
    q = cbp.Code.from_workload(get_code("qc2304"))
    assert 0 < cbp.workspace_size(q, "cbp", 131072) <= 4096
    # streamed kernel: one slot of state per frame in flight, at most 2048 slots
    big = cbp.Code.from_workload(get_code("qc26112"))
    per_slot = 4 * (26112 + 76800) + 8 * 17664 + 26112  # Q, R, check-beliefs, decisions
    n = cbp.workspace_size(big, "cbp", 4096)
    assert 2048 * per_slot <= n <= 2048 * (per_slot + 512) + 256
    assert cbp.workspace_size(big, "cbp", 3) <= 3 * (per_slot + 512) + 256


def test_log_tanh_baselines_run_on_the_sparse_kernel(L):
    c = cbp.Code.from_workload(get_code("reg36_n96"))
    S = 2048
    # hand-off items: (frame, sweeps) and one contiguous frame state per slot
    r256 = lambda x: (x + 255) // 256 * 256
    item = 2 * r256(4 * 96) + r256(4 * 288) + r256(96)
    for dec in ("lbp", "fbp", "lbp_nms"):
        # Lambda, R, flooding accumulator, decisions, each frame-interleaved
        n = cbp.workspace_size(c, dec, 2000, kernel="sparse")
        lo = (2 * 96 + 288) * 4 * S + 96 * S + 256 + r256(8 * S) + S * item
        assert lo <= n <= lo + 9 * 256
        assert cbp.workspace_size(c, dec, 2000) == 256   # auto: the LDS-staged kernel
    with env(CBP_SPARSE_HANDOFF="0"):   # no hand-off: header and lane blocks only
        n = cbp.workspace_size(c, "lbp", 2000, kernel="sparse")
        assert (2 * 96 + 288) * 4 * S + 96 * S <= n <= (2 * 96 + 288) * 4 * S + 96 * S + 9 * 256
    # options the level-parallel kernel does not serve reserve no items
    lane = cbp.workspace_size(c, "cbp", 2000, kernel="sparse")
    assert cbp.workspace_size(c, "cbp", 2000, stop_rule=1) < lane
    assert cbp.workspace_size(c, "cbp", 2000, hd_mode=1) < lane
    q = cbp.Code.from_workload(get_code("qc2304"))
    # a QC code: lbp/fbp run on the CSR kernels; auto picks the LDS-staged one
    # (frame state in LDS, only the frame counter in device memory) where a
    # frame fits, else the one-frame-per-lane kernel (a large frame-interleaved
    # workspace)
    assert cbp.workspace_size(q, "lbp", 4096) == 256
    assert cbp.workspace_size(q, "lbp", 4096, kernel="sparse") > 4096 * (2304 + 6912) * 4
    big = cbp.Code.from_workload(get_code("qc26112"))
    assert cbp.workspace_size(big, "fbp", 64) > 64 * (2 * 26112 + 76800) * 4
    for k in ("qc_reg", "qc_stream"):
        with pytest.raises(cbp.CbpError) as e:
            cbp.workspace_size(q, "fbp", 64, kernel=k)
        assert e.value.status == cbp.CBP_EUNSUPPORTED
    o = cbp.Opts()
    L.cbp_opts_default(ctypes.byref(o))
    o.stop_rule = 1  # the paper's rule is CBP's
    fake = ctypes.c_void_p(16)
    assert L.lbp_decode(c.handle, fake, fake, fake, 5, 8, ctypes.byref(o), None) == cbp.CBP_EINVAL
    assert L.fbp_decode(None, fake, fake, fake, 5, 8, None, None) == cbp.CBP_EINVAL
    n = ctypes.c_size_t()
    assert L.cbp_workspace_size(c.handle, 5, 10, None, ctypes.byref(n)) == cbp.CBP_EINVAL


def test_mix_plan_validation(L):
    from paper_2305_05286_amd.workload import mixed_family
    fam = mixed_family()
    handles = [cbp.Code.from_workload(c) for c in fam]
    mix = cbp.Mix(handles)
    assert mix.schedule == (384, 0, 0)               # lcm(16, 32, 64, 128, 384) fills whole waves
    mix.schedule = (768, 2)
    assert mix.schedule == (768, 2, 0)
    mix.schedule = (768, 2, 1)                       # LDS-staged part: one workgroup per CU
    assert mix.schedule == (768, 2, 1)
    for bad in [(384 + 16, 0), (0, 0), (1152, 0), (384, -1), (384, 2, 3), (384, 2, -1)]:
        with pytest.raises(cbp.CbpError):
            mix.schedule = bad
    small = cbp.Mix([cbp.Code.from_workload(c) for c in fam if c.Z == 16])
    assert small.schedule == (64, 0, 0)              # 16 -> doubled to a whole wave
    # Z values whose workgroup would need more than 1024 lanes, and a non-QC code
    q96 = cbp.Code.from_qc(np.array([[0, 1, -1], [2, 0, 1]]), 96)
    q100 = cbp.Code.from_qc(np.array([[0, 1, -1], [2, 0, 1]]), 100)
    with pytest.raises(cbp.CbpError) as e:
        cbp.Mix([q96, q100])
    assert e.value.status == cbp.CBP_EUNSUPPORTED
    with pytest.raises(cbp.CbpError) as e:
        cbp.Mix([cbp.Code.from_workload(get_code("reg36_n96"))])
    assert e.value.status == cbp.CBP_EUNSUPPORTED
    arr = (ctypes.c_void_p * 1)(None)
    h = ctypes.c_void_p()
    assert L.cbp_mix_create(arr, 1, ctypes.byref(h)) == cbp.CBP_EINVAL
    assert L.cbp_mix_create(arr, 0, ctypes.byref(h)) == cbp.CBP_EINVAL
    assert L.cbp_mix_create(arr, 257, ctypes.byref(h)) == cbp.CBP_EINVAL


def test_unrolled_workspace_and_validation(L):
    q = cbp.Code.from_workload(get_code("qc2304"))
    n = cbp.unrolled_workspace_size(q, 10, 8192)
    state = 4 * (2304 + 7296) + 8 * 1152                # Q, R, check-beliefs per frame
    # working state + 9 checkpoints (the final state stays in the working
    # area), adjoints, one sweep of tape
    per_frame = state * 10 + 4 * (2304 + 7296 + 1152) + 16 * 7296
    assert 8192 * per_frame <= n <= 8192 * (per_frame + 512) + 4096 * 10 * 24 * 8 + 256
    assert cbp.unrolled_workspace_size(q, 10, 0) == 0
    for sweeps in (0, 65):
        with pytest.raises(cbp.CbpError):
            cbp.unrolled_workspace_size(q, sweeps, 10)
    with pytest.raises(cbp.CbpError):
        cbp.unrolled_workspace_size(cbp.Code.from_workload(get_code("reg36_n96")), 5, 10)
    sz = ctypes.c_size_t()
    assert L.cbp_unrolled_workspace_size(q.handle, 5, -1, ctypes.byref(sz)) == cbp.CBP_EINVAL
    assert L.cbp_unrolled_forward(None, None, 1, 5, None, None, None, None, None, 0, None) == cbp.CBP_EINVAL
