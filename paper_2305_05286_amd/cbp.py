"""Python binding of libcbp.so (include/cbp.h): argument marshalling only.

Every decoding step runs in the HIP kernels of the shared library; PyTorch
provides device memory and the current stream.  If the library has not been
built this module raises on use (there is no fallback path).

    from paper_2305_05286_amd import cbp
    code = cbp.Code.from_workload(workload_code)
    bits, iters = cbp.cbp_decode(code, llr_cuda_f32, max_iter=50)
"""
from __future__ import annotations

import ctypes
from pathlib import Path
from typing import Optional

import numpy as np

LIB_PATH = Path(__file__).resolve().parent / "libcbp.so"

CBP_OK, CBP_EINVAL, CBP_EUNSUPPORTED, CBP_EHIP, CBP_ENOMEM = 0, -1, -2, -3, -4
KERNELS = {"auto": 0, "qc_reg": 1, "qc_stream": 2, "sparse": 4, "sparse_lds": 8}
RULES = {"log_tanh": 0, "min_sum": 1}
DECODERS = {"cbp": 0, "lbp_nms": 1, "fbp_nms": 2, "lbp": 3, "fbp": 4}

# exported names declared in include/cbp.h
EXPORTS = ("cbp_code_from_csr", "cbp_code_from_qc", "cbp_code_free", "cbp_code_info", "cbp_code_levels",
           "cbp_opts_default", "cbp_decode", "lbp_nms_decode", "fbp_nms_decode",
           "lbp_decode", "fbp_decode", "cbp_decode_static", "cbp_workspace_size", "cbp_syndrome", "cbp_strerror", "cbp_last_error",
           "cbp_version", "cbp_mix_create", "cbp_mix_free", "cbp_mix_get_schedule",
           "cbp_mix_set_schedule", "cbp_mix_workspace_size", "cbp_mix_decode", "cbp_mix_tune",
           "cbp_mix_graph_create", "cbp_graph_launch", "cbp_graph_free",
           "cbp_unrolled_workspace_size", "cbp_unrolled_forward", "cbp_unrolled_backward")


class CbpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class MixSchedule(ctypes.Structure):
    """Mirror of cbp_mix_schedule_t."""
    _fields_ = [("lanes", ctypes.c_int32), ("groups_per_cu", ctypes.c_int32), ("lds_groups_per_cu", ctypes.c_int32)]


class Opts(ctypes.Structure):
    """Mirror of cbp_opts_t."""
    _fields_ = [
        ("stop_rule", ctypes.c_int32),
        ("hd_mode", ctypes.c_int32),
        ("lmax", ctypes.c_float),
        ("alpha", ctypes.c_float),
        ("kernel", ctypes.c_int32),
        ("check_rule", ctypes.c_int32),
        ("dump_sweep", ctypes.c_int32),
        ("validate", ctypes.c_int32),
        ("dump_frames", ctypes.c_int64),
        ("dump_q", ctypes.c_void_p),
        ("dump_r", ctypes.c_void_p),
        ("dump_om", ctypes.c_void_p),
        ("dump_lam", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


_lib = None


def lib():
    """Load libcbp.so (raises if it is missing: build it with paper_2305_05286_amd.build)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2305_05286_amd.build`")
        L = ctypes.CDLL(str(LIB_PATH))
        i32, i64, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
        L.cbp_code_from_csr.argtypes = [i32, i32, vp, vp, ctypes.POINTER(vp)]
        L.cbp_code_from_qc.argtypes = [i32, i32, i32, vp, ctypes.POINTER(vp)]
        L.cbp_code_free.argtypes = [vp]
        L.cbp_code_free.restype = None
        L.cbp_code_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                    ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.cbp_code_levels.argtypes = [vp, ctypes.POINTER(i32), vp, vp]
        L.cbp_opts_default.argtypes = [ctypes.POINTER(Opts)]
        L.cbp_opts_default.restype = None
        for name in ("cbp_decode", "lbp_nms_decode", "fbp_nms_decode", "lbp_decode", "fbp_decode"):
            if not hasattr(L, name):
                continue
            getattr(L, name).argtypes = [vp, vp, vp, vp, i32, i64, ctypes.POINTER(Opts), vp]
            getattr(L, name).restype = ctypes.c_int
        L.cbp_decode_static.argtypes = [vp, i32, vp, vp, vp, i32, i64, ctypes.POINTER(Opts), vp]
        L.cbp_decode_static.restype = ctypes.c_int
        L.cbp_workspace_size.argtypes = [vp, i32, i64, ctypes.POINTER(Opts), ctypes.POINTER(sz)]
        L.cbp_syndrome.argtypes = [vp, vp, vp, i64, vp]
        L.cbp_strerror.argtypes = [ctypes.c_int]
        L.cbp_strerror.restype = ctypes.c_char_p
        L.cbp_last_error.argtypes = []
        L.cbp_last_error.restype = ctypes.c_char_p
        L.cbp_version.argtypes = []
        L.cbp_version.restype = i32
        if not hasattr(L, "cbp_mix_create"):  # a library built before the mixed-batch entry points
            _lib = L
            return _lib
        L.cbp_mix_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]
        L.cbp_mix_free.argtypes = [vp]
        L.cbp_mix_free.restype = None
        L.cbp_mix_get_schedule.argtypes = [vp, ctypes.POINTER(MixSchedule)]
        L.cbp_mix_set_schedule.argtypes = [vp, ctypes.POINTER(MixSchedule)]
        L.cbp_mix_workspace_size.argtypes = [vp, i32, i64, ctypes.POINTER(Opts), ctypes.POINTER(sz)]
        mix_args = [vp, i32, vp, i64, vp, vp, vp, vp, i32, i64, ctypes.POINTER(Opts)]
        L.cbp_mix_decode.argtypes = mix_args + [vp, sz, vp]
        L.cbp_mix_tune.argtypes = mix_args + [vp, ctypes.POINTER(MixSchedule), ctypes.POINTER(ctypes.c_float)]
        L.cbp_mix_graph_create.argtypes = mix_args + [vp, sz, ctypes.POINTER(vp)]
        L.cbp_graph_launch.argtypes = [vp, vp]
        L.cbp_graph_free.argtypes = [vp]
        L.cbp_graph_free.restype = None
        L.cbp_unrolled_workspace_size.argtypes = [vp, i32, i64, ctypes.POINTER(sz)]
        L.cbp_unrolled_forward.argtypes = [vp, vp, i64, i32, vp, vp, vp, ctypes.POINTER(Opts), vp, sz, vp]
        L.cbp_unrolled_backward.argtypes = [vp, vp, i64, i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Opts),
                                            vp, sz, vp]
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != CBP_OK:
        L = lib()
        raise CbpError(status, f"{L.cbp_strerror(status).decode()}: {L.cbp_last_error().decode()}")


class Code:
    """Owning wrapper of a cbp_code_t handle."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        M, N, Z, K = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        E = ctypes.c_int64()
        check(lib().cbp_code_info(handle, ctypes.byref(M), ctypes.byref(N), ctypes.byref(E),
                                  ctypes.byref(Z), ctypes.byref(K)))
        self.M, self.N, self.E, self.Z, self.kernels = M.value, N.value, E.value, Z.value, K.value

    @property
    def handle(self):
        return self._h

    @classmethod
    def from_csr(cls, M: int, N: int, row_ptr, col_idx) -> "Code":
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        h = ctypes.c_void_p()
        check(lib().cbp_code_from_csr(M, N, rp.ctypes.data, ci.ctypes.data, ctypes.byref(h)))
        return cls(h)

    @classmethod
    def from_qc(cls, shifts, Z: int) -> "Code":
        sh = np.ascontiguousarray(shifts, dtype=np.int32)
        mb, nb = sh.shape
        h = ctypes.c_void_p()
        check(lib().cbp_code_from_qc(mb, nb, Z, sh.ctypes.data, ctypes.byref(h)))
        return cls(h)

    @classmethod
    def from_workload(cls, code) -> "Code":
        """From a paper_2305_05286_amd.workload.Code (QC if it has shifts)."""
        if getattr(code, "shifts", None) is not None:
            return cls.from_qc(code.shifts, code.Z)
        return cls.from_csr(code.M, code.N, code.row_ptr, code.col_idx)

    def has_kernel(self, name: str) -> bool:
        return bool(self.kernels & KERNELS[name])

    def levels(self):
        """Row levels (cbp_code_levels): (nlev, lvl_ptr int32 [nlev+1], rows int32 [M])."""
        import numpy as np
        n = ctypes.c_int32()
        check(lib().cbp_code_levels(self.handle, ctypes.byref(n), None, None))
        ptr = np.empty(n.value + 1, np.int32)
        rows = np.empty(self.M, np.int32)
        check(lib().cbp_code_levels(self.handle, None, ptr.ctypes.data, rows.ctypes.data))
        return n.value, ptr, rows

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.cbp_code_free(h)
            self._h = None


def _opts(stop_rule=0, hd_mode=0, lmax=20.0, alpha=0.75, kernel="auto", dump=None,
          workspace=None, check_rule="log_tanh", validate=False) -> Opts:
    o = Opts()
    lib().cbp_opts_default(ctypes.byref(o))
    o.stop_rule, o.hd_mode, o.lmax, o.alpha = stop_rule, hd_mode, lmax, alpha
    o.validate = 1 if validate else 0
    o.kernel = KERNELS[kernel]
    o.check_rule = RULES[check_rule]
    if dump is not None:
        o.dump_sweep = dump["sweep"]
        o.dump_frames = dump["frames"]
        for k in ("q", "r", "om", "lam"):
            t = dump.get(k)
            setattr(o, f"dump_{k}", t.data_ptr() if t is not None else None)
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return o


def _run(which: str, code: Code, llr, max_iter: int, *, stop_rule=0, hd_mode=0, lmax=20.0,
         alpha=0.75, kernel="auto", dump_sweep: int = 0, dump_frames: int = 0,
         workspace=None, out=None, stream=None, check_rule="log_tanh", validate=False,
         static=False):
    import torch
    if not (isinstance(llr, torch.Tensor) and llr.is_cuda and llr.dtype == torch.float32):
        raise TypeError("llr must be a float32 CUDA tensor")
    if llr.dim() != 2 or llr.shape[1] != code.N:
        raise ValueError(f"llr must be [batch, {code.N}]")
    llr = llr.contiguous()
    B = llr.shape[0]
    dev = llr.device
    if out is None:
        bits = torch.empty((B, code.N), dtype=torch.uint8, device=dev)
        iters = torch.empty((B,), dtype=torch.int32, device=dev)
    else:
        bits, iters = out
    dump = None
    if dump_sweep > 0 and dump_frames > 0:
        nd = min(dump_frames, B)
        dump = {"sweep": dump_sweep, "frames": nd}
        dump["lam"] = torch.full((nd, code.N), float("nan"), device=dev)
        dump["r"] = torch.full((nd, code.E), float("nan"), device=dev)
        if which in ("cbp", "cbp_nms"):
            dump["q"] = torch.full((nd, code.N), float("nan"), device=dev)
            dump["om"] = torch.full((nd, code.M), float("nan"), device=dev)
    if which == "cbp_nms":  # CBP with the normalized min-sum rule of Sec. IV-D
        which, check_rule = "cbp", "min_sum"
    o = _opts(stop_rule, hd_mode, lmax, alpha, kernel, dump, workspace, check_rule, validate)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        if static:
            check(lib().cbp_decode_static(code.handle, DECODERS[which], llr.data_ptr(), bits.data_ptr(),
                                          iters.data_ptr(), int(max_iter), B, ctypes.byref(o),
                                          ctypes.c_void_p(s.cuda_stream)))
        else:
            fn = getattr(lib(), {"cbp": "cbp_decode", "lbp_nms": "lbp_nms_decode", "fbp_nms": "fbp_nms_decode",
                                 "lbp": "lbp_decode", "fbp": "fbp_decode"}[which])
            check(fn(code.handle, llr.data_ptr(), bits.data_ptr(), iters.data_ptr(), int(max_iter),
                     B, ctypes.byref(o), ctypes.c_void_p(s.cuda_stream)))
    if dump is not None:
        return bits, iters, dump
    return bits, iters


def cbp_decode(code: Code, llr, max_iter: int, **kw):
    """CBP decoding (Sec. IV-C).  Returns (bits uint8 [B,N], iters int32 [B]) on llr's device,
    plus a dump dict when dump_sweep/dump_frames are given.  validate=True rejects NaN / +-Inf
    LLRs (CbpError, CBP_EINVAL) before decoding and synchronises the stream."""
    return _run("cbp", code, llr, max_iter, **kw)


def lbp_nms_decode(code: Code, llr, max_iter: int, **kw):
    """Layered normalized min-sum baseline (same arguments as cbp_decode)."""
    return _run("lbp_nms", code, llr, max_iter, **kw)


def fbp_nms_decode(code: Code, llr, max_iter: int, **kw):
    """Flooding normalized min-sum baseline (same arguments as cbp_decode)."""
    return _run("fbp_nms", code, llr, max_iter, **kw)


def lbp_decode(code: Code, llr, max_iter: int, **kw):
    """Layered BP with the log-tanh check rule (sparse kernel; same arguments as cbp_decode)."""
    return _run("lbp", code, llr, max_iter, **kw)


def fbp_decode(code: Code, llr, max_iter: int, **kw):
    """Flooding BP with the log-tanh check rule (sparse kernel; same arguments as cbp_decode)."""
    return _run("fbp", code, llr, max_iter, **kw)


def decode(code: Code, llr, max_iter: int, algo: str = "cbp", **kw):
    """algo: "cbp", "cbp_nms" (cbp_decode with the min-sum rule), "lbp_nms", "fbp_nms",
    "lbp", "fbp"."""
    return _run(algo, code, llr, max_iter, **kw)


def decode_static(code: Code, llr, max_iter: int, algo: str = "cbp", **kw):
    """cbp_decode_static: the decoder `algo` (as in decode) with the library's static
    device scratch as workspace, so the call allocates nothing in the library (the output
    tensors are allocated here unless out=(bits, iters) is given).  The code's device tables
    must already exist on llr's device (any earlier decode or cbp_syndrome call builds them)."""
    return _run(algo, code, llr, max_iter, static=True, **kw)


def cbp_syndrome(code: Code, bits, stream=None):
    """ok uint8 [B]: 1 where H bits^T = 0."""
    import torch
    if not (bits.is_cuda and bits.dtype == torch.uint8 and bits.dim() == 2 and bits.shape[1] == code.N):
        raise ValueError("bits must be a uint8 CUDA tensor [batch, N]")
    bits = bits.contiguous()
    ok = torch.empty((bits.shape[0],), dtype=torch.uint8, device=bits.device)
    s = stream if stream is not None else torch.cuda.current_stream(bits.device)
    with torch.cuda.device(bits.device):
        check(lib().cbp_syndrome(code.handle, bits.data_ptr(), ok.data_ptr(), bits.shape[0],
                                 ctypes.c_void_p(s.cuda_stream)))
    return ok


def workspace_size(code: Code, decoder: str, batch: int, **kw) -> int:
    if decoder == "cbp_nms":  # cbp_decode with the min-sum rule
        decoder, kw = "cbp", {**kw, "check_rule": "min_sum"}
    o = _opts(**kw)
    n = ctypes.c_size_t()
    check(lib().cbp_workspace_size(code.handle, DECODERS[decoder], batch, ctypes.byref(o),
                                   ctypes.byref(n)))
    return n.value


def version() -> int:
    return int(lib().cbp_version())


# ---- mixed-code batches (cbp_mix_*) -----------------------------------------

_MIX_ALGOS = {"cbp": (0, "log_tanh"), "cbp_nms": (0, "min_sum"), "lbp_nms": (1, "log_tanh"),
              "fbp_nms": (2, "log_tanh")}


class Graph:
    """A captured cbp_mix_decode (cbp_graph_t); launch() replays it."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep  # buffers the graph reads and writes

    def launch(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        check(lib().cbp_graph_launch(self._h, ctypes.c_void_p(s.cuda_stream)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.cbp_graph_free(h)
            self._h = None


class Mix:
    """A plan over several QC codes decoded together in one persistent launch (cbp_mix_t).

    Frames are packed: frame f has code index frame_code[f] and its N LLRs start at
    frame_offset[f] of a flat float32 tensor; decisions go to the same offsets of a flat
    uint8 tensor."""

    def __init__(self, codes):
        self.codes = list(codes)  # the handles must outlive the plan
        arr = (ctypes.c_void_p * len(self.codes))(*[c.handle for c in self.codes])
        h = ctypes.c_void_p()
        check(lib().cbp_mix_create(arr, len(self.codes), ctypes.byref(h)))
        self._h = h
        self.N = [c.N for c in self.codes]

    @property
    def schedule(self):
        sc = MixSchedule()
        check(lib().cbp_mix_get_schedule(self._h, ctypes.byref(sc)))
        return (sc.lanes, sc.groups_per_cu, sc.lds_groups_per_cu)

    @schedule.setter
    def schedule(self, value):
        """(lanes, groups_per_cu[, lds_groups_per_cu = 0]), cbp_mix_schedule_t."""
        sc = MixSchedule(int(value[0]), int(value[1]), int(value[2]) if len(value) > 2 else 0)
        check(lib().cbp_mix_set_schedule(self._h, ctypes.byref(sc)))

    def workspace_size(self, batch, algo="cbp", **kw):
        dec, rule = _MIX_ALGOS[algo]
        o = _opts(check_rule=rule, **kw)
        n = ctypes.c_size_t()
        check(lib().cbp_mix_workspace_size(self._h, dec, int(batch), ctypes.byref(o), ctypes.byref(n)))
        return n.value

    def _args(self, algo, llr, frame_code, frame_offset, max_iter, out, kw):
        import torch
        if not (llr.is_cuda and llr.dtype == torch.float32 and llr.dim() == 1 and llr.is_contiguous()):
            raise TypeError("llr must be a contiguous 1-D float32 CUDA tensor")
        if not (frame_code.is_cuda and frame_code.dtype == torch.int32 and frame_code.is_contiguous()):
            raise TypeError("frame_code must be a contiguous int32 CUDA tensor")
        if not (frame_offset.is_cuda and frame_offset.dtype == torch.int64 and frame_offset.is_contiguous()):
            raise TypeError("frame_offset must be a contiguous int64 CUDA tensor")
        B = frame_code.numel()
        if frame_offset.numel() != B:
            raise ValueError("frame_code and frame_offset differ in length")
        if out is None:
            bits = torch.zeros(llr.numel(), dtype=torch.uint8, device=llr.device)
            iters = torch.empty(B, dtype=torch.int32, device=llr.device)
        else:
            bits, iters = out
        dec, rule = _MIX_ALGOS[algo]
        o = _opts(check_rule=rule, **kw)
        args = [self._h, dec, llr.data_ptr(), llr.numel(), frame_code.data_ptr(), frame_offset.data_ptr(),
                bits.data_ptr(), iters.data_ptr(), int(max_iter), B, ctypes.byref(o)]
        return args, bits, iters, B

    def decode(self, llr, frame_code, frame_offset, max_iter, algo="cbp", workspace=None, out=None,
               stream=None, **kw):
        """Returns (bits uint8 [len(llr)], iters int32 [batch]); allocates the workspace with
        torch when none is given."""
        import torch
        args, bits, iters, B = self._args(algo, llr, frame_code, frame_offset, max_iter, out, kw)
        if workspace is None:
            workspace = torch.empty(self.workspace_size(B, algo), dtype=torch.uint8, device=llr.device)
        s = stream if stream is not None else torch.cuda.current_stream(llr.device)
        with torch.cuda.device(llr.device):
            check(lib().cbp_mix_decode(*args, workspace.data_ptr(), workspace.numel(),
                                       ctypes.c_void_p(s.cuda_stream)))
        return bits, iters

    def tune(self, llr, frame_code, frame_offset, max_iter, algo="cbp", out=None, stream=None, **kw):
        """Times every candidate schedule on this batch and keeps the fastest.
        Returns ((lanes, groups_per_cu, lds_groups_per_cu), ms)."""
        import torch
        args, bits, iters, B = self._args(algo, llr, frame_code, frame_offset, max_iter, out, kw)
        s = stream if stream is not None else torch.cuda.current_stream(llr.device)
        best, ms = MixSchedule(), ctypes.c_float()
        with torch.cuda.device(llr.device):
            check(lib().cbp_mix_tune(*args, ctypes.c_void_p(s.cuda_stream), ctypes.byref(best), ctypes.byref(ms)))
        return (best.lanes, best.groups_per_cu, best.lds_groups_per_cu), ms.value

    def graph(self, llr, frame_code, frame_offset, max_iter, algo="cbp", workspace=None, out=None, **kw):
        """Captures one decode of these buffers into a HIP graph.  Returns (graph, bits, iters)."""
        import torch
        args, bits, iters, B = self._args(algo, llr, frame_code, frame_offset, max_iter, out, kw)
        if workspace is None:
            workspace = torch.empty(self.workspace_size(B, algo), dtype=torch.uint8, device=llr.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(llr.device):
            check(lib().cbp_mix_graph_create(*args, workspace.data_ptr(), workspace.numel(), ctypes.byref(h)))
        return Graph(h, (llr, frame_code, frame_offset, bits, iters, workspace)), bits, iters

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.cbp_mix_free(h)
            self._h = None


# ---- unrolled differentiable CBP (cbp_unrolled_*) ------------------------------

def unrolled_workspace_size(code: Code, sweeps: int, batch: int) -> int:
    n = ctypes.c_size_t()
    check(lib().cbp_unrolled_workspace_size(code.handle, int(sweeps), int(batch), ctypes.byref(n)))
    return n.value


def _unrolled_fn():
    import torch

    class UnrolledCBPFunction(torch.autograd.Function):
        """Soft output of `sweeps` weighted CBP sweeps; backward is the library's adjoint kernel."""

        @staticmethod
        def forward(ctx, llr, w, beta, code, sweeps, lmax):
            if not (llr.is_cuda and llr.dtype == torch.float32 and llr.dim() == 2 and llr.shape[1] == code.N):
                raise TypeError(f"llr must be a float32 CUDA tensor [batch, {code.N}]")
            llr, w, beta = llr.contiguous(), w.detach().contiguous(), beta.detach().contiguous()
            B = llr.shape[0]
            ws = torch.empty(unrolled_workspace_size(code, sweeps, B), dtype=torch.uint8, device=llr.device)
            out = torch.empty_like(llr)
            o = _opts(lmax=lmax)
            s = torch.cuda.current_stream(llr.device)
            with torch.cuda.device(llr.device):
                check(lib().cbp_unrolled_forward(code.handle, llr.data_ptr(), B, int(sweeps), w.data_ptr(),
                                                 beta.data_ptr(), out.data_ptr(), ctypes.byref(o),
                                                 ws.data_ptr(), ws.numel(), ctypes.c_void_p(s.cuda_stream)))
            ctx.save_for_backward(llr, w, beta)
            ctx.ws, ctx.code, ctx.sweeps, ctx.lmax = ws, code, sweeps, lmax
            return out

        @staticmethod
        def backward(ctx, gout):
            if ctx.ws is None:
                raise RuntimeError("the unrolled decoder's backward pass consumes the forward pass's "
                                   "checkpoints: run the forward pass again (retain_graph is not supported)")
            llr, w, beta = ctx.saved_tensors
            gout = gout.contiguous()
            B = llr.shape[0]
            gllr = torch.empty_like(llr) if ctx.needs_input_grad[0] else None
            gw, gb = torch.empty_like(w), torch.empty_like(beta)
            o = _opts(lmax=ctx.lmax)
            s = torch.cuda.current_stream(llr.device)
            with torch.cuda.device(llr.device):
                check(lib().cbp_unrolled_backward(ctx.code.handle, llr.data_ptr(), B, int(ctx.sweeps),
                                                  w.data_ptr(), beta.data_ptr(), gout.data_ptr(),
                                                  gllr.data_ptr() if gllr is not None else None,
                                                  gw.data_ptr(), gb.data_ptr(), ctypes.byref(o), ctx.ws.data_ptr(),
                                                  ctx.ws.numel(), ctypes.c_void_p(s.cuda_stream)))
            ctx.ws = None
            return gllr, gw, gb, None, None, None

    return UnrolledCBPFunction


_UNROLLED = None


def unrolled_cbp(code: Code, llr, w, beta, sweeps: int, lmax: float = 20.0):
    """Differentiable soft output [batch, N] of `sweeps` weighted CBP sweeps (autograd-aware)."""
    global _UNROLLED
    if _UNROLLED is None:
        _UNROLLED = _unrolled_fn()
    return _UNROLLED.apply(llr, w, beta, code, int(sweeps), float(lmax))


def unrolled_module(code: Code, sweeps: int, lmax: float = 20.0):
    """A torch.nn.Module with learnable w (init 1) and beta (init 0), [sweeps, nb]."""
    import torch

    nb = code.N // code.Z

    class UnrolledCBP(torch.nn.Module):
        def __init__(self):
            super().__init__()
            self.code, self.sweeps, self.lmax = code, sweeps, lmax
            self.w = torch.nn.Parameter(torch.ones(sweeps, nb))
            self.beta = torch.nn.Parameter(torch.zeros(sweeps, nb))

        def forward(self, llr):
            return unrolled_cbp(self.code, llr, self.w, self.beta, self.sweeps, self.lmax)

    return UnrolledCBP()
