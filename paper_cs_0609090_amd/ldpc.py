"""Python binding of ``libldpc.so`` (include/ldpc.h): argument marshalling only.

Every decoding step runs in the library's HIP kernels; torch provides device
memory and the stream.  If the library is not built this module raises
instead of falling back to anything else.

    code = Code.from_parity_check(H, device=0)
    out = code.decode(llr_cuda_tensor, max_iter=50, alpha=0.8, msg="int8")
    out["hard"], out["llr"], out["iters"], out["ok"]
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldpc.so")

LDPC_OK, LDPC_EINVAL, LDPC_EBADCODE, LDPC_ENOMEM, LDPC_EDEVICE, LDPC_EUNSUPPORTED = range(6)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "EBADCODE", 3: "ENOMEM", 4: "EDEVICE", 5: "EUNSUPPORTED"}
MSG = {"fp32": 0, "int8": 1, "1bit": 2}
SCHED = {"single_scan": 0, "two_scan": 1}
F_CHECK_INPUT = 0x1
LAYOUT = {"auto": 0, "lds": 1, "hbm": 2, "reg": 3, "reg1": 4, "frames": 5}
LAYOUT_SHIFT = 8

EXPORTS = ("ldpc_code_create", "ldpc_code_destroy", "ldpc_code_query",
           "ldpc_decode_workspace_size", "ldpc_decode_plan", "ldpc_decode_batch", "ldpc_last_error",
           "ldpc_version",
           # include/ldpc_sim.h
           "ldpc_encoder_info", "ldpc_encode_batch", "ldpc_random_bits", "ldpc_channel_awgn",
           "ldpc_count_errors",
           # include/ldpc_learn.h
           "ldpc_learn_classes", "ldpc_learn_workspace_size", "ldpc_learn_forward",
           "ldpc_learn_backward",
           # include/ldpc_multi.h
           "ldpc_multi_workspace_size", "ldpc_decode_multi", "ldpc_autotune")
LAYOUT_NAME = {v: k for k, v in LAYOUT.items()}
KERNEL_NAME = {0: "generic_int", 1: "generic_f32", 2: "two_scan", 3: "reg1", 4: "packed",
               5: "f32_frames", 6: "two_scan_frames"}  # ldpc_kernel
ENC_KIND = {0: "none", 1: "staircase", 2: "dense"}


class LdpcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class DecodeParams(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("alpha", ctypes.c_float),
                ("beta", ctypes.c_float), ("early_stop", ctypes.c_int32),
                ("msg", ctypes.c_int32), ("sched", ctypes.c_int32),
                ("llr_step", ctypes.c_float), ("flags", ctypes.c_uint32),
                ("weights", ctypes.c_void_p), ("weight_iters", ctypes.c_int32),
                ("weight_classes", ctypes.c_int32), ("msg_bits", ctypes.c_int32)]


class CodeInfo(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("N", ctypes.c_int32), ("E", ctypes.c_int64),
                ("min_row_deg", ctypes.c_int32), ("max_row_deg", ctypes.c_int32),
                ("max_col_deg", ctypes.c_int32), ("slots_per_row", ctypes.c_int32),
                ("rows_padded", ctypes.c_int32), ("device", ctypes.c_int32),
                ("addr_bytes_single", ctypes.c_int64), ("addr_bytes_two", ctypes.c_int64),
                ("msg_bits_int8", ctypes.c_int64), ("msg_bits_1bit", ctypes.c_int64),
                ("lds_bytes_per_cu", ctypes.c_int32), ("reg_slots", ctypes.c_int32),
                ("reg_rows_per_thread", ctypes.c_int32), ("reg_zpack", ctypes.c_int32),
                ("pk_slots", ctypes.c_int32), ("pk_rows_per_thread", ctypes.c_int32),
                ("pk_threads", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    """ldpc_plan_info of include/ldpc.h."""
    _fields_ = [("kernel", ctypes.c_int32), ("layout", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("frames_per_lane", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("workspace_bytes", ctypes.c_size_t)]


class Job(ctypes.Structure):
    """ldpc_job of include/ldpc_multi.h."""
    _fields_ = [("code", ctypes.c_void_p), ("n_frames", ctypes.c_int32), ("llr_in", ctypes.c_void_p),
                ("params", DecodeParams), ("hard_out", ctypes.c_void_p), ("llr_out", ctypes.c_void_p),
                ("iters_out", ctypes.c_void_p), ("syndrome_ok", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libldpc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_cs_0609090_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.ldpc_code_create.argtypes = [i32, i32, i64, vp, vp, i32, ctypes.POINTER(vp)]
        L.ldpc_code_destroy.argtypes = [vp]
        L.ldpc_code_query.argtypes = [vp, ctypes.POINTER(CodeInfo)]
        L.ldpc_decode_workspace_size.argtypes = [vp, i32, ctypes.POINTER(DecodeParams),
                                                 ctypes.POINTER(sz)]
        L.ldpc_decode_plan.argtypes = [vp, i32, ctypes.POINTER(DecodeParams), ctypes.POINTER(PlanInfo)]
        L.ldpc_decode_batch.argtypes = [vp, i32, vp, ctypes.POINTER(DecodeParams), vp, vp, vp,
                                        vp, vp, sz, vp]
        u32, dbl = ctypes.c_uint32, ctypes.c_double
        L.ldpc_encoder_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), vp]
        L.ldpc_encode_batch.argtypes = [vp, i32, vp, vp, vp]
        L.ldpc_random_bits.argtypes = [i32, i32, u32, u32, u32, u32, vp, vp]
        L.ldpc_channel_awgn.argtypes = [i32, i32, vp, vp, u32, u32, u32, u32, vp, vp, dbl, i32, vp]
        L.ldpc_count_errors.argtypes = [i32, i32, vp, vp, vp, vp]
        L.ldpc_learn_classes.argtypes = [vp, ctypes.POINTER(i32), vp]
        L.ldpc_learn_workspace_size.argtypes = [vp, i32, i32, i32, ctypes.POINTER(sz)]
        L.ldpc_learn_forward.argtypes = [vp, i32, vp, vp, i32, vp, i32, vp, sz, vp, vp, vp]
        L.ldpc_learn_backward.argtypes = [vp, i32, vp, i32, vp, i32, vp, sz, vp, vp]
        L.ldpc_multi_workspace_size.argtypes = [ctypes.POINTER(Job), i32, ctypes.POINTER(sz)]
        L.ldpc_decode_multi.argtypes = [ctypes.POINTER(Job), i32, vp, sz, vp]
        L.ldpc_autotune.argtypes = [vp, i32, ctypes.POINTER(DecodeParams), ctypes.POINTER(i32),
                                    ctypes.POINTER(ctypes.c_float), ctypes.POINTER(i32)]
        for f in ("ldpc_code_create", "ldpc_code_destroy", "ldpc_code_query",
                  "ldpc_decode_workspace_size", "ldpc_decode_plan", "ldpc_decode_batch", "ldpc_encoder_info",
                  "ldpc_encode_batch", "ldpc_random_bits", "ldpc_channel_awgn", "ldpc_count_errors",
                  "ldpc_learn_classes", "ldpc_learn_workspace_size", "ldpc_learn_forward",
                  "ldpc_learn_backward", "ldpc_multi_workspace_size", "ldpc_decode_multi",
                  "ldpc_autotune"):
            getattr(L, f).restype = ctypes.c_int
        L.ldpc_last_error.restype = ctypes.c_char_p
        L.ldpc_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status: int):
    if status != LDPC_OK:
        raise LdpcError(status, lib().ldpc_last_error().decode())


def make_params(max_iter=50, alpha=0.8, beta=0.0, early_stop=True, msg="int8",
                sched="single_scan", llr_step=0.5, check_input=False, layout="auto",
                weights=None, weight_classes=0, msg_bits=0) -> DecodeParams:
    """``weights``: None, or a float32 device tensor [T][C][2] of per-iteration
    (a, b) pairs; it must outlive the call.  C = the code's degree classes
    (``weight_classes=0``, binary32) or 1 (``weight_classes=1``: one pair per
    iteration, binary32 and fixed point).  ``msg_bits``: fixed-point message
    width 6 (default), 7 or 8 (INT8 single-scan)."""
    flags = (F_CHECK_INPUT if check_input else 0) | (LAYOUT[layout] << LAYOUT_SHIFT)
    wp = None if weights is None else weights.data_ptr()
    wt = 0 if weights is None else int(weights.shape[0])
    return DecodeParams(int(max_iter), float(alpha), float(beta), 1 if early_stop else 0,
                        MSG[msg] if isinstance(msg, str) else int(msg),
                        SCHED[sched] if isinstance(sched, str) else int(sched),
                        float(llr_step), int(flags), wp, wt, int(weight_classes), int(msg_bits))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Code:
    """Handle of a parity-check matrix resident on one GPU."""

    def __init__(self, M: int, N: int, row_ptr, col_idx, device: int = 0):
        self._h = None
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(lib().ldpc_code_create(int(M), int(N), int(rp[-1]) if rp.size else 0,
                                      rp.ctypes.data_as(ctypes.c_void_p),
                                      ci.ctypes.data_as(ctypes.c_void_p), int(device),
                                      ctypes.byref(h)))
        self._h = h
        self.M, self.N, self.device = int(M), int(N), int(device)

    @classmethod
    def from_parity_check(cls, H, device: int = 0) -> "Code":
        return cls(H.M, H.N, H.row_ptr, H.col_idx, device)

    def close(self):
        if self._h is not None and _lib is not None:
            lib().ldpc_code_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def degree_classes(self) -> np.ndarray:
        """Check-degree classes of the learned decoder (distinct row degrees)."""
        n = ctypes.c_int32()
        _check(lib().ldpc_learn_classes(self._h, ctypes.byref(n), None))
        d = np.empty(n.value, dtype=np.int32)
        _check(lib().ldpc_learn_classes(self._h, ctypes.byref(n), d.ctypes.data_as(ctypes.c_void_p)))
        return d

    def learn_workspace_size(self, n_frames: int, T: int, ckpt: int) -> int:
        b = ctypes.c_size_t()
        _check(lib().ldpc_learn_workspace_size(self._h, int(n_frames), int(T), int(ckpt), ctypes.byref(b)))
        return b.value

    def learn_forward(self, llr, target, weights, ckpt, workspace, post_out=None):
        """Raw forward pass (include/ldpc_learn.h); returns the per-iteration loss [T]."""
        T = int(weights.shape[0])
        loss = torch.empty(T, dtype=torch.float32, device=llr.device)
        _check(lib().ldpc_learn_forward(self._h, int(llr.shape[0]), _ptr(llr), _ptr(target), T, _ptr(weights),
                                        int(ckpt), _ptr(workspace), workspace.numel(), _ptr(loss),
                                        _ptr(post_out), _stream()))
        return loss

    def learn_backward(self, n_frames, target, weights, ckpt, workspace):
        """Raw adjoint: d(sum of the forward's losses)/d(weights), [T][C][2]."""
        grad = torch.empty_like(weights)
        _check(lib().ldpc_learn_backward(self._h, int(n_frames), _ptr(target), int(weights.shape[0]),
                                         _ptr(weights), int(ckpt), _ptr(workspace), workspace.numel(),
                                         _ptr(grad), _stream()))
        return grad

    def encoder_info(self) -> dict:
        """Systematic encoder of the code: kind, K and the column order
        (K information columns, then the parity columns)."""
        kind, k = ctypes.c_int32(), ctypes.c_int32()
        pos = np.empty(self.N, dtype=np.int32)
        _check(lib().ldpc_encoder_info(self._h, ctypes.byref(kind), ctypes.byref(k),
                                       pos.ctypes.data_as(ctypes.c_void_p)))
        return {"kind": ENC_KIND.get(kind.value, kind.value), "K": k.value, "info_pos": pos}

    def encode(self, info) -> "torch.Tensor":
        """uint8 [F, N] codewords of the uint8 [F, K] information words."""
        F = int(info.shape[0])
        out = torch.empty((F, self.N), dtype=torch.uint8, device=info.device)
        _check(lib().ldpc_encode_batch(self._h, F, _ptr(info), _ptr(out), _stream()))
        return out

    def info(self) -> dict:
        i = CodeInfo()
        _check(lib().ldpc_code_query(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in CodeInfo._fields_}

    def workspace_size(self, n_frames: int, params: DecodeParams) -> int:
        b = ctypes.c_size_t()
        _check(lib().ldpc_decode_workspace_size(self._h, int(n_frames), ctypes.byref(params),
                                                ctypes.byref(b)))
        return int(b.value)

    def plan(self, n_frames: int, params: DecodeParams) -> dict:
        """The plan a decode of n_frames frames follows (ldpc_decode_plan):
        kernel and layout by name, threads, LDS bytes, frames per lane,
        workspace bytes."""
        i = PlanInfo()
        _check(lib().ldpc_decode_plan(self._h, int(n_frames), ctypes.byref(params), ctypes.byref(i)))
        return {"kernel": KERNEL_NAME[i.kernel], "layout": LAYOUT_NAME[i.layout], "threads": i.threads,
                "lds_bytes": i.lds_bytes, "frames_per_lane": i.frames_per_lane,
                "workspace_bytes": int(i.workspace_bytes)}

    def decode_into(self, llr, params: DecodeParams, hard, llr_out, iters, ok, workspace,
                    stream=None) -> None:
        """Raw call: all tensors are caller-allocated device tensors."""
        n_frames = llr.shape[0] if llr.dim() == 2 else llr.numel() // self.N
        s = stream if stream is not None else torch.cuda.current_stream(llr.device)
        ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
        _check(lib().ldpc_decode_batch(self._h, int(n_frames), _ptr(llr), ctypes.byref(params),
                                       _ptr(hard), _ptr(llr_out), _ptr(iters), _ptr(ok),
                                       _ptr(workspace), ws_bytes, ctypes.c_void_p(s.cuda_stream)))

    def autotune(self, n_frames: int, params: DecodeParams) -> dict:
        """Time every layout that can run these parameters and make AUTO use
        the fastest from now on (ldpc_autotune)."""
        lay, ms, tried = ctypes.c_int32(), ctypes.c_float(), ctypes.c_int32()
        _check(lib().ldpc_autotune(self._h, int(n_frames), ctypes.byref(params), ctypes.byref(lay),
                                   ctypes.byref(ms), ctypes.byref(tried)))
        return {"layout": LAYOUT_NAME[int(lay.value)], "ms": float(ms.value), "tried": int(tried.value)}

    def alloc_outputs(self, n_frames: int, device, with_llr: bool = True) -> dict:
        return {
            "hard": torch.empty((n_frames, self.N), dtype=torch.uint8, device=device),
            "llr": torch.empty((n_frames, self.N), dtype=torch.float32, device=device)
            if with_llr else None,
            "iters": torch.empty(n_frames, dtype=torch.int32, device=device),
            "ok": torch.empty(n_frames, dtype=torch.uint8, device=device),
        }

    def alloc_workspace(self, n_frames: int, params: DecodeParams, device):
        b = self.workspace_size(n_frames, params)
        if b == 0:
            return None
        # torch's caching allocator returns 512-byte aligned blocks
        return torch.empty(b, dtype=torch.uint8, device=device)

    def decode(self, llr, max_iter=50, alpha=0.8, beta=0.0, early_stop=True, msg=None,
               sched="single_scan", llr_step=0.5, check_input=False, layout="auto",
               with_llr=True, stream=None, weights=None, weight_classes=0, msg_bits=0) -> dict:
        """Decode a [F, N] device tensor (float32 or int8) and return device
        tensors ``hard``, ``llr``, ``iters``, ``ok``."""
        if not llr.is_cuda:
            raise ValueError("llr must be a device tensor")
        llr = llr.contiguous()
        if msg is None:
            msg = "fp32" if llr.dtype == torch.float32 else "int8"
        want = torch.float32 if msg == "fp32" else torch.int8
        if llr.dtype != want:
            raise ValueError(f"msg={msg} needs a {want} tensor")
        p = make_params(max_iter, alpha, beta, early_stop, msg, sched, llr_step,
                        check_input, layout, weights, weight_classes, msg_bits)
        F = llr.shape[0]
        out = self.alloc_outputs(F, llr.device, with_llr)
        ws = self.alloc_workspace(F, p, llr.device)
        self.decode_into(llr, p, out["hard"], out["llr"], out["iters"], out["ok"], ws, stream)
        return out


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class MultiBatch:
    """Several (code, llr, params) jobs decoded together by ldpc_decode_multi
    (include/ldpc_multi.h).  Outputs and the shared workspace are allocated
    once here; ``run()`` only enqueues, so it can be captured into a graph
    (after one eager ``run()``, which creates the library's stream pool)."""

    def __init__(self, items, with_llr: bool = False):
        self.items = list(items)  # (Code, llr device tensor, DecodeParams); kept alive here
        n = len(self.items)
        self._jobs = (Job * max(n, 1))()
        self.outputs = []
        for k, (code, llr, p) in enumerate(self.items):
            F = int(llr.shape[0])
            out = code.alloc_outputs(F, llr.device, with_llr)
            self.outputs.append(out)
            self._jobs[k] = Job(code._h.value, F, llr.data_ptr(), p, out["hard"].data_ptr(),
                                None if out["llr"] is None else out["llr"].data_ptr(),
                                out["iters"].data_ptr(), out["ok"].data_ptr())
        b = ctypes.c_size_t()
        _check(lib().ldpc_multi_workspace_size(self._jobs, n, ctypes.byref(b)))
        self.workspace_bytes = int(b.value)
        dev = self.items[0][1].device if n else "cuda"
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=dev) \
            if self.workspace_bytes else None

    def run(self, stream=None) -> None:
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().ldpc_decode_multi(self._jobs, len(self.items), _ptr(self.workspace),
                                       self.workspace_bytes, ctypes.c_void_p(s.cuda_stream)))


def random_bits(n_frames: int, n_bits: int, key=(0x5EED, 0), stream_id: int = 0,
                frame_offset: int = 0, device="cuda") -> "torch.Tensor":
    """uint8 [n_frames, n_bits] of Philox4x32-10 bits (include/ldpc_sim.h)."""
    out = torch.empty((n_frames, n_bits), dtype=torch.uint8, device=device)
    _check(lib().ldpc_random_bits(int(n_frames), int(n_bits), int(key[0]) & 0xFFFFFFFF,
                                  int(key[1]) & 0xFFFFFFFF, int(stream_id), int(frame_offset),
                                  _ptr(out), _stream()))
    return out


def channel_awgn(sigma, N: int, codewords=None, key=(0x5EED, 0), stream_id: int = 0,
                 frame_offset: int = 0, want_f32: bool = True, want_q: bool = False,
                 step: float = 0.5, qmax: int = 31):
    """BPSK/AWGN channel LLRs for the frames of ``sigma`` (float64 device
    tensor, one value per frame); returns (llr_f32 or None, llr_int8 or None)."""
    F = int(sigma.shape[0])
    dev = sigma.device
    f32 = torch.empty((F, N), dtype=torch.float32, device=dev) if want_f32 else None
    q = torch.empty((F, N), dtype=torch.int8, device=dev) if want_q else None
    _check(lib().ldpc_channel_awgn(F, int(N), _ptr(codewords), _ptr(sigma), int(key[0]) & 0xFFFFFFFF,
                                   int(key[1]) & 0xFFFFFFFF, int(stream_id), int(frame_offset),
                                   _ptr(f32), _ptr(q), float(step), int(qmax), _stream()))
    return f32, q


def count_errors(hard, codewords=None) -> "torch.Tensor":
    """int32 [F]: bit errors of each frame's hard decision against its codeword."""
    F, N = int(hard.shape[0]), int(hard.shape[1])
    out = torch.empty((F,), dtype=torch.int32, device=hard.device)
    _check(lib().ldpc_count_errors(F, N, _ptr(hard), _ptr(codewords), _ptr(out), _stream()))
    return out


def version() -> str:
    return lib().ldpc_version().decode()
