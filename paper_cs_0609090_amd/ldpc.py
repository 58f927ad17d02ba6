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
NOALLOC_SCRATCH_BYTES = 128 << 20  # LDPC_NOALLOC_SCRATCH_BYTES

EXPORTS = ("ldpc_code_create", "ldpc_code_destroy", "ldpc_code_query",
           "ldpc_decode_workspace_size", "ldpc_decode_plan", "ldpc_decode_batch", "ldpc_last_error",
           "ldpc_version", "ldpc_decode_batch_noalloc",
           # include/ldpc_sim.h
           "ldpc_encoder_info", "ldpc_encode_batch", "ldpc_random_bits", "ldpc_channel_awgn",
           "ldpc_count_errors",
           # include/ldpc_learn.h
           "ldpc_learn_classes", "ldpc_learn_workspace_size", "ldpc_learn_forward",
           "ldpc_learn_backward", "ldpc_learn_backward_weighted",
           # include/ldpc_multi.h
           "ldpc_multi_workspace_size", "ldpc_decode_multi", "ldpc_autotune",
           "ldpc_multi_persistent_workspace_size", "ldpc_decode_multi_persistent",
           "ldpc_code_packed_shapes", "ldpc_code_set_packed_shape")
LAYOUT_NAME = {v: k for k, v in LAYOUT.items()}
KERNEL_NAME = {0: "generic_int", 1: "generic_f32", 2: "two_scan", 3: "reg1", 4: "packed",
               5: "f32_frames", 6: "two_scan_frames"}  # ldpc_kernel
ENC_KIND = {0: "none", 1: "staircase", 2: "dense"}
STRUCT = {0x1: "qc", 0x2: "ira", 0x4: "ira_groups"}  # LDPC_STRUCT_* bits


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
                ("pk_threads", ctypes.c_int32),
                ("row_deg_hist", ctypes.c_int32 * 65), ("col_deg_hist", ctypes.c_int32 * 65),
                ("structure", ctypes.c_int32), ("qc_lift", ctypes.c_int32), ("ira_group", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("var_values_single", ctypes.c_int64), ("var_values_two", ctypes.c_int64),
                ("msg_bytes_int8", ctypes.c_int64), ("msg_bytes_1bit", ctypes.c_int64),
                ("msg_bytes_fp32", ctypes.c_int64), ("post_bytes_int", ctypes.c_int64),
                ("post_bytes_fp32", ctypes.c_int64),
                ("stream_bytes_int8", ctypes.c_int64), ("stream_bytes_1bit", ctypes.c_int64),
                ("stream_bytes_fp32", ctypes.c_int64), ("stream_bytes_two_int8", ctypes.c_int64),
                ("stream_bytes_two_fp32", ctypes.c_int64)]


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
        L.ldpc_decode_batch_noalloc.argtypes = [vp, i32, vp, ctypes.POINTER(DecodeParams), vp, vp, vp,
                                                vp, vp]
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
        L.ldpc_learn_backward_weighted.argtypes = [vp, i32, vp, i32, vp, i32, vp, sz, vp, vp, vp]
        L.ldpc_multi_workspace_size.argtypes = [ctypes.POINTER(Job), i32, ctypes.POINTER(sz)]
        L.ldpc_decode_multi.argtypes = [ctypes.POINTER(Job), i32, vp, sz, vp]
        L.ldpc_multi_persistent_workspace_size.argtypes = [ctypes.POINTER(Job), i32, ctypes.POINTER(sz)]
        L.ldpc_decode_multi_persistent.argtypes = [ctypes.POINTER(Job), i32, vp, sz, vp]
        L.ldpc_autotune.argtypes = [vp, i32, ctypes.POINTER(DecodeParams), ctypes.POINTER(i32),
                                    ctypes.POINTER(ctypes.c_float), ctypes.POINTER(i32)]
        L.ldpc_code_packed_shapes.argtypes = [vp, ctypes.POINTER(i32), i32, ctypes.POINTER(i32)]
        L.ldpc_code_set_packed_shape.argtypes = [vp, i32, i32, i32]
        for f in ("ldpc_code_create", "ldpc_code_destroy", "ldpc_code_query",
                  "ldpc_decode_workspace_size", "ldpc_decode_plan", "ldpc_decode_batch",
                  "ldpc_decode_batch_noalloc", "ldpc_encoder_info",
                  "ldpc_encode_batch", "ldpc_random_bits", "ldpc_channel_awgn", "ldpc_count_errors",
                  "ldpc_learn_classes", "ldpc_learn_workspace_size", "ldpc_learn_forward",
                  "ldpc_learn_backward", "ldpc_learn_backward_weighted", "ldpc_multi_workspace_size",
                  "ldpc_decode_multi", "ldpc_multi_persistent_workspace_size", "ldpc_decode_multi_persistent",
                  "ldpc_autotune", "ldpc_code_packed_shapes", "ldpc_code_set_packed_shape"):
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
    if weights is not None:
        # (the device is checked per decode call: planning calls never read the pairs)
        if not isinstance(weights, torch.Tensor) or weights.dtype != torch.float32 or \
                weights.dim() != 3 or weights.shape[2] != 2 or \
                weights.shape[0] < 1 or not weights.is_contiguous():
            raise ValueError("weights must be a contiguous float32 tensor [T][C][2], T >= 1")
    wp = None if weights is None else weights.data_ptr()
    wt = 0 if weights is None else int(weights.shape[0])
    p = DecodeParams(int(max_iter), float(alpha), float(beta), 1 if early_stop else 0,
                     MSG[msg] if isinstance(msg, str) else int(msg),
                     SCHED[sched] if isinstance(sched, str) else int(sched),
                     float(llr_step), int(flags), wp, wt, int(weight_classes), int(msg_bits))
    p._weights = weights  # kept alive with the parameters and checked against the code per call
    return p


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t, name: str, dtype, shape, device: int, optional: bool = False) -> None:
    """Raise ValueError unless ``t`` is a contiguous ``dtype`` tensor of
    exactly ``shape`` on cuda:``device`` (or None when ``optional``).  The
    kernels index these buffers by the code's sizes, so a wrong shape or
    device would otherwise be read or written out of bounds."""
    if t is None:
        if optional:
            return
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"{name} must be on cuda:{device} (the code's device), not {t.device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, not {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, not {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


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

    @property
    def n_classes(self) -> int:
        """Number of check-degree classes (distinct row degrees)."""
        if getattr(self, "_n_classes", None) is None:
            n = ctypes.c_int32()
            _check(lib().ldpc_learn_classes(self._h, ctypes.byref(n), None))
            self._n_classes = int(n.value)
        return self._n_classes

    def _check_weights(self, params: DecodeParams) -> None:
        """The weights a DecodeParams points at must match the code: float32
        [weight_iters][C][2] on its device, C = 1 or the code's classes."""
        if not params.weights:
            return
        w = getattr(params, "_weights", None)
        if w is None:
            raise ValueError("params.weights must be set by make_params(weights=...) so that it can be checked")
        C = 1 if params.weight_classes == 1 else self.n_classes
        _need(w, "weights", torch.float32, (int(params.weight_iters), C, 2), self.device)
        if w.data_ptr() != params.weights:
            raise ValueError("params.weights does not point at the tensor make_params was given")

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
        if not isinstance(llr, torch.Tensor) or llr.dim() != 2:
            raise ValueError("llr must be a float32 device tensor [F, N]")
        F = int(llr.shape[0])
        _need(llr, "llr", torch.float32, (F, self.N), self.device)
        _need(target, "target", torch.uint8, (F, self.N), self.device, optional=True)
        if not isinstance(weights, torch.Tensor) or weights.dim() != 3:
            raise ValueError("weights must be a float32 device tensor [T][C][2]")
        T = int(weights.shape[0])
        _need(weights, "weights", torch.float32, (T, self.n_classes, 2), self.device)
        _need(post_out, "post_out", torch.float32, (F, self.N), self.device, optional=True)
        _need(workspace, "workspace", torch.uint8, (workspace.numel(),), self.device)
        loss = torch.empty(T, dtype=torch.float32, device=llr.device)
        _check(lib().ldpc_learn_forward(self._h, int(llr.shape[0]), _ptr(llr), _ptr(target), T, _ptr(weights),
                                        int(ckpt), _ptr(workspace), workspace.numel(), _ptr(loss),
                                        _ptr(post_out), _stream()))
        return loss

    def learn_backward(self, n_frames, target, weights, ckpt, workspace, loss_weights=None):
        """Raw adjoint: d(sum_t w_t loss_t)/d(weights), [T][C][2]; w_t from
        ``loss_weights`` (a sequence of T finite numbers, copied to the host),
        all ones if None."""
        F = int(n_frames)
        _need(target, "target", torch.uint8, (F, self.N), self.device, optional=True)
        if not isinstance(weights, torch.Tensor) or weights.dim() != 3:
            raise ValueError("weights must be a float32 device tensor [T][C][2]")
        _need(weights, "weights", torch.float32, (int(weights.shape[0]), self.n_classes, 2), self.device)
        _need(workspace, "workspace", torch.uint8, (workspace.numel(),), self.device)
        grad = torch.empty_like(weights)
        T = int(weights.shape[0])
        lw = None
        if loss_weights is not None:
            lw = np.ascontiguousarray(np.asarray(loss_weights, dtype=np.float32).reshape(-1))
            if lw.size != T:
                raise ValueError(f"loss_weights must hold T = {T} values, not {lw.size}")
        _check(lib().ldpc_learn_backward_weighted(self._h, int(n_frames), _ptr(target), T,
                                                  _ptr(weights), int(ckpt), _ptr(workspace), workspace.numel(),
                                                  None if lw is None else lw.ctypes.data_as(ctypes.c_void_p),
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
        """ldpc_code_query as a dict; histograms as lists, ``structure`` as
        the set of names of its LDPC_STRUCT_* bits."""
        i = CodeInfo()
        _check(lib().ldpc_code_query(self._h, ctypes.byref(i)))
        d = {k: getattr(i, k) for k, _ in CodeInfo._fields_}
        d["row_deg_hist"] = list(i.row_deg_hist)
        d["col_deg_hist"] = list(i.col_deg_hist)
        d["structure"] = {n for b, n in STRUCT.items() if i.structure & b}
        return d

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
        """Raw call: all tensors are caller-allocated device tensors on the
        code's device: llr [F, N] (float32 for FP32 messages, int8 otherwise),
        hard uint8 [F, N], llr_out float32 [F, N] or None, iters int32 [F],
        ok uint8 [F], workspace uint8 (or None).  Checked here (ValueError)
        before the library is called."""
        self.check_io(llr, params, hard, llr_out, iters, ok, workspace)
        n_frames = int(llr.shape[0])
        s = stream if stream is not None else torch.cuda.current_stream(llr.device)
        ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
        _check(lib().ldpc_decode_batch(self._h, int(n_frames), _ptr(llr), ctypes.byref(params),
                                       _ptr(hard), _ptr(llr_out), _ptr(iters), _ptr(ok),
                                       _ptr(workspace), ws_bytes, ctypes.c_void_p(s.cuda_stream)))

    def decode_noalloc_into(self, llr, params: DecodeParams, hard, llr_out, iters, ok, stream=None) -> None:
        """ldpc_decode_batch_noalloc: as ``decode_into`` with no workspace
        argument; the library takes it from its static per-device scratch of
        NOALLOC_SCRATCH_BYTES (calls overlapping on one GPU race)."""
        self.check_io(llr, params, hard, llr_out, iters, ok, None)
        s = stream if stream is not None else torch.cuda.current_stream(llr.device)
        _check(lib().ldpc_decode_batch_noalloc(self._h, int(llr.shape[0]), _ptr(llr), ctypes.byref(params),
                                               _ptr(hard), _ptr(llr_out), _ptr(iters), _ptr(ok),
                                               ctypes.c_void_p(s.cuda_stream)))

    def check_io(self, llr, params: DecodeParams, hard, llr_out, iters, ok, workspace) -> None:
        """Shape, dtype, contiguity and device of one decode call's buffers."""
        if not isinstance(llr, torch.Tensor) or llr.dim() != 2:
            raise ValueError(f"llr must be a device tensor [F, {self.N}]")
        F = int(llr.shape[0])
        _need(llr, "llr", torch.float32 if params.msg == MSG["fp32"] else torch.int8, (F, self.N), self.device)
        _need(hard, "hard", torch.uint8, (F, self.N), self.device)
        _need(llr_out, "llr_out", torch.float32, (F, self.N), self.device, optional=True)
        _need(iters, "iters", torch.int32, (F,), self.device)
        _need(ok, "ok", torch.uint8, (F,), self.device)
        if workspace is not None:
            _need(workspace, "workspace", torch.uint8, (workspace.numel(),), self.device)
        self._check_weights(params)

    def autotune(self, n_frames: int, params: DecodeParams) -> dict:
        """Time every layout that can run these parameters (and, for the packed
        kernel, each of packed_shapes()) and make AUTO use the fastest from now
        on (ldpc_autotune)."""
        lay, ms, tried = ctypes.c_int32(), ctypes.c_float(), ctypes.c_int32()
        _check(lib().ldpc_autotune(self._h, int(n_frames), ctypes.byref(params), ctypes.byref(lay),
                                   ctypes.byref(ms), ctypes.byref(tried)))
        return {"layout": LAYOUT_NAME[int(lay.value)], "ms": float(ms.value), "tried": int(tried.value)}

    def packed_shapes(self) -> list[tuple[int, int, int]]:
        """(slots per lane, rows per thread, threads) of the packed shapes that
        autotune times, the handle's current one first (ldpc_code_packed_shapes)."""
        n = ctypes.c_int32()
        _check(lib().ldpc_code_packed_shapes(self._h, None, 0, ctypes.byref(n)))
        buf = (ctypes.c_int32 * max(3 * n.value, 1))()
        _check(lib().ldpc_code_packed_shapes(self._h, buf, n.value, ctypes.byref(n)))
        return [(buf[3 * i], buf[3 * i + 1], buf[3 * i + 2]) for i in range(n.value)]

    def set_packed_shape(self, slots: int, rows_per_thread: int, threads: int) -> None:
        """Make one of packed_shapes() the handle's (ldpc_code_set_packed_shape)."""
        _check(lib().ldpc_code_set_packed_shape(self._h, int(slots), int(rows_per_thread), int(threads)))

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
        if not isinstance(llr, torch.Tensor) or not llr.is_cuda:
            raise ValueError("llr must be a device tensor")
        if msg is None:
            msg = "fp32" if llr.dtype == torch.float32 else "int8"
        want = torch.float32 if msg == "fp32" else torch.int8
        if llr.dtype != want:
            raise ValueError(f"msg={msg} needs a {want} tensor")
        if llr.dim() != 2 or llr.shape[1] != self.N or llr.device.index != self.device:
            raise ValueError(f"llr must be [F, {self.N}] on cuda:{self.device}, not "
                             f"{list(llr.shape)} on {llr.device}")
        p = make_params(max_iter, alpha, beta, early_stop, msg, sched, llr_step,
                        check_input, layout, weights, weight_classes, msg_bits)
        cur = torch.cuda.current_stream(llr.device)
        s = stream if stream is not None else cur
        llr = llr.contiguous()  # on the current stream, like the caller's own writes to llr
        if s != cur:
            # the decode on `s` must see llr (and the copy just made) complete;
            # outputs and workspace come from `s`'s pool, and the inputs are
            # marked as used there so that the allocator does not reuse them early
            s.wait_stream(cur)
            llr.record_stream(s)
            if weights is not None:
                weights.record_stream(s)
        F = llr.shape[0]
        with torch.cuda.stream(s):
            out = self.alloc_outputs(F, llr.device, with_llr)
            ws = self.alloc_workspace(F, p, llr.device)
        self.decode_into(llr, p, out["hard"], out["llr"], out["iters"], out["ok"], ws, s)
        return out


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class MultiBatch:
    """Several (code, llr, params) jobs decoded together by ldpc_decode_multi
    (include/ldpc_multi.h), or with ``persistent=True`` by
    ldpc_decode_multi_persistent (one launch).  Outputs and the shared
    workspace are allocated once here; ``run()`` only enqueues, so it can be
    captured into a graph (after one eager ``run()``, which creates the
    library's stream pool)."""

    def __init__(self, items, with_llr: bool = False, persistent: bool = False):
        self.persistent = persistent
        self.items = list(items)  # (Code, llr device tensor, DecodeParams); kept alive here
        n = len(self.items)
        self._jobs = (Job * max(n, 1))()
        self.outputs = []
        for k, (code, llr, p) in enumerate(self.items):
            if not isinstance(llr, torch.Tensor) or llr.dim() != 2:
                raise ValueError(f"job {k}: llr must be a device tensor [F, {code.N}]")
            F = int(llr.shape[0])
            out = code.alloc_outputs(F, llr.device, with_llr)
            code.check_io(llr, p, out["hard"], out["llr"], out["iters"], out["ok"], None)
            self.outputs.append(out)
            self._jobs[k] = Job(code._h.value, F, llr.data_ptr(), p, out["hard"].data_ptr(),
                                None if out["llr"] is None else out["llr"].data_ptr(),
                                out["iters"].data_ptr(), out["ok"].data_ptr())
        b = ctypes.c_size_t()
        size_fn = lib().ldpc_multi_persistent_workspace_size if persistent else lib().ldpc_multi_workspace_size
        _check(size_fn(self._jobs, n, ctypes.byref(b)))
        self.workspace_bytes = int(b.value)
        dev = self.items[0][1].device if n else "cuda"
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=dev) \
            if self.workspace_bytes else None

    def run(self, stream=None) -> None:
        s = stream if stream is not None else torch.cuda.current_stream()
        fn = lib().ldpc_decode_multi_persistent if self.persistent else lib().ldpc_decode_multi
        _check(fn(self._jobs, len(self.items), _ptr(self.workspace), self.workspace_bytes,
                  ctypes.c_void_p(s.cuda_stream)))


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
