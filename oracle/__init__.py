"""ctypes front-end of the CPU oracle (``oracle.c``) -- TEST INFRASTRUCTURE.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The decoder library does not use it.

``decode(code, llr, algo=..., arith=...)`` runs one of the three decoders of
the paper (two-scan Sec. III, single-scan Sec. IV, 1-bit Sec. V) in b-bit
fixed point (``arith='int'``, int8 input; b = 6, or 6-8 with ``qbits`` for
single-scan and 1-bit), binary32 or binary64 and returns numpy arrays.
``sched`` (fixed point, single-scan and 1-bit) is a [T][2] array of
per-iteration (alpha_k, beta_k) pairs; iteration k uses row min(k, T) - 1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "oracle_float.inc")]
_lib = None

ALGOS = ("two_scan", "single_scan", "one_bit")
ARITHS = ("int", "f32", "f64")


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, no FP contraction).  ``sanitize``:
    with AddressSanitizer and UndefinedBehaviorSanitizer (load it with gcc's
    libasan preloaded: LD_PRELOAD=$(gcc -print-file-name=libasan.so))."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-fno-omit-frame-pointer"] if sanitize else []
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", *san, "-o", tmp, _SRC[0], "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or any(
                os.path.getmtime(s) > os.path.getmtime(_LIB_PATH) for s in _SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB_PATH)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def decode(code, llr, algo: str = "single_scan", arith: str = "int", max_iter: int = 50,
           alpha: float = 0.8, beta: float = 0.0, early_stop: bool = True,
           step: float = 0.5, trace: bool = False, state: bool = False, sched=None,
           qbits: int = 6) -> dict:
    """Decode a batch [F, N].  Returns dict with ``post`` (float32 for int and
    f32, float64 for f64), ``hard`` (uint8), ``iters`` (int32), ``ok`` (uint8)
    and, with ``trace``, per-iteration ``L`` [F, max_iter, E], ``Z``
    [F, max_iter, N] (and ``Zmn`` for two-scan)."""
    if algo not in ALGOS or arith not in ARITHS:
        raise ValueError("bad algo/arith")
    L = lib()
    rp = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(code.col_idx, dtype=np.int32)
    M, N, E = int(code.M), int(code.N), int(rp[-1])
    if arith == "int":
        x = np.ascontiguousarray(llr, dtype=np.int8).reshape(-1, N)
        real, post_t = np.int32, np.float32
    else:
        x = np.ascontiguousarray(llr, dtype=np.float32).reshape(-1, N)
        real = np.float32 if arith == "f32" else np.float64
        post_t = real
    F = x.shape[0]
    post = np.zeros((F, N), dtype=post_t)
    hard = np.zeros((F, N), dtype=np.uint8)
    iters = np.zeros(F, dtype=np.int32)
    ok = np.zeros(F, dtype=np.uint8)
    T = max(max_iter, 1)
    tl = np.zeros((F, T, E), dtype=real) if trace else None
    tz = np.zeros((F, T, N), dtype=real) if trace else None
    tzmn = np.zeros((F, T, E), dtype=real) if (trace and algo == "two_scan") else None
    out = {}
    ex = sched is not None or qbits != 6
    if ex and (arith != "int" or algo == "two_scan"):
        raise ValueError("schedules and message widths: fixed-point single-scan and 1-bit only")
    sch = None if sched is None else np.ascontiguousarray(sched, dtype=np.float64).reshape(-1, 2)
    common = [ctypes.c_int(M), ctypes.c_int(N), _p(rp), _p(ci), ctypes.c_int(F), _p(x),
              ctypes.c_int(max_iter)]
    if ex:
        common += [_p(sch), ctypes.c_int(0 if sch is None else sch.shape[0])]
    common += [ctypes.c_double(alpha), ctypes.c_double(beta)]
    if ex:
        common.append(ctypes.c_int(qbits))
    common.append(ctypes.c_int(1 if early_stop else 0))
    if arith == "int":
        common.append(ctypes.c_double(step))
    tail = [_p(post), _p(hard), _p(iters), _p(ok), _p(tl), _p(tz)]
    if algo == "two_scan":
        tail.append(_p(tzmn))
    st = sg = None
    if algo == "one_bit" and arith == "int":
        st = np.zeros((F, M, 3), dtype=np.int32) if state else None
        sg = np.zeros((F, E), dtype=np.uint8) if state else None
        tail += [_p(st), _p(sg)]
    fn = getattr(L, (f"oracle_{algo}_int" + ("_ex" if ex else "")) if arith == "int" else f"oracle_{algo}_{arith}")
    rc = fn(*common, *tail)
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (rc={rc})")
    out.update(post=post, hard=hard, iters=iters, ok=ok)
    if trace:
        out.update(L=tl, Z=tz)
        if tzmn is not None:
            out["Zmn"] = tzmn
    if st is not None:
        out.update(state=st, signs=sg)
    return out


def row_update_int(t, alpha=1.0, beta=0.0, step=0.5) -> np.ndarray:
    """Literal check update of one row in fixed point (Eq.(1))."""
    t = np.ascontiguousarray(t, dtype=np.int32)
    out = np.zeros_like(t)
    lib().oracle_row_update_int(ctypes.c_int(t.size), _p(t), ctypes.c_double(alpha),
                                ctypes.c_double(beta), ctypes.c_double(step), _p(out))
    return out


def compress_row_int(L):
    """Sec. V compression of one row: (A, B, n~, signs)."""
    L = np.ascontiguousarray(L, dtype=np.int32)
    A, B, ix = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    s = np.zeros(L.size, dtype=np.uint8)
    lib().oracle_compress_row_int(ctypes.c_int(L.size), _p(L), ctypes.byref(A),
                                  ctypes.byref(B), ctypes.byref(ix), _p(s))
    return A.value, B.value, ix.value, s


def expand_row_int(d, A, B, idx, s) -> np.ndarray:
    """L_mn = s_mn f(A, B, n, n~) for one row."""
    s = np.ascontiguousarray(s, dtype=np.uint8)
    out = np.zeros(d, dtype=np.int32)
    lib().oracle_expand_row_int(ctypes.c_int(d), ctypes.c_int32(A), ctypes.c_int32(B),
                                ctypes.c_int32(idx), _p(s), _p(out))
    return out
