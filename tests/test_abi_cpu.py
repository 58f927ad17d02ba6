"""C-ABI surface on the CPU: the library loads, exports every symbol of
include/ldpc.h, validates codes and parameters, and sizes workspaces, all
without a GPU (host-only handles, device = -1)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_cs_0609090_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_cs_0609090_amd import ldpc
    return ldpc


def _declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ldpc_\w+)\s*\(", src, flags=re.M))
    return sorted(names)


def test_exports_every_declared_symbol(L):
    names = _declared_functions()
    assert len(names) >= 12
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)
    assert L.version().startswith("ldpc")


def test_struct_layouts_match_header(L, tmp_path):
    """The ctypes mirrors of ldpc_decode_params / ldpc_code_info have the
    C compiler's sizes and field offsets."""
    import subprocess
    fields = {"ldpc_decode_params": [f for f, _ in L.DecodeParams._fields_],
              "ldpc_code_info": [f for f, _ in L.CodeInfo._fields_],
              "ldpc_job": [f for f, _ in L.Job._fields_],
              "ldpc_plan_info": [f for f, _ in L.PlanInfo._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ldpc.h"', '#include "ldpc_multi.h"',
             'int main(void) {']
    for st, fs in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append('return 0; }')
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    for st, cls in (("ldpc_decode_params", L.DecodeParams), ("ldpc_code_info", L.CodeInfo), ("ldpc_job", L.Job),
                    ("ldpc_plan_info", L.PlanInfo)):
        assert int(out[st]) == ctypes.sizeof(cls), st
        for f in fields[st]:
            assert int(out[f"{st}.{f}"]) == getattr(cls, f).offset, f"{st}.{f}"


def _create(L, M, N, rp, ci, device=-1):
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    st = L.lib().ldpc_code_create(M, N, int(rp[-1]) if rp.size else 0,
                                  rp.ctypes.data_as(ctypes.c_void_p),
                                  ci.ctypes.data_as(ctypes.c_void_p), device, ctypes.byref(h))
    return st, h


def test_bad_codes_rejected(L):
    # degree-1 row
    st, _ = _create(L, 2, 4, [0, 1, 3], [0, 1, 2])
    assert st == L.LDPC_EBADCODE and b"degree" in L.lib().ldpc_last_error()
    # duplicate entry
    st, _ = _create(L, 1, 4, [0, 3], [1, 2, 1])
    assert st == L.LDPC_EBADCODE and b"duplicate" in L.lib().ldpc_last_error()
    # out of range
    st, _ = _create(L, 1, 4, [0, 2], [1, 4])
    assert st == L.LDPC_EBADCODE
    st, _ = _create(L, 1, 4, [0, 2], [-1, 2])
    assert st == L.LDPC_EBADCODE
    # inconsistent row_ptr
    st, _ = _create(L, 2, 4, [1, 2, 4], [0, 1, 2, 3])
    assert st == L.LDPC_EBADCODE
    st, _ = _create(L, 2, 4, [0, 3, 2], [0, 1, 2, 3])
    assert st == L.LDPC_EBADCODE
    # row degree above 64
    st, _ = _create(L, 1, 70, [0, 65], np.arange(65))
    assert st == L.LDPC_EUNSUPPORTED
    # null pointers
    h = ctypes.c_void_p()
    assert L.lib().ldpc_code_create(1, 4, 2, None, None, -1, ctypes.byref(h)) == L.LDPC_EINVAL
    assert L.lib().ldpc_code_create(1, 4, 2, None, None, -1, None) == L.LDPC_EINVAL


def test_host_only_handle_query_and_footprint(L):
    """P11: single-scan needs only the check-to-variable index (half of the
    two-scan addressing, Sec. IV); the 1-bit store is E sign bits plus
    M (5 + 5 + ceil(log2 d_c)) state bits (Sec. V)."""
    code = W.code_c0_peg1008()
    c = L.Code.from_parity_check(code, device=-1)
    info = c.info()
    assert (info["M"], info["N"], info["E"]) == (504, 1008, 3024)
    assert info["max_row_deg"] == 6 and info["min_row_deg"] == 6 and info["max_col_deg"] == 3
    assert info["rows_padded"] == 512
    assert info["addr_bytes_two"] == 2 * info["addr_bytes_single"]
    assert info["msg_bits_int8"] == 8 * 3024
    assert info["msg_bits_1bit"] == 3024 + 504 * (5 + 5 + 3)
    assert info["lds_bytes_per_cu"] == 160 * 1024
    c.close()


def test_param_validation(L):
    c = L.Code.from_parity_check(W.code_c0_peg1008(), device=-1)
    ok = L.make_params()
    assert c.workspace_size(10, ok) == 0  # everything of the 1008-bit code fits in LDS
    bad = [L.make_params(max_iter=-1), L.make_params(alpha=0.0), L.make_params(alpha=1.5),
           L.make_params(beta=-0.1), L.make_params(llr_step=0.0), L.make_params(msg=7),
           L.make_params(sched=3)]
    for p in bad:
        with pytest.raises(L.LdpcError) as ei:
            c.workspace_size(10, p)
        assert ei.value.status == L.LDPC_EINVAL
    with pytest.raises(L.LdpcError) as ei:
        c.workspace_size(10, L.make_params(msg="1bit", sched="two_scan"))
    assert ei.value.status == L.LDPC_EUNSUPPORTED
    with pytest.raises(L.LdpcError) as ei:
        c.workspace_size(-1, ok)
    assert ei.value.status == L.LDPC_EINVAL
    # a host-only handle cannot decode
    p = L.make_params()
    st = L.lib().ldpc_decode_batch(c._h, 1, None, ctypes.byref(p), None, None, None, None,
                                   None, 0, None)
    assert st == L.LDPC_EINVAL
    c.close()


def test_workspace_plans(L):
    """Layout planning: fixed-point messages of the 64800-bit code live in
    registers (no workspace); the generic kernels keep them in the workspace;
    smaller codes fit in LDS; forcing HBM always costs workspace."""
    big = L.Code.from_parity_check(W.code_c2_ira64800(), device=-1)
    info = big.info()
    assert (info["reg_slots"], info["reg_rows_per_thread"], info["reg_zpack"]) == (7, 32, 3)
    assert (info["pk_slots"], info["pk_rows_per_thread"], info["pk_threads"]) == (7, 32, 1024)
    # rows of up to 21 slots: 11 slots on each lane of a pair, 512 threads
    qc = L.Code.from_parity_check(W.code_c1_qc7493(), device=-1).info()
    assert (qc["pk_slots"], qc["pk_rows_per_thread"], qc["pk_threads"]) == (11, 12, 512)
    for msg in ("int8", "1bit"):
        assert big.workspace_size(4, L.make_params(msg=msg)) == 0
        assert big.workspace_size(4, L.make_params(msg=msg, layout="reg")) == 0
        assert big.workspace_size(4, L.make_params(msg=msg, layout="reg1")) == 0
        assert big.workspace_size(4, L.make_params(msg=msg, layout="hbm")) > 0
    # binary32 single-scan of the big code streams frames-across-lanes: the
    # workspace covers the call (64-frame groups) and holds one flag row per iteration
    f1 = big.workspace_size(1, L.make_params(msg="fp32"))
    assert f1 == big.workspace_size(64, L.make_params(msg="fp32"))
    assert f1 >= 64 * 4 * (3 * 64800 + 226799)
    assert big.workspace_size(65, L.make_params(msg="fp32")) > f1
    assert big.workspace_size(1, L.make_params(msg="fp32", max_iter=80)) > f1
    assert big.workspace_size(1, L.make_params(msg="fp32", layout="frames")) == f1
    for bad in (dict(msg="int8", layout="frames"), dict(msg="1bit", layout="frames"),
                dict(msg="1bit", sched="two_scan", layout="frames")):
        with pytest.raises(L.LdpcError) as ei:
            big.workspace_size(4, L.make_params(**bad))
        assert ei.value.status == L.LDPC_EUNSUPPORTED
    # the two-scan baseline of the big code streams both per-edge arrays (Z_mn
    # and L_mn) frames-across-lanes: int8 1 byte per edge and frame, fp32 4
    t8 = big.workspace_size(64, L.make_params(msg="int8", sched="two_scan"))
    t32 = big.workspace_size(64, L.make_params(msg="fp32", sched="two_scan"))
    assert t8 >= 64 * (2 * 226799 + 64800 + 2 * 64800)
    assert t32 >= 64 * 4 * (2 * 226799 + 2 * 64800) and t32 > 3 * t8
    assert t8 == big.workspace_size(64, L.make_params(msg="int8", sched="two_scan", layout="frames"))
    with pytest.raises(L.LdpcError) as ei:
        big.workspace_size(4, L.make_params(msg="fp32", layout="reg"))
    assert ei.value.status == L.LDPC_EUNSUPPORTED
    b1 = big.workspace_size(1, L.make_params(msg="int8", layout="hbm"))
    assert big.workspace_size(8, L.make_params(msg="int8", layout="hbm")) == 8 * b1
    assert b1 >= 226799  # one int8 message per edge
    small = L.Code.from_parity_check(W.code_c0_peg1008(), device=-1)
    for msg in ("int8", "1bit", "fp32"):
        assert small.workspace_size(4, L.make_params(msg=msg)) == 0
        assert small.workspace_size(4, L.make_params(msg=msg, layout="hbm")) > 0
    assert small.workspace_size(4, L.make_params(msg="int8", sched="two_scan")) == 0
    chk = small.workspace_size(4, L.make_params(msg="int8", check_input=True))
    assert chk >= 4
    with pytest.raises(L.LdpcError) as ei:
        big.workspace_size(4, L.make_params(msg="fp32", layout="lds"))
    assert ei.value.status == L.LDPC_EUNSUPPORTED
    big.close()
    small.close()


def _gf2_rank(rows: np.ndarray) -> int:
    """Rank over GF(2) of a 0/1 matrix (plain elimination on packed rows)."""
    A = np.packbits(rows.astype(np.uint8), axis=1)
    r = 0
    ncols = rows.shape[1]
    for c in range(ncols):
        byte, bit = c // 8, 0x80 >> (c % 8)
        piv = np.nonzero(A[r:, byte] & bit)[0]
        if piv.size == 0:
            continue
        p = r + piv[0]
        A[[r, p]] = A[[p, r]]
        hit = np.nonzero(A[:, byte] & bit)[0]
        hit = hit[hit != r]
        A[hit] ^= A[r]
        r += 1
        if r == A.shape[0]:
            break
    return r


@pytest.mark.parametrize("name", ["peg1008", "ira16200", "ira64800", "qc7493", "tiny"])
def test_encoder_description(L, name):
    """The systematic split the encoder reports is valid: K = N - rank(H) and
    the parity columns carry a nonsingular submatrix (so every information
    word has exactly one codeword).  IRA codes take the staircase form with
    the information bits first."""
    code = {"peg1008": W.code_c0_peg1008, "ira16200": W.code_ira16200, "ira64800": W.code_c2_ira64800,
            "qc7493": W.code_c1_qc7493,
            "tiny": lambda: W.random_small_code(9, 20, (2, 6), seed=77)}[name]()
    c = L.Code.from_parity_check(code, device=-1)
    e = c.encoder_info()
    c.close()
    pos = e["info_pos"]
    K = e["K"]
    assert sorted(pos.tolist()) == list(range(code.N))
    assert list(pos[:K]) == sorted(pos[:K].tolist())
    if name.startswith("ira"):
        assert e["kind"] == "staircase" and K == code.N - code.M
        assert list(pos) == list(range(code.N))
        return
    assert e["kind"] == "dense"
    H = code.dense()
    rank = _gf2_rank(H)
    assert K == code.N - rank
    assert _gf2_rank(H[:, pos[K:]]) == rank


# ---------------------------------------------------------------------------
# mixed batches (include/ldpc_multi.h), host side
def _host_code(L, code):
    st, h = _create(L, code.M, code.N, code.row_ptr, code.col_idx)
    assert st == L.LDPC_OK
    return h


def _job(L, h, F, p, fake=0x100000):
    return L.Job(h.value, F, fake, p, fake, None, fake, fake)


def test_multi_workspace_is_the_concatenation(L):
    """ldpc_multi_workspace_size = the jobs' ldpc_decode_workspace_size,
    each started on a 256-byte boundary, in job order."""
    codes = [W.code_c0_peg1008(), W.code_ira16200(), W.random_small_code(40, 90, (3, 9), seed=31)]
    hs = [_host_code(L, c) for c in codes]
    plist = [L.make_params(msg="int8", layout="hbm"), L.make_params(msg="fp32", max_iter=20),
             L.make_params(msg="fp32", sched="two_scan", layout="hbm"),
             L.make_params(msg="int8", sched="two_scan", max_iter=7, layout="frames")]
    sel = [(0, 0, 333), (1, 1, 65), (2, 2, 7), (1, 3, 129), (0, 1, 0)]
    jobs = (L.Job * len(sel))()
    want = 0
    for k, (ci, pi, F) in enumerate(sel):
        b = ctypes.c_size_t()
        assert L.lib().ldpc_decode_workspace_size(hs[ci], F, ctypes.byref(plist[pi]), ctypes.byref(b)) == 0
        want = (want + 255) // 256 * 256 + b.value
        jobs[k] = _job(L, hs[ci], F, plist[pi])
    got = ctypes.c_size_t()
    assert L.lib().ldpc_multi_workspace_size(jobs, len(sel), ctypes.byref(got)) == L.LDPC_OK
    assert got.value == want and want > 0
    for h in hs:
        L.lib().ldpc_code_destroy(h)


def test_multi_argument_errors(L):
    code = W.code_c0_peg1008()
    h = _host_code(L, code)
    p = L.make_params(msg="int8")
    lib = L.lib()
    sz = ctypes.c_size_t()
    jobs = (L.Job * 2)(_job(L, h, 10, p), _job(L, h, 20, p))
    assert lib.ldpc_multi_workspace_size(jobs, -1, ctypes.byref(sz)) == L.LDPC_EINVAL
    assert lib.ldpc_multi_workspace_size(None, 2, ctypes.byref(sz)) == L.LDPC_EINVAL
    assert lib.ldpc_multi_workspace_size(jobs, 0, ctypes.byref(sz)) == L.LDPC_OK and sz.value == 0
    # a missing code names its job
    jobs[1].code = None
    assert lib.ldpc_multi_workspace_size(jobs, 2, ctypes.byref(sz)) == L.LDPC_EINVAL
    assert lib.ldpc_last_error().startswith(b"job 1:")
    jobs[1].code = h.value
    # invalid parameters of one job reject the whole call
    jobs[1].params.alpha = 1.5
    assert lib.ldpc_decode_multi(jobs, 2, None, 0, None) == L.LDPC_EINVAL
    assert b"job 1:" in lib.ldpc_last_error() and b"alpha" in lib.ldpc_last_error()
    jobs[1].params.alpha = 0.8
    # the synchronising input check is not allowed inside a mixed call
    jobs[0].params.flags |= L.F_CHECK_INPUT
    assert lib.ldpc_decode_multi(jobs, 2, None, 0, None) == L.LDPC_EINVAL
    assert b"CHECK_INPUT" in lib.ldpc_last_error()
    jobs[0].params.flags &= ~L.F_CHECK_INPUT
    # a missing output pointer, and host-only handles, fail before any launch
    jobs[0].iters_out = None
    assert lib.ldpc_decode_multi(jobs, 2, None, 0, None) == L.LDPC_EINVAL
    assert lib.ldpc_last_error().startswith(b"job 0:")
    jobs[0].iters_out = 0x100000
    assert lib.ldpc_decode_multi(jobs, 2, None, 0, None) == L.LDPC_EINVAL
    assert b"host-only" in lib.ldpc_last_error()
    # workspace checks of the whole call
    jobs2 = (L.Job * 1)(_job(L, h, 10, L.make_params(msg="int8", layout="hbm")))
    assert lib.ldpc_multi_workspace_size(jobs2, 1, ctypes.byref(sz)) == 0 and sz.value > 0
    assert lib.ldpc_decode_multi(jobs2, 1, None, 0, None) == L.LDPC_EINVAL
    assert lib.ldpc_decode_multi(jobs2, 1, ctypes.c_void_p(0x100000), sz.value - 1, None) == L.LDPC_EINVAL
    assert lib.ldpc_decode_multi(jobs2, 1, ctypes.c_void_p(0x100010), sz.value, None) == L.LDPC_EINVAL
    assert b"aligned" in lib.ldpc_last_error()
    # autotuning needs a device handle and no per-iteration weights
    lay = ctypes.c_int32()
    assert lib.ldpc_autotune(h, 64, ctypes.byref(p), ctypes.byref(lay), None, None) == L.LDPC_EINVAL
    assert lib.ldpc_autotune(h, 0, ctypes.byref(p), ctypes.byref(lay), None, None) == L.LDPC_EINVAL
    lib.ldpc_code_destroy(h)


# ---------------------------------------------------------------------------
# per-iteration schedules and 7-8 bit messages: validation and planning
def test_schedule_and_width_validation(L):
    import torch
    small = L.Code.from_parity_check(W.code_c0_peg1008(), device=-1)        # one degree class
    irr = L.Code.from_parity_check(W.random_small_code(40, 90, (3, 9), seed=31), device=-1)
    big = L.Code.from_parity_check(W.code_ira16200(), device=-1)            # two classes
    huge = L.Code.from_parity_check(W.code_c2_ira64800(), device=-1)
    w = torch.zeros((4, 1, 2), dtype=torch.float32)                           # host stand-in: planning only

    def status(code, **kw):
        try:
            code.workspace_size(8, L.make_params(**kw))
            return L.LDPC_OK
        except L.LdpcError as e:
            return e.status

    # widths: 0/6 default, 7 and 8 for INT8 single-scan on the LDS/HBM kernel
    for bits in (0, 6, 7, 8):
        assert status(small, msg="int8", msg_bits=bits) == L.LDPC_OK
        assert status(big, msg="int8", msg_bits=bits, layout="hbm") == L.LDPC_OK
    for bits in (5, 9, -1):
        assert status(small, msg="int8", msg_bits=bits) == L.LDPC_EINVAL
    for kw in (dict(msg="1bit", msg_bits=7), dict(msg="int8", sched="two_scan", msg_bits=7),
               dict(msg="fp32", msg_bits=8), dict(msg="int8", msg_bits=8, layout="reg1"),
               dict(msg="int8", msg_bits=7, layout="frames")):
        assert status(big, **kw) == L.LDPC_EUNSUPPORTED, kw
    # the packed register kernel takes 7-8 bits where the accumulator has one
    # field per word (the 16200-bit code), not with three 10-bit fields (64800)
    for bits in (7, 8):
        assert status(big, msg="int8", msg_bits=bits, layout="reg") == L.LDPC_OK
        assert status(huge, msg="int8", msg_bits=bits, layout="reg") == L.LDPC_EUNSUPPORTED
        assert big.plan(64, L.make_params(msg="int8", msg_bits=bits))["kernel"] == "packed"
        assert small.plan(64, L.make_params(msg="int8", msg_bits=bits))["kernel"] == "packed"
    # 8-bit messages keep Z_old as int16: two bytes per variable on chip
    lds6 = big.plan(64, L.make_params(msg="int8"))["lds_bytes"]
    lds7 = big.plan(64, L.make_params(msg="int8", msg_bits=7))["lds_bytes"]
    lds8 = big.plan(64, L.make_params(msg="int8", msg_bits=8))["lds_bytes"]
    assert lds6 == lds7 and lds8 - lds6 >= W.code_ira16200().N
    # wider messages widen the posterior accumulator (|Z| <= Q (d_v + 1)): for
    # the 64800-bit code (d_v = 8) 7 bits need 16-bit fields, which with Z_old
    # no longer fit in LDS
    assert status(huge, msg="int8", msg_bits=6, layout="hbm") == L.LDPC_OK
    for bits in (7, 8):
        assert status(huge, msg="int8", msg_bits=bits) == L.LDPC_EUNSUPPORTED
    # the 16200-bit code's messages still fit on chip at 7 bits in the LDS kernel
    assert big.workspace_size(4, L.make_params(msg="int8", msg_bits=7)) == \
        big.workspace_size(4, L.make_params(msg="int8", msg_bits=7, layout="lds")) == 0
    # schedules: one pair per iteration on every single-scan path; per-class
    # pairs on fixed point only when the code has a single class
    for msg in ("int8", "1bit"):
        for lay in ("auto", "reg", "reg1", "lds", "hbm"):
            st = status(big, msg=msg, layout=lay, weights=w, weight_classes=1)
            assert st in (L.LDPC_OK, L.LDPC_EUNSUPPORTED)  # LDS may not fit the big code
            assert status(big, msg=msg, layout=lay, weights=w, weight_classes=1) == \
                status(big, msg=msg, layout=lay)
        assert status(small, msg=msg, weights=w, weight_classes=0) == L.LDPC_OK
        assert status(irr, msg=msg, weights=w, weight_classes=0) == L.LDPC_EUNSUPPORTED
        assert status(irr, msg=msg, weights=w, weight_classes=1) == L.LDPC_OK
    assert status(irr, msg="fp32", weights=w, weight_classes=0) == L.LDPC_OK
    assert status(irr, msg="fp32", weights=w, weight_classes=1) == L.LDPC_OK
    assert status(small, msg="int8", weights=w, weight_classes=2) == L.LDPC_EINVAL
    assert status(small, msg="int8", sched="two_scan", weights=w, weight_classes=1) == L.LDPC_EUNSUPPORTED
    # the width changes only the on-chip posterior copy: HBM message bytes stay one per edge
    assert big.workspace_size(1, L.make_params(msg="int8", msg_bits=8, layout="hbm")) == \
        big.workspace_size(1, L.make_params(msg="int8", layout="hbm"))
    for c in (small, irr, big, huge):
        c.close()


# ---------------------------------------------------------------------------
# ldpc_decode_plan: the plan of a call, on host-only handles
PLAN_CASES = [("int8", "single_scan"), ("1bit", "single_scan"), ("fp32", "single_scan"),
              ("int8", "two_scan"), ("fp32", "two_scan")]


@pytest.mark.parametrize("name", ["peg1008", "qc7493", "ira16200", "ira64800"])
def test_decode_plan_matches_workspace_and_forced_layout(L, name):
    code = {"peg1008": W.code_c0_peg1008, "qc7493": W.code_c1_qc7493, "ira16200": W.code_ira16200,
            "ira64800": W.code_c2_ira64800}[name]()
    c = L.Code.from_parity_check(code, device=-1)
    seen = set()
    for msg, sched in PLAN_CASES:
        for F in (1, 100, 256, 300, 512):
            for flags in (0, L.F_CHECK_INPUT):
                p = L.make_params(msg=msg, sched=sched, max_iter=20)
                p.flags |= flags
                pl = c.plan(F, p)
                assert pl["workspace_bytes"] == c.workspace_size(F, p)
                seen.add(pl["kernel"])
                # forcing the reported layout gives the same plan
                pf = L.make_params(msg=msg, sched=sched, max_iter=20, layout=pl["layout"])
                pf.flags |= flags
                assert c.plan(F, pf) == pl, (msg, sched, F, pl)
                frames = pl["kernel"] in ("f32_frames", "two_scan_frames")
                assert (pl["frames_per_lane"] > 0) == frames
                assert pl["threads"] % 64 == 0 and 0 < pl["threads"] <= 1024
                if frames:
                    assert pl["lds_bytes"] == 0 and pl["threads"] == 256
                else:
                    assert 0 < pl["lds_bytes"] <= c.info()["lds_bytes_per_cu"]
                if frames:
                    # four frames per lane from 256 frames, rows of at most 16 entries
                    wide = c.info()["max_row_deg"] > 16
                    assert pl["frames_per_lane"] == (4 if F >= 256 and not wide else 1)
                if pl["kernel"] == "packed":
                    assert pl["threads"] == c.info()["pk_threads"]
    c.close()
    expect = {"peg1008": {"packed", "generic_f32", "two_scan"},
              "qc7493": {"packed", "f32_frames", "two_scan", "two_scan_frames"},
              "ira16200": {"packed", "f32_frames", "two_scan", "two_scan_frames"},
              "ira64800": {"packed", "f32_frames", "two_scan_frames"}}[name]
    assert seen == expect


def test_decode_plan_wide_rows_one_frame_per_lane(L):
    """Rows above 16 entries: binary32 frames across lanes keeps one frame per
    lane at any batch size."""
    p = L.make_params(msg="fp32", layout="frames", max_iter=10)
    code = W.random_small_code(60, 200, (17, 21), seed=17)
    c = L.Code.from_parity_check(code, device=-1)
    assert c.plan(300, p)["frames_per_lane"] == 1
    code2 = W.random_small_code(60, 200, (13, 16), seed=13)
    c2 = L.Code.from_parity_check(code2, device=-1)
    assert c2.plan(300, p)["frames_per_lane"] == 4 and c2.plan(255, p)["frames_per_lane"] == 1
    c.close()
    c2.close()


def test_decode_plan_errors(L):
    c = L.Code.from_parity_check(W.code_c0_peg1008(), device=-1)
    p = L.make_params(msg="int8")
    lib = L.lib()
    assert lib.ldpc_decode_plan(c._h, 10, ctypes.byref(p), None) == 1  # LDPC_EINVAL
    out = L.PlanInfo()
    assert lib.ldpc_decode_plan(None, 10, ctypes.byref(p), ctypes.byref(out)) == 1
    assert lib.ldpc_decode_plan(c._h, -1, ctypes.byref(p), ctypes.byref(out)) == 1
    assert lib.ldpc_decode_plan(c._h, 10, None, ctypes.byref(out)) == 1
    bad = L.make_params(msg="1bit", sched="two_scan")
    assert lib.ldpc_decode_plan(c._h, 10, ctypes.byref(bad), ctypes.byref(out)) == 5  # LDPC_EUNSUPPORTED
    fr = L.make_params(msg="int8", layout="frames")  # frames-across-lanes single-scan is FP32 only
    with pytest.raises(L.LdpcError):
        c.plan(10, fr)
    c.close()


# ---------------------------------------------------------------------------
# ldpc_code_query: degree histograms, block structure and per-frame storage.
def _qc_from_base(base, Z):
    """H from a base matrix of shifts (-1: empty block), Z x Z circulants."""
    mb, nb = base.shape
    rows = [[] for _ in range(mb * Z)]
    for i in range(mb):
        for j in range(nb):
            s = base[i, j]
            if s >= 0:
                for r in range(Z):
                    rows[i * Z + r].append(j * Z + (r + s) % Z)
    return W.ParityCheck.from_rows(mb * Z, nb * Z, rows, "qc_small")


@pytest.mark.parametrize("name", ["peg1008", "qc7493", "ira16200", "ira64800"])
def test_query_histograms_and_storage(L, name):
    """Histograms add up to M, N and E; single-scan keeps N stored
    variable-side values where two-scan keeps N x mean column degree = E
    (Sec. IV); addressing is halved; messages are b E bits with b <= 8 in
    one byte, and the 1-bit form E sign bits plus a few bits per check
    (Sec. V); the streaming traffic model follows from those sizes."""
    code = {"peg1008": W.code_c0_peg1008, "qc7493": W.code_c1_qc7493, "ira16200": W.code_ira16200,
            "ira64800": W.code_c2_ira64800}[name]()
    i = L.Code.from_parity_check(code, device=-1).info()
    M, N, E = code.M, code.N, code.E
    rh, ch = np.array(i["row_deg_hist"]), np.array(i["col_deg_hist"])
    np.testing.assert_array_equal(rh, np.bincount(code.row_degrees(), minlength=65))
    np.testing.assert_array_equal(ch, np.bincount(code.col_degrees(), minlength=65))
    assert rh.sum() == M and ch.sum() == N
    assert (rh * np.arange(65)).sum() == E and (ch * np.arange(65)).sum() == E
    assert i["var_values_single"] == N
    assert i["var_values_two"] == E
    assert i["var_values_two"] == pytest.approx(N * code.col_degrees().mean())
    assert i["addr_bytes_two"] == 2 * i["addr_bytes_single"] == 8 * E
    assert i["msg_bytes_int8"] * 8 == i["msg_bits_int8"] == 8 * E
    assert i["msg_bytes_fp32"] == 4 * E and i["post_bytes_fp32"] == 4 * N and i["post_bytes_int"] == 2 * N
    lg = int(np.ceil(np.log2(code.row_degrees().max())))
    assert i["msg_bits_1bit"] == E + M * (5 + 5 + lg)
    assert i["msg_bytes_1bit"] == (E + 7) // 8 + 2 * M
    assert 8 * i["msg_bytes_1bit"] >= i["msg_bits_1bit"]  # the stored form holds the Sec. V state
    assert i["stream_bytes_int8"] == 2 * E + 5 * N
    assert i["stream_bytes_1bit"] == 2 * ((E + 7) // 8) + 4 * M + 5 * N
    assert i["stream_bytes_fp32"] == 8 * E + 12 * N
    assert i["stream_bytes_two_int8"] == 4 * E + 3 * N
    assert i["stream_bytes_two_fp32"] == 16 * E + 8 * N
    want = {"peg1008": (set(), 0, 0), "qc7493": ({"qc"}, 127, 0), "ira16200": ({"ira", "ira_groups"}, 0, 180),
            "ira64800": ({"ira", "ira_groups"}, 0, 360)}[name]
    assert (i["structure"], i["qc_lift"], i["ira_group"]) == want


def test_query_structure_detection(L):
    rng = np.random.default_rng(3)
    base = rng.integers(-1, 13, size=(4, 9))
    base[:, 0] = rng.integers(0, 13, size=4)  # no empty block column
    code = _qc_from_base(base, 13)
    i = L.Code.from_parity_check(code, device=-1).info()
    assert i["structure"] == {"qc"} and i["qc_lift"] == 13
    # one entry moved inside its block breaks the circulant: no QC lift of 13
    rows = [list(code.col_idx[code.row_ptr[m]:code.row_ptr[m + 1]]) for m in range(code.M)]
    c0 = rows[0][0]
    alt = (c0 // 13) * 13 + (c0 % 13 + 1) % 13
    if alt not in rows[0]:
        rows[0][0] = alt
        broken = W.ParityCheck.from_rows(code.M, code.N, rows, "qc_broken")
        assert L.Code.from_parity_check(broken, device=-1).info()["qc_lift"] != 13
    # columns permuted at random: no structure left
    perm = rng.permutation(code.N)
    shuffled = W.ParityCheck.from_rows(code.M, code.N, [perm[r] for r in rows], "qc_shuffled")
    assert L.Code.from_parity_check(shuffled, device=-1).info()["structure"] == set()
    # a small repeat-accumulate code: staircase and 36-column groups
    ira = W.ira_code(720, 360, 36, {5: 5, 3: 5}, seed=11, name="ira720")
    i = L.Code.from_parity_check(ira, device=-1).info()
    assert i["structure"] == {"ira", "ira_groups"} and i["ira_group"] == 36
    # swap two staircase columns: neither bit
    rows = [list(ira.col_idx[ira.row_ptr[m]:ira.row_ptr[m + 1]]) for m in range(ira.M)]
    a, b = ira.N - ira.M + 5, ira.N - ira.M + 9
    sw = W.ParityCheck.from_rows(ira.M, ira.N, [[b if c == a else a if c == b else c for c in r] for r in rows],
                                 "ira_swapped")
    assert L.Code.from_parity_check(sw, device=-1).info()["structure"] == set()


def test_binding_rejects_host_tensors(L):
    """Buffers on the wrong device are refused before the library is called."""
    import torch
    code = W.code_c0_peg1008()
    gc = L.Code.from_parity_check(code, device=-1)
    x = torch.zeros((2, code.N), dtype=torch.int8)
    o = {"hard": torch.zeros((2, code.N), dtype=torch.uint8), "llr": None,
         "iters": torch.zeros(2, dtype=torch.int32), "ok": torch.zeros(2, dtype=torch.uint8)}
    with pytest.raises(ValueError):
        gc.decode_into(x, L.make_params(msg="int8"), o["hard"], o["llr"], o["iters"], o["ok"], None)
    with pytest.raises(ValueError):
        gc.decode(x, msg="int8")
    for w in (torch.zeros((3, 1, 2), dtype=torch.float64), torch.zeros((3, 1, 3)), torch.zeros((0, 1, 2))):
        with pytest.raises(ValueError):
            L.make_params(msg="fp32", weights=w)
    p = L.make_params(msg="fp32", weights=torch.zeros((3, 1, 2)), weight_classes=1)  # planning only
    assert gc.workspace_size(300, p) > 0
    with pytest.raises(ValueError):  # a host table cannot be decoded with
        gc.decode_into(x.float(), p, o["hard"], o["llr"], o["iters"], o["ok"], None)


def test_noalloc_entry_point_checks(L):
    """ldpc_decode_batch_noalloc validates like ldpc_decode_batch, refuses a
    call whose workspace exceeds its static scratch (before any device work)
    and, like every decode, refuses host-only handles."""
    lib = L.lib()
    big = L.Code.from_parity_check(W.code_c2_ira64800(), device=-1)
    small = L.Code.from_parity_check(W.code_c0_peg1008(), device=-1)
    fp = L.make_params(max_iter=10, msg="fp32")
    assert big.workspace_size(256, fp) > L.NOALLOC_SCRATCH_BYTES
    st = lib.ldpc_decode_batch_noalloc(big._h, 256, None, ctypes.byref(fp), None, None, None, None, None)
    assert st == L.LDPC_EUNSUPPORTED and b"static scratch" in lib.ldpc_last_error()
    hbm = L.make_params(max_iter=10, msg="int8", layout="hbm")
    assert 0 < small.workspace_size(200, hbm) <= L.NOALLOC_SCRATCH_BYTES
    st = lib.ldpc_decode_batch_noalloc(small._h, 200, None, ctypes.byref(hbm), None, None, None, None, None)
    assert st == L.LDPC_EINVAL and b"host-only" in lib.ldpc_last_error()
    bad = L.make_params(max_iter=-1, msg="int8")
    assert lib.ldpc_decode_batch_noalloc(small._h, 4, None, ctypes.byref(bad), None, None, None, None,
                                         None) == L.LDPC_EINVAL
    assert lib.ldpc_decode_batch_noalloc(None, 4, None, ctypes.byref(hbm), None, None, None, None,
                                         None) == L.LDPC_EINVAL


def test_persistent_multi_host_checks(L):
    """ldpc_multi_persistent_workspace_size is the 256-byte counter for valid
    jobs and fails like ldpc_multi_workspace_size on invalid ones; a call
    without a workspace is refused before anything else."""
    codes = [W.code_c0_peg1008(), W.code_c1_qc7493(), W.code_ira16200()]
    hs = [_host_code(L, c) for c in codes]
    p = L.make_params(msg="int8")
    jobs = (L.Job * 3)()
    for k, h in enumerate(hs):
        jobs[k] = _job(L, h, 100, p)
    got = ctypes.c_size_t()
    assert L.lib().ldpc_multi_persistent_workspace_size(jobs, 3, ctypes.byref(got)) == L.LDPC_OK
    assert got.value == 256
    bad = L.make_params(msg="int8", max_iter=-1)
    jobs[1] = _job(L, hs[1], 100, bad)
    assert L.lib().ldpc_multi_persistent_workspace_size(jobs, 3, ctypes.byref(got)) == L.LDPC_EINVAL
    assert b"job 1" in L.lib().ldpc_last_error()
    jobs[1] = _job(L, hs[1], 100, p)
    assert L.lib().ldpc_decode_multi_persistent(jobs, 3, None, 0, None) == L.LDPC_EINVAL
    for h in hs:
        L.lib().ldpc_code_destroy(h)


@pytest.mark.parametrize("name,expect", [
    ("peg1008", [(6, 2, 256), (6, 2, 1024)]),      # 256 threads (several frames per CU) or 1024
    ("qc7493", [(11, 12, 512), (21, 4, 768)]),     # rows over a lane pair (two frames per CU) or one lane
    ("ira16200", [(7, 8, 1024)]),
    ("ira64800", [(7, 32, 1024)]),
])
def test_packed_shape_candidates(L, name, expect):
    """The packed shapes autotuning times: the handle's own first, one per
    (threads, lanes per row), each covering every row and every slot of the
    longest row; host-only handles list them but cannot install one."""
    code = {"peg1008": W.code_c0_peg1008, "qc7493": W.code_c1_qc7493, "ira16200": W.code_ira16200,
            "ira64800": W.code_c2_ira64800}[name]()
    gc = L.Code.from_parity_check(code, device=-1)
    info = gc.info()
    shapes = gc.packed_shapes()
    assert shapes == expect
    assert shapes[0] == (info["pk_slots"], info["pk_rows_per_thread"], info["pk_threads"])
    D, M = int(code.row_degrees().max()), code.M
    pairs = set()
    for d, r, t in shapes:
        lanes = 2 if d < D else 1
        assert d * lanes >= D and r * (t // lanes) >= M
        pairs.add((t, lanes))
    assert len(pairs) == len(shapes)
    # a short buffer gets the first triples only; the count is the full one
    lib = L.lib()
    buf, n = (ctypes.c_int32 * 3)(), ctypes.c_int32()
    assert lib.ldpc_code_packed_shapes(gc._h, buf, 1, ctypes.byref(n)) == L.LDPC_OK
    assert n.value == len(shapes) and tuple(buf) == shapes[0]
    assert lib.ldpc_code_packed_shapes(gc._h, None, 1, ctypes.byref(n)) == L.LDPC_EINVAL
    assert lib.ldpc_code_packed_shapes(None, None, 0, ctypes.byref(n)) == L.LDPC_EINVAL
    assert lib.ldpc_code_set_packed_shape(gc._h, *shapes[-1]) == L.LDPC_EINVAL
    assert b"host-only" in lib.ldpc_last_error()
    gc.close()
