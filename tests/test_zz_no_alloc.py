"""GPU test of ldpc_decode_batch_noalloc, the entry point for callers that
cannot allocate: the same decode as ldpc_decode_batch with the workspace
taken from the library's static per-device scratch.  Each case runs two
calls in a row, the second with fewer frames (the scratch keeps the first
call's contents), and compares every output with ldpc_decode_batch given a
freshly allocated workspace, bit for bit, on the same inputs.
"""
import numpy as np
import pytest

from paper_cs_0609090_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


@pytest.fixture(scope="module")
def L(torch_dev):
    from paper_cs_0609090_amd import ldpc
    ldpc.lib()
    return ldpc


def _with_workspace(torch, L, gc, x, p):
    out = gc.alloc_outputs(x.shape[0], x.device, True)
    ws = gc.alloc_workspace(x.shape[0], p, x.device)
    gc.decode_into(x, p, out["hard"], out["llr"], out["iters"], out["ok"], ws)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _noalloc(torch, L, gc, x, p):
    out = gc.alloc_outputs(x.shape[0], x.device, True)
    gc.decode_noalloc_into(x, p, out["hard"], out["llr"], out["iters"], out["ok"])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


# (code, message type, schedule, layout, Eb/N0, first and second frame count):
# kernels whose state lives in the workspace -- binary32 frames across lanes,
# the generic fixed-point kernel with messages in device memory, and the
# two-scan baseline across lanes
CASES = [
    ("code_c1_qc7493", "fp32", "single_scan", "auto", 3.25, 256, 37),
    ("code_c0_peg1008", "int8", "single_scan", "hbm", 2.0, 200, 51),
    ("code_ira16200", "int8", "two_scan", "frames", 1.3, 64, 5),
    ("code_c0_peg1008", "1bit", "single_scan", "hbm", 1.5, 300, 1),
]


@pytest.mark.parametrize("ctor,msg,sched,layout,ebn0,f1,f2", CASES)
def test_noalloc_matches_decode_batch(torch_dev, L, ctor, msg, sched, layout, ebn0, f1, f2):
    torch = torch_dev
    code = getattr(W, ctor)()
    print(f"[noalloc] {ctor} {msg} {sched} {layout} frames {f1} then {f2}", flush=True)
    gc = L.Code.from_parity_check(code)
    for i, F in enumerate((f1, f2)):
        llr = W.awgn_llr(code.N, F, ebn0, code.design_rate, key=(0xA110C, i))
        host = llr if msg == "fp32" else W.quantize_llr(llr)
        x = torch.from_numpy(host).to("cuda")
        for early in (True, False):
            p = L.make_params(max_iter=30, alpha=0.8, early_stop=early, msg=msg, sched=sched, layout=layout)
            need = gc.workspace_size(F, p)
            assert 0 < need <= L.NOALLOC_SCRATCH_BYTES
            ref = _with_workspace(torch, L, gc, x, p)
            got = _noalloc(torch, L, gc, x, p)
            for k in ("hard", "llr", "iters", "ok"):
                np.testing.assert_array_equal(got[k], ref[k], err_msg=f"{k}, call {i + 1}, early_stop={early}")
    gc.close()


def test_noalloc_rejects_oversized_call(torch_dev, L):
    torch = torch_dev
    code = W.code_c2_ira64800()
    gc = L.Code.from_parity_check(code)
    F = 256
    p = L.make_params(max_iter=5, msg="fp32")
    assert gc.workspace_size(F, p) > L.NOALLOC_SCRATCH_BYTES
    x = torch.zeros((F, code.N), dtype=torch.float32, device="cuda")
    out = gc.alloc_outputs(F, x.device, True)
    with pytest.raises(L.LdpcError) as ei:
        gc.decode_noalloc_into(x, p, out["hard"], out["llr"], out["iters"], out["ok"])
    assert ei.value.status == L.LDPC_EUNSUPPORTED
    # the same handle still decodes a call that fits, and no workspace is
    # needed for the register kernel at all
    q = L.make_params(max_iter=5, msg="int8")
    xi = torch.zeros((4, code.N), dtype=torch.int8, device="cuda")
    o2 = gc.alloc_outputs(4, xi.device, True)
    gc.decode_noalloc_into(xi, q, o2["hard"], o2["llr"], o2["iters"], o2["ok"])
    torch.cuda.synchronize()
    assert (o2["hard"].cpu().numpy() == 1).all()  # Z = 0 decides 1
    gc.close()
