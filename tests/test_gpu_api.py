"""GPU tests of the binding's argument checks, autotuning across message
widths, offsets past every magnitude, and the two-fields-per-word posterior
accumulator of the register kernels, each against the CPU oracle where a
decode runs.
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


def _np(out):
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


# ---------------------------------------------------------------------------
# Argument checks in the binding: a wrong shape, dtype or device raises
# ValueError before the library is called (the kernels index buffers by the
# code's N and class count).
def test_binding_rejects_mismatched_buffers(torch_dev, L):
    torch = torch_dev
    code = W.random_small_code(12, 30, (3, 7), seed=909)
    gc = L.Code.from_parity_check(code)
    C = gc.n_classes
    assert C >= 2
    good = torch.zeros((4, code.N), dtype=torch.int8, device="cuda")
    with pytest.raises(ValueError):  # N too small
        gc.decode(torch.zeros((4, code.N - 1), dtype=torch.int8, device="cuda"), msg="int8")
    with pytest.raises(ValueError):  # host tensor
        gc.decode(torch.zeros((4, code.N), dtype=torch.int8), msg="int8")
    with pytest.raises(ValueError):  # dtype of the message type
        gc.decode(torch.zeros((4, code.N), dtype=torch.float32, device="cuda"), msg="int8")
    with pytest.raises(ValueError):  # 1-D input
        gc.decode(torch.zeros((4 * code.N,), dtype=torch.int8, device="cuda"), msg="int8")
    xf = torch.zeros((4, code.N), dtype=torch.float32, device="cuda")
    for bad_w, wc in ((torch.zeros((3, C + 1, 2), device="cuda"), 0),
                      (torch.zeros((3, C, 2), device="cuda"), 1),
                      (torch.zeros((3, C, 2), dtype=torch.float64, device="cuda"), 0),
                      (torch.zeros((3, C, 3), device="cuda"), 0),
                      (torch.zeros((3, C, 2)), 0)):
        with pytest.raises(ValueError):
            gc.decode(xf, msg="fp32", weights=bad_w, weight_classes=wc)
    p = L.make_params(msg="int8")
    o = gc.alloc_outputs(4, good.device)
    for key, bad in (("hard", torch.zeros((4, code.N - 1), dtype=torch.uint8, device="cuda")),
                     ("llr", torch.zeros((4, code.N), dtype=torch.float64, device="cuda")),
                     ("iters", torch.zeros((3,), dtype=torch.int32, device="cuda")),
                     ("ok", torch.zeros((4,), dtype=torch.int32, device="cuda"))):
        oo = dict(o)
        oo[key] = bad
        with pytest.raises(ValueError):
            gc.decode_into(good, p, oo["hard"], oo["llr"], oo["iters"], oo["ok"], None)
    with pytest.raises(ValueError):  # a weights pointer set by hand cannot be checked
        pw = L.make_params(msg="int8")
        pw.weights = xf.data_ptr()
        pw.weight_iters = 1
        gc.decode_into(good, pw, o["hard"], o["llr"], o["iters"], o["ok"], None)
    # learned forward: N and the class count
    ws = torch.empty(gc.learn_workspace_size(4, 3, 1), dtype=torch.uint8, device="cuda")
    w = torch.zeros((3, C, 2), device="cuda")
    with pytest.raises(ValueError):
        gc.learn_forward(torch.zeros((4, code.N + 1), device="cuda"), None, w, 1, ws)
    with pytest.raises(ValueError):
        gc.learn_forward(xf, None, torch.zeros((3, C - 1, 2), device="cuda"), 1, ws)
    with pytest.raises(ValueError):
        gc.learn_forward(xf, torch.zeros((4, code.N), dtype=torch.int8, device="cuda"), w, 1, ws)
    # mixed batches check every job
    with pytest.raises(ValueError):
        L.MultiBatch([(gc, torch.zeros((2, code.N + 3), dtype=torch.int8, device="cuda"), p)])
    # nothing above reached a kernel: a correct call still works
    out = gc.decode(good, msg="int8", max_iter=3)
    torch.cuda.synchronize()
    assert out["hard"].shape == (4, code.N)
    gc.close()


def test_explicit_stream(torch_dev, L, orc):
    """decode(stream=s) on a side stream: the input, written on the current
    stream just before, is seen complete; results equal the oracle."""
    torch = torch_dev
    code = W.code_c0_peg1008()
    x = W.quantize_llr(W.awgn_llr(code.N, 64, 2.0, code.design_rate, key=(0x57E, 1)))
    gc = L.Code.from_parity_check(code)
    s = torch.cuda.Stream()
    src = torch.from_numpy(x).cuda()
    for _ in range(3):
        t = torch.zeros_like(src)
        t.copy_(src)                       # on the current stream
        tt = t.t().contiguous().t()        # a non-contiguous view: decode makes its own copy
        out = gc.decode(tt, msg="int8", max_iter=20, stream=s)
        s.synchronize()
        r = orc.decode(code, x, algo="single_scan", arith="int", max_iter=20, alpha=0.8)
        g = _np(out)
        np.testing.assert_array_equal(g["hard"], r["hard"])
        np.testing.assert_array_equal(g["iters"], r["iters"])
        np.testing.assert_array_equal(g["llr"], r["post"])
    gc.close()


# ---------------------------------------------------------------------------
# Autotuning keyed by message width: a layout tuned for 6-bit messages does not
# leak into 7- or 8-bit calls (which the one-row register kernel cannot run:
# they keep the built-in choice, the packed kernel on this code), and a 7-bit
# tune does not move 6-bit calls off their own choice.
def test_autotune_then_other_width(torch_dev, L, orc):
    torch = torch_dev
    code = W.code_ira16200()
    gc = L.Code.from_parity_check(code)
    F = 8
    llr = W.awgn_llr(code.N, F, 1.3, code.design_rate, key=(0xA7, 1))
    p6 = L.make_params(msg="int8", max_iter=12)
    before6 = gc.plan(F, p6)
    t6 = gc.autotune(F, p6)
    assert t6["tried"] >= 3
    assert gc.plan(F, p6)["layout"] == t6["layout"]
    for bits, step in ((7, 0.25), (8, 0.125)):
        q = W.quantize_llr(llr, step=step, qmax=(1 << (bits - 1)) - 1)
        pb = L.make_params(msg="int8", max_iter=12, msg_bits=bits, llr_step=step)
        assert gc.plan(F, pb)["kernel"] == "packed"
        g = _np(gc.decode(torch.from_numpy(q).cuda(), msg="int8", max_iter=12, msg_bits=bits, llr_step=step,
                          early_stop=True))
        r = orc.decode(code, q, algo="single_scan", arith="int", max_iter=12, qbits=bits, step=step,
                       early_stop=True)
        for k in ("hard", "iters", "ok"):
            np.testing.assert_array_equal(g[k], r[k], err_msg=f"{k} {bits} bits")
        np.testing.assert_array_equal(g["llr"], r["post"], err_msg=f"llr {bits} bits")
    # a 7-bit tune: 6-bit AUTO keeps the 6-bit tuned layout
    p7 = L.make_params(msg="int8", max_iter=12, msg_bits=7, llr_step=0.25)
    t7 = gc.autotune(F, p7)
    assert t7["layout"] in ("reg", "lds", "hbm")
    assert gc.plan(F, p6)["layout"] == t6["layout"]
    assert before6["kernel"] in ("packed", "reg1")
    q6 = W.quantize_llr(llr)
    g = _np(gc.decode(torch.from_numpy(q6).cuda(), msg="int8", max_iter=12))
    r = orc.decode(code, q6, algo="single_scan", arith="int", max_iter=12)
    np.testing.assert_array_equal(g["llr"], r["post"])
    np.testing.assert_array_equal(g["iters"], r["iters"])
    gc.close()


# ---------------------------------------------------------------------------
# Offsets past every magnitude zero every message (Sec. III OMS), including
# offsets whose step count does not fit 32 bits: posteriors stay at Z(0).
@pytest.mark.parametrize("beta", [1e6, 1e12, 3.0e38])
def test_huge_offset_zeroes_messages(torch_dev, L, orc, beta):
    torch = torch_dev
    code = W.code_c0_peg1008()
    llr = W.awgn_llr(code.N, 16, 1.5, code.design_rate, key=(0xB7A, 2))
    q = W.quantize_llr(llr)
    gc = L.Code.from_parity_check(code)
    cases = [("int8", "single_scan", lay, q) for lay in ("auto", "reg1", "lds", "hbm")] + \
            [("1bit", "single_scan", lay, q) for lay in ("auto", "reg1", "lds")] + \
            [("int8", "two_scan", "auto", q), ("int8", "two_scan", "frames", q),
             ("fp32", "single_scan", "auto", llr), ("fp32", "single_scan", "frames", llr),
             ("fp32", "two_scan", "frames", llr)]
    for msg, sched, lay, x in cases:
        g = _np(gc.decode(torch.from_numpy(x).cuda(), msg=msg, sched=sched, layout=lay, max_iter=6,
                          beta=beta, early_stop=False))
        z0 = x.astype(np.float32) * (np.float32(0.5) if msg != "fp32" else np.float32(1.0))
        np.testing.assert_array_equal(g["llr"], z0, err_msg=f"{msg} {sched} {lay}")
        np.testing.assert_array_equal(g["hard"], (z0 <= 0).astype(np.uint8))
    # per-iteration schedule: the huge offset from iteration 2 on freezes Z^(1)
    sched = torch.tensor([[[0.8, 0.0]], [[0.8, beta]]], dtype=torch.float32, device="cuda")
    for msg in ("int8", "1bit"):
        g = _np(gc.decode(torch.from_numpy(q).cuda(), msg=msg, max_iter=5, weights=sched, weight_classes=1,
                          early_stop=False))
        algo = "one_bit" if msg == "1bit" else "single_scan"
        r = orc.decode(code, q, algo=algo, arith="int", max_iter=5, sched=[[0.8, 0.0], [0.8, beta]],
                       early_stop=False)
        np.testing.assert_array_equal(g["llr"], r["post"])
    gc.close()


# ---------------------------------------------------------------------------
# Two 16-bit posterior fields per LDS word (bias 32768, signed-delta atomics):
# the register kernels take this packing for codes whose posteriors fit LDS
# only at two fields per word.  A rate-2/3 IRA code (N = 43200, M = 14400,
# check degree 8, column degrees 3 and 2) is one.
def _ira43200():
    return W.ira_code(43200, 28800, 360, {3: 80}, seed=0x2F2, name="ira43200_r23")


@pytest.mark.parametrize("layout", ["reg", "reg1"])
@pytest.mark.parametrize("msg", ["int8", "1bit"])
def test_two_fields_per_word_accumulator(torch_dev, L, orc, msg, layout):
    torch = torch_dev
    code = _ira43200()
    gc = L.Code.from_parity_check(code)
    info = gc.info()
    assert info["reg_zpack"] == 2
    assert gc.plan(24, L.make_params(msg=msg, layout=layout))["kernel"] == ("packed" if layout == "reg" else "reg1")
    eb = np.linspace(1.5, 4.0, 24)
    for step, alpha, es in ((0.5, 0.8, False), (0.125, 1.0, False), (0.5, 0.8, True)):
        q = W.quantize_llr(W.awgn_llr(code.N, 24, eb, code.design_rate, key=(0x2F2, int(8 * step))), step=step)
        for with_llr in (True, False):
            g = _np(gc.decode(torch.from_numpy(q).cuda(), msg=msg, layout=layout, max_iter=25, alpha=alpha,
                              early_stop=es, llr_step=step, with_llr=with_llr))
            algo = "one_bit" if msg == "1bit" else "single_scan"
            r = orc.decode(code, q, algo=algo, arith="int", max_iter=25, alpha=alpha, early_stop=es, step=step)
            for k in ("hard", "iters", "ok"):
                np.testing.assert_array_equal(g[k], r[k], err_msg=f"{k} step {step} es {es}")
            if with_llr:
                np.testing.assert_array_equal(g["llr"], r["post"])
        if es:
            assert len(set(r["iters"].tolist())) > 2
    gc.close()


# ---------------------------------------------------------------------------
# Device allocation failures (injected from the host: LDPC_FAIL_ALLOC=k fails
# the k-th device allocation of an entry point) are reported as LDPC_ENOMEM,
# leave no half-built state behind, and the same call succeeds afterwards.
def test_injected_allocation_failures(torch_dev, L, orc, monkeypatch):
    torch = torch_dev
    code = W.code_c0_peg1008()
    free0 = torch.cuda.mem_get_info()[0]
    first_ok = None
    for k in range(1, 25):
        monkeypatch.setenv("LDPC_FAIL_ALLOC", str(k))
        try:
            gc = L.Code.from_parity_check(code)
        except L.LdpcError as e:
            assert e.status == L.LDPC_ENOMEM, (k, str(e))
            continue
        gc.close()
        first_ok = k
        break
    assert first_ok is not None and first_ok >= 8  # the handle's device tables, each failed in turn
    monkeypatch.delenv("LDPC_FAIL_ALLOC")
    torch.cuda.synchronize()
    assert abs(torch.cuda.mem_get_info()[0] - free0) < (64 << 20)
    gc = L.Code.from_parity_check(code)
    q = W.quantize_llr(W.awgn_llr(code.N, 8, 2.0, code.design_rate, key=(0xFA, 1)))
    g = _np(gc.decode(torch.from_numpy(q).cuda(), msg="int8", max_iter=10))
    r = orc.decode(code, q, algo="single_scan", arith="int", max_iter=10)
    np.testing.assert_array_equal(g["llr"], r["post"])
    # the encoder's tables, built on first use: each allocation failed in turn
    for k in (1, 2):
        monkeypatch.setenv("LDPC_FAIL_ALLOC", str(k))
        with pytest.raises(L.LdpcError) as ei:
            gc.encoder_info()
        assert ei.value.status == L.LDPC_ENOMEM
    monkeypatch.delenv("LDPC_FAIL_ALLOC")
    K = gc.encoder_info()["K"]
    info = torch.randint(0, 2, (4, K), dtype=torch.uint8, device="cuda")
    cw = gc.encode(info).cpu().numpy()
    assert not code.syndrome(cw).any()
    # autotuning's trial buffers
    monkeypatch.setenv("LDPC_FAIL_ALLOC", "2")
    with pytest.raises(L.LdpcError):
        gc.autotune(16, L.make_params(msg="int8", max_iter=5))
    monkeypatch.delenv("LDPC_FAIL_ALLOC")
    assert gc.autotune(16, L.make_params(msg="int8", max_iter=5))["tried"] >= 2
    gc.close()


@pytest.mark.parametrize("msg,layout", [("int8", "auto"), ("1bit", "auto"), ("fp32", "frames")])
def test_noalloc_call_captured_in_a_graph(torch_dev, L, msg, layout):
    """The allocation-free call is meant for code under graph capture: one
    ldpc_decode_batch_noalloc captured into a HIP graph, replayed three times
    with new inputs copied in and eager work on the same stream between the
    replays, equals the eager call on the same inputs every time (the
    binary32 frames-across-lanes plan uses the library's static scratch)."""
    torch = torch_dev
    code = W.code_ira16200()
    F = 96
    gc = L.Code.from_parity_check(code)
    p = L.make_params(max_iter=15, msg=msg, layout=layout, early_stop=True)
    def inputs(seed):
        x = W.awgn_llr(code.N, F, 2.0 + 0.2 * seed, code.design_rate, key=(0x6A, seed))
        return torch.from_numpy(x if msg == "fp32" else W.quantize_llr(x)).cuda()
    xin = inputs(0)
    out = gc.alloc_outputs(F, xin.device)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # a first eager call before the capture
        gc.decode_noalloc_into(xin, p, out["hard"], out["llr"], out["iters"], out["ok"])
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gc.decode_noalloc_into(xin, p, out["hard"], out["llr"], out["iters"], out["ok"])
    for rep in range(3):
        x = inputs(rep + 1)
        xin.copy_(x)
        _ = (x.float() * 2).sum()  # eager work between the replays
        g.replay()
        torch.cuda.synchronize()
        got = {k: v.clone() for k, v in out.items() if v is not None}
        ref = gc.decode(x, max_iter=15, msg=msg, layout=layout, early_stop=True)
        torch.cuda.synchronize()
        for k in got:
            assert torch.equal(got[k], ref[k]), f"replay {rep} {k}"
    gc.close()
