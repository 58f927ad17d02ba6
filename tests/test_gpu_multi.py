"""Mixed batches and layout autotuning on the GPU (include/ldpc_multi.h).

A mixed call must give every job exactly what a separate ldpc_decode_batch
call gives (each frame's result depends only on its own input), and sampled
frames of every job must equal the oracle (bit-exact, as in the single-code
parity tests).  Inputs are host-generated (Philox normals, per-frame Eb/N0
uniform in [1, 3] dB), the same arrays for the GPU and the oracle.
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


ORACLE_VARIANT = {("int8", "single_scan"): ("single_scan", "int"), ("1bit", "single_scan"): ("one_bit", "int"),
                  ("fp32", "single_scan"): ("single_scan", "f32"), ("int8", "two_scan"): ("two_scan", "int"),
                  ("fp32", "two_scan"): ("two_scan", "f32")}


def _host_llr(code, F, msg, seed):
    eb = np.random.default_rng(seed).uniform(1.0, 3.0, size=F)
    x = W.awgn_llr(code.N, F, eb, code.design_rate, key=(0xC3, seed))
    return W.quantize_llr(x) if msg in ("int8", "1bit") else x


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(out):
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


def _check_jobs(torch, L, orc, spec, max_iter, early_stop, samples, with_llr=True, persistent=False):
    """spec: (code, frames, msg, sched, layout).  Runs the mixed call (or the
    persistent one-launch form), the separate calls and the oracle on
    sampled frames."""
    torch.cuda.synchronize()
    items, hosts, gcs = [], [], []
    for k, (code, F, msg, sched, layout) in enumerate(spec):
        x = _host_llr(code, F, msg, 100 + k)
        gc = L.Code.from_parity_check(code)
        p = L.make_params(max_iter=max_iter, early_stop=early_stop, msg=msg, sched=sched, layout=layout)
        items.append((gc, _dev(torch, x), p))
        hosts.append(x)
        gcs.append(gc)
    mb = L.MultiBatch(items, with_llr=with_llr, persistent=persistent)
    print(f"[multi] persistent={persistent} jobs={[(c.name, F, m) for c, F, m, _, _ in spec]}", flush=True)
    mb.run()
    torch.cuda.synchronize()
    got = [_np(o) for o in mb.outputs]
    rng = np.random.default_rng(7)
    for k, ((code, F, msg, sched, layout), (gc, x, p), g) in enumerate(zip(spec, items, got)):
        where = f"job {k}: {code.name} F={F} {msg} {sched} {layout}"
        sep = _np(gc.decode(x, max_iter=max_iter, early_stop=early_stop, msg=msg, sched=sched, layout=layout,
                            with_llr=with_llr))
        for key in ("hard", "iters", "ok") + (("llr",) if with_llr else ()):
            np.testing.assert_array_equal(g[key], sep[key], err_msg=f"{key} {where}")
        if F == 0:
            continue
        sel = np.unique(np.concatenate([[0, F - 1], rng.integers(0, F, size=max(samples - 2, 0))]))
        algo, arith = ORACLE_VARIANT[(msg, sched)]
        kw = {"step": 0.5} if arith == "int" else {}
        r = orc.decode(code, hosts[k][sel], algo=algo, arith=arith, max_iter=max_iter, alpha=0.8,
                       early_stop=early_stop, **kw)
        np.testing.assert_array_equal(g["iters"][sel], r["iters"], err_msg=f"iters {where}")
        np.testing.assert_array_equal(g["ok"][sel], r["ok"], err_msg=f"ok {where}")
        np.testing.assert_array_equal(g["hard"][sel], r["hard"], err_msg=f"hard {where}")
        if with_llr:
            np.testing.assert_array_equal(g["llr"][sel], r["post"].astype(np.float32), err_msg=f"llr {where}")
    for gc in gcs:
        gc.close()
    return got


@pytest.mark.parametrize("early_stop", [True, False])
def test_mixed_codes_and_paths(torch_dev, L, orc, early_stop):
    """Five jobs over four codes and five kernel families in one call; a job
    of zero frames rides along."""
    small = W.random_small_code(40, 90, (3, 9), seed=31)
    spec = [(W.code_c0_peg1008(), 300, "int8", "single_scan", "auto"),
            (W.code_c1_qc7493(), 70, "1bit", "single_scan", "auto"),
            (W.code_ira16200(), 20, "int8", "single_scan", "reg"),
            (small, 0, "int8", "single_scan", "auto"),
            (small, 65, "fp32", "two_scan", "frames"),
            (W.code_c0_peg1008(), 130, "fp32", "single_scan", "frames")]
    got = _check_jobs(torch_dev, L, orc, spec, max_iter=30, early_stop=early_stop, samples=6)
    if early_stop:  # Eb/N0 spread: frames stop at different iterations
        assert len(set(got[0]["iters"].tolist())) > 3


def test_mixed_whole_cu_jobs_lead(torch_dev, L, orc):
    """Two jobs whose workgroups each take a whole CU's LDS (N=64800, int8
    and 1-bit): the larger-LDS one is launched first on the caller's stream,
    the other forked with the rest; every job equals its separate call and
    sampled frames the oracle."""
    ira = W.code_c2_ira64800()
    spec = [(W.code_c0_peg1008(), 200, "int8", "single_scan", "auto"),
            (ira, 24, "int8", "single_scan", "auto"),
            (ira, 16, "1bit", "single_scan", "auto"),
            (W.code_ira16200(), 40, "int8", "single_scan", "auto")]
    _check_jobs(torch_dev, L, orc, spec, max_iter=12, early_stop=True, samples=3)


def test_mixed_full_workload_sampled(torch_dev, L, orc):
    """The full mixed workload (8192 x PEG1008, 2048 x QC7493, 256 x IRA16200,
    128 x IRA64800; int8; 50 iterations; early stop), in the launch
    configuration the measurement uses, against separate calls on every frame
    and the oracle on sampled frames."""
    spec = [(W.code_c0_peg1008(), 8192, "int8", "single_scan", "auto"),
            (W.code_c1_qc7493(), 2048, "int8", "single_scan", "auto"),
            (W.code_ira16200(), 256, "int8", "single_scan", "auto"),
            (W.code_c2_ira64800(), 128, "int8", "single_scan", "auto")]
    _check_jobs(torch_dev, L, orc, spec, max_iter=50, early_stop=True, samples=3, with_llr=False)


def test_graph_replay_equals_eager(torch_dev, L):
    """The mixed call captured into one HIP graph: every replay (with eager
    work and synchronisation between replays) equals the eager call."""
    torch = torch_dev
    spec = [(W.code_c0_peg1008(), 257, "int8"), (W.code_ira16200(), 9, "int8"),
            (W.code_c1_qc7493(), 33, "fp32")]
    items, gcs = [], []
    for k, (code, F, msg) in enumerate(spec):
        gc = L.Code.from_parity_check(code)
        items.append((gc, _dev(torch, _host_llr(code, F, msg, 200 + k)),
                      L.make_params(max_iter=25, early_stop=True, msg=msg)))
        gcs.append(gc)
    mb = L.MultiBatch(items, with_llr=True)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        mb.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    ref = [{k: v.clone() for k, v in o.items()} for o in mb.outputs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mb.run()
    for rep in range(3):
        for o in mb.outputs:
            for v in o.values():
                v.zero_()
        torch.randn(1 << 20, device="cuda").sum().item()  # eager work and a sync between replays
        g.replay()
        torch.cuda.synchronize()
        for k, (o, r) in enumerate(zip(mb.outputs, ref)):
            for key in o:
                assert torch.equal(o[key], r[key]), f"replay {rep} job {k} {key}"
    for gc in gcs:
        gc.close()


@pytest.mark.parametrize("name,msg,sched", [("ira16200", "int8", "single_scan"), ("qc7493", "fp32", "single_scan"),
                                            ("peg1008", "int8", "two_scan")])
def test_autotune_picks_a_feasible_layout(torch_dev, L, name, msg, sched):
    """After autotuning, AUTO decodes with the chosen layout: same results
    as before (layout invariance) and the workspace size of that layout."""
    torch = torch_dev
    code = {"ira16200": W.code_ira16200, "qc7493": W.code_c1_qc7493, "peg1008": W.code_c0_peg1008}[name]()
    F = 96
    x = _dev(torch, _host_llr(code, F, msg, 300))
    gc = L.Code.from_parity_check(code)
    p = L.make_params(max_iter=20, msg=msg, sched=sched)
    before = _np(gc.decode(x, max_iter=20, msg=msg, sched=sched))
    r = gc.autotune(F, p)
    assert r["layout"] in ("reg", "reg1", "lds", "hbm", "frames") and r["tried"] >= 1 and r["ms"] > 0
    forced = L.make_params(max_iter=20, msg=msg, sched=sched, layout=r["layout"])
    assert gc.workspace_size(F, p) == gc.workspace_size(F, forced)
    after = _np(gc.decode(x, max_iter=20, msg=msg, sched=sched))
    for k in before:
        np.testing.assert_array_equal(after[k], before[k], err_msg=f"{k} {name} tuned={r}")
    gc.close()


@pytest.mark.parametrize("name", ["peg1008", "qc7493"])
def test_every_packed_shape_gives_the_same_results(torch_dev, L, orc, name):
    """Each packed shape autotuning may install (PEG: 256 or 1024 threads;
    QC: rows over a lane pair in 512 threads, or on one lane in 768) decodes
    6-, 7- and 8-bit int8 and the 1-bit state on the REG layout exactly as the
    handle's first shape does, and sampled frames equal the oracle."""
    torch = torch_dev
    code = {"qc7493": W.code_c1_qc7493, "peg1008": W.code_c0_peg1008}[name]()
    F, T = 300, 20
    gc = L.Code.from_parity_check(code)
    shapes = gc.packed_shapes()
    assert len(shapes) == 2
    cases = [("int8", 6), ("int8", 7), ("int8", 8), ("1bit", 6)]
    hosts = {}
    for msg, bits in cases:
        Q = (1 << (bits - 1)) - 1
        eb = np.random.default_rng(bits).uniform(1.0, 3.0, size=F)
        hosts[(msg, bits)] = W.quantize_llr(W.awgn_llr(code.N, F, eb, code.design_rate, key=(0xC5, bits)),
                                            step=0.5 if bits == 6 else 0.25, qmax=Q)
    first = {}
    with pytest.raises(L.LdpcError) as ei:  # not one of the listed shapes
        gc.set_packed_shape(99, 2, 256)
    assert ei.value.status == L.LDPC_EUNSUPPORTED
    assert gc.packed_shapes() == shapes
    for shape in shapes + [shapes[0]]:  # and back to the first
        gc.set_packed_shape(*shape)
        info = gc.info()
        assert (info["pk_slots"], info["pk_rows_per_thread"], info["pk_threads"]) == shape
        assert gc.packed_shapes()[0] == shape
        for msg, bits in cases:
            for early_stop in (True, False):
                print(f"[shape] {name} {shape} {msg} {bits}-bit early_stop={early_stop}", flush=True)
                x = _dev(torch, hosts[(msg, bits)])
                g = _np(gc.decode(x, max_iter=T, early_stop=early_stop, msg=msg, layout="reg",
                                  llr_step=0.5 if bits == 6 else 0.25, msg_bits=bits))
                key = (msg, bits, early_stop)
                if key not in first:
                    first[key] = g
                    sel = np.array([0, 1, 77, F - 1])
                    algo = "one_bit" if msg == "1bit" else "single_scan"
                    r = orc.decode(code, hosts[(msg, bits)][sel], algo=algo, arith="int", max_iter=T, alpha=0.8,
                                   early_stop=early_stop, step=0.5 if bits == 6 else 0.25, qbits=bits)
                    for k, rk in (("iters", "iters"), ("ok", "ok"), ("hard", "hard"), ("llr", "post")):
                        np.testing.assert_array_equal(g[k][sel], r[rk].astype(g[k].dtype),
                                                      err_msg=f"{k} {key} {shape}")
                else:
                    for k in g:
                        np.testing.assert_array_equal(g[k], first[key][k], err_msg=f"{k} {key} {shape}")
    gc.close()


@pytest.mark.parametrize("name", ["peg1008", "qc7493"])
def test_autotune_times_packed_shapes(torch_dev, L, name):
    """Autotuning int8 single-scan also times the other packed shape; the
    handle ends on one of the listed shapes (its own unless REG won) and
    decodes as before."""
    torch = torch_dev
    code = {"qc7493": W.code_c1_qc7493, "peg1008": W.code_c0_peg1008}[name]()
    F = 256
    x = _dev(torch, _host_llr(code, F, "int8", 301))
    gc = L.Code.from_parity_check(code)
    shapes = gc.packed_shapes()
    before = _np(gc.decode(x, max_iter=20, msg="int8"))
    p = L.make_params(max_iter=20, msg="int8")
    n_layouts = sum(1 for lay in ("reg", "reg1", "lds", "hbm", "frames")
                    if _feasible(L, gc, F, L.make_params(max_iter=20, msg="int8", layout=lay)))
    r = gc.autotune(F, p)
    assert r["tried"] == n_layouts + len(shapes) - 1, r
    now = gc.packed_shapes()
    assert sorted(now) == sorted(shapes)
    if r["layout"] != "reg":
        assert now[0] == shapes[0]
    after = _np(gc.decode(x, max_iter=20, msg="int8"))
    for k in before:
        np.testing.assert_array_equal(after[k], before[k], err_msg=f"{k} {name} tuned={r} shape={now[0]}")
    gc.close()


def _feasible(L, gc, F, p):
    try:
        gc.workspace_size(F, p)
        return True
    except L.LdpcError:
        return False


def test_single_and_empty_calls(torch_dev, L, orc):
    """One active job runs on the caller's stream; no active job is a no-op."""
    torch = torch_dev
    code = W.code_c0_peg1008()
    _check_jobs(torch, L, orc, [(code, 0, "int8", "single_scan", "auto"),
                                (code, 77, "int8", "single_scan", "hbm")], max_iter=20, early_stop=True, samples=4)
    gc = L.Code.from_parity_check(code)
    x = torch.empty((0, code.N), dtype=torch.int8, device="cuda")
    mb = L.MultiBatch([(gc, x, L.make_params(msg="int8"))])
    mb.run()
    mb0 = L.MultiBatch([])
    mb0.run()
    torch.cuda.synchronize()
    gc.close()


# ---------------------------------------------------------------------------
# One persistent launch (ldpc_decode_multi_persistent): workgroups of 1024
# threads hold 1024 / T frames of one job (PEG code: 4 frames of 256 threads;
# QC code: 2 of 512; IRA codes: 1 of 1024) and take work items from a counter.
@pytest.mark.parametrize("early_stop,with_llr", [(True, False), (True, True), (False, True)])
def test_persistent_mixed_codes(torch_dev, L, orc, early_stop, with_llr):
    """Frame counts that leave groups of the last work item idle (301 = 4 x
    75 + 1 PEG frames, 71 QC frames), a job without frames, and results equal
    to separate calls and to the oracle; with posteriors or without early stop
    every job takes the separate syndrome pass, else the fused one."""
    spec = [(W.code_c0_peg1008(), 301, "int8", "single_scan", "auto"),
            (W.code_c1_qc7493(), 71, "int8", "single_scan", "auto"),
            (W.code_c0_peg1008(), 0, "int8", "single_scan", "auto"),
            (W.code_ira16200(), 21, "int8", "single_scan", "reg"),
            (W.code_c2_ira64800(), 3, "int8", "single_scan", "auto")]
    got = _check_jobs(torch_dev, L, orc, spec, max_iter=30, early_stop=early_stop, samples=5, with_llr=with_llr,
                      persistent=True)
    if early_stop:
        assert len(set(got[0]["iters"].tolist())) > 3


def test_persistent_full_workload(torch_dev, L, orc):
    """The full mixed workload in one persistent launch: every frame equals
    its separate call, sampled frames equal the oracle."""
    spec = [(W.code_c0_peg1008(), 8192, "int8", "single_scan", "auto"),
            (W.code_c1_qc7493(), 2048, "int8", "single_scan", "auto"),
            (W.code_ira16200(), 256, "int8", "single_scan", "auto"),
            (W.code_c2_ira64800(), 128, "int8", "single_scan", "auto")]
    _check_jobs(torch_dev, L, orc, spec, max_iter=50, early_stop=True, samples=3, with_llr=False, persistent=True)


def test_persistent_graph_replays(torch_dev, L):
    """The persistent launch (counter reset kernel + decode kernel) captured
    into a graph: every replay equals the eager call."""
    torch = torch_dev
    spec = [(W.code_c0_peg1008(), 257), (W.code_ira16200(), 9), (W.code_c1_qc7493(), 33)]
    items, gcs = [], []
    for k, (code, F) in enumerate(spec):
        gc = L.Code.from_parity_check(code)
        items.append((gc, _dev(torch, _host_llr(code, F, "int8", 400 + k)),
                      L.make_params(max_iter=25, early_stop=True, msg="int8")))
        gcs.append(gc)
    mb = L.MultiBatch(items, with_llr=False, persistent=True)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        mb.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    ref = [{k: (v.clone() if v is not None else None) for k, v in o.items()} for o in mb.outputs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mb.run()
    for rep in range(3):
        for o in mb.outputs:
            for v in o.values():
                if v is not None:
                    v.zero_()
        torch.randn(1 << 20, device="cuda").sum().item()
        g.replay()
        torch.cuda.synchronize()
        for k, (o, r) in enumerate(zip(mb.outputs, ref)):
            for key in o:
                if o[key] is not None:
                    assert torch.equal(o[key], r[key]), f"replay {rep} job {k} {key}"
    for gc in gcs:
        gc.close()


def test_persistent_refuses_other_kernels(torch_dev, L):
    """Jobs that do not run the 6-bit int8 packed kernel are refused before
    anything is launched."""
    torch = torch_dev
    code = W.code_c0_peg1008()
    gc = L.Code.from_parity_check(code)
    x8 = torch.zeros((8, code.N), dtype=torch.int8, device="cuda")
    xf = torch.zeros((8, code.N), dtype=torch.float32, device="cuda")
    for x, kw in ((xf, dict(msg="fp32")), (x8, dict(msg="1bit")), (x8, dict(msg="int8", layout="hbm")),
                  (x8, dict(msg="int8", msg_bits=7)), (x8, dict(msg="int8", sched="two_scan"))):
        mb = L.MultiBatch([(gc, x, L.make_params(**kw))], persistent=True)
        with pytest.raises(L.LdpcError) as ei:
            mb.run()
        assert ei.value.status == L.LDPC_EUNSUPPORTED, kw
    gc.close()
