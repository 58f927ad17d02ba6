"""Mixed batch of several codes through ldpc_decode_multi (include/ldpc_multi.h).

Workload: 8192 frames of the N=1008 (3,6) PEG code, 2048 of the N=7493 QC
code, 256 of the N=16200 IRA code and 128 of the N=64800 IRA code; int8
messages (6-bit values, step 0.5), Eb/N0 drawn uniformly in [1, 3] dB per
frame, all-zero codeword, 50 iterations, normalisation 0.8, per-frame early
stop.  Channel LLRs are drawn on the GPU (ldpc_channel_awgn) before timing.

Timed, each on inputs already in device memory:
  sequential  the four ldpc_decode_batch calls one after another on one stream
  multi       one ldpc_decode_multi call (jobs forked onto library streams)
  graph       a HIP graph holding that call, replayed
  persistent  one ldpc_decode_multi_persistent call (a single launch of
              1024-thread workgroups taking work items from a counter)

    python -m paper_cs_0609090_amd.mixed --reps 20 [--autotune] [--no-early-stop]
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import torch

from . import ldpc
from . import workloads as W

MIX = (("peg1008", W.code_c0_peg1008, 8192), ("qc7493", W.code_c1_qc7493, 2048),
       ("ira16200", W.code_ira16200, 256), ("ira64800", W.code_c2_ira64800, 128))


def ebn0_per_frame(n: int, seed: int, lo: float = 1.0, hi: float = 3.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


def device_llr(code, ebn0: np.ndarray, key, step: float = 0.5):
    """int8 channel LLRs [F, N] on the GPU, one Eb/N0 per frame (design rate)."""
    sig = torch.tensor([W.ebn0_to_sigma(float(e), code.design_rate) for e in ebn0], dtype=torch.float64,
                       device="cuda")
    _, q = ldpc.channel_awgn(sig, code.N, key=key, want_f32=False, want_q=True, step=step)
    return q


def build(scale: float = 1.0, max_iter: int = 50, early_stop: bool = True, alpha: float = 0.8,
          autotune: bool = False, with_llr: bool = False, seed: int = 0xC3):
    """Codes, device handles, inputs and a MultiBatch of the workload (frame
    counts multiplied by ``scale``)."""
    codes, gcodes, items, tuned = [], [], [], {}
    for k, (name, make, F) in enumerate(MIX):
        F = max(1, int(round(F * scale)))
        code = make()
        gc = ldpc.Code.from_parity_check(code)
        p = ldpc.make_params(max_iter=max_iter, alpha=alpha, early_stop=early_stop, msg="int8")
        if autotune:
            tuned[name] = gc.autotune(F, p)
        x = device_llr(code, ebn0_per_frame(F, seed + k), key=(seed, k))
        codes.append(code)
        gcodes.append(gc)
        items.append((gc, x, p))
    return codes, gcodes, ldpc.MultiBatch(items, with_llr=with_llr), tuned


def _time(fn, reps: int, warmup: int) -> float:
    """Median milliseconds of fn() on the current stream (events bracket the
    caller's stream, which every forked job joins back into)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(s)
        fn()
        b.record(s)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def measure(reps: int = 20, warmup: int = 3, scale: float = 1.0, early_stop: bool = True,
            autotune: bool = False, graph: bool = True) -> dict:
    codes, gcodes, mb, tuned = build(scale=scale, early_stop=early_stop, autotune=autotune)
    bits = sum(int(x.shape[0]) * c.N for c, (_, x, _) in zip(codes, mb.items))

    def sequential():
        for (gc, x, p), out in zip(mb.items, mb.outputs):
            gc.decode_into(x, p, out["hard"], None, out["iters"], out["ok"], mb.workspace)

    t_seq = _time(sequential, reps, warmup)
    iters_seq = [o["iters"].clone() for o in mb.outputs]
    hard_seq = [o["hard"].clone() for o in mb.outputs]
    t_multi = _time(mb.run, reps, warmup)
    same = all(torch.equal(a, o["iters"]) and torch.equal(h, o["hard"])
               for a, h, o in zip(iters_seq, hard_seq, mb.outputs))
    mp = ldpc.MultiBatch(mb.items, with_llr=False, persistent=True)
    t_pers = _time(mp.run, reps, warmup)
    same_p = all(torch.equal(a, o["iters"]) and torch.equal(h, o["hard"])
                 for a, h, o in zip(iters_seq, hard_seq, mp.outputs))
    res = {"workload": "mixed: " + ", ".join(f"{int(x.shape[0])}x{n}" for (n, _, _), (_, x, _) in
                                              zip(MIX, mb.items)),
           "coded_bits": bits, "early_stop": early_stop, "ms_sequential": t_seq, "ms_multi": t_multi,
           "gbps_sequential": bits / t_seq / 1e6, "gbps_multi": bits / t_multi / 1e6,
           "multi_equals_sequential": bool(same), "tuned": tuned,
           "ms_persistent": t_pers, "gbps_persistent": bits / t_pers / 1e6,
           "persistent_equals_sequential": bool(same_p)}
    if graph:
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            mb.run()  # the first call creates the library's stream pool
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            mb.run()
        t_graph = _time(g.replay, reps, warmup)
        same_g = all(torch.equal(a, o["iters"]) and torch.equal(h, o["hard"])
                     for a, h, o in zip(iters_seq, hard_seq, mb.outputs))
        res.update({"ms_graph": t_graph, "gbps_graph": bits / t_graph / 1e6, "graph_equals_sequential": bool(same_g)})
    iters = [float(o["iters"].float().mean()) for o in mb.outputs]
    ok = [float(o["ok"].float().mean()) for o in mb.outputs]
    res["avg_iters"] = {n: round(i, 3) for (n, _, _), i in zip(MIX, iters)}
    res["frac_codeword"] = {n: round(o, 4) for (n, _, _), o in zip(MIX, ok)}
    edge_updates = sum(float(o["iters"].double().sum()) * c.E for c, o in zip(codes, mb.outputs))
    res["edge_updates_per_s_multi"] = edge_updates / (t_multi * 1e-3)
    for gc in gcodes:
        gc.close()
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0, help="multiply every job's frame count")
    ap.add_argument("--no-early-stop", action="store_true")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    a = ap.parse_args(argv)
    print(json.dumps(measure(a.reps, a.warmup, a.scale, not a.no_early_stop, a.autotune, not a.no_graph)),
          flush=True)


if __name__ == "__main__":
    main()
