#!/usr/bin/env python3
"""Decoder throughput on one MI355X.

Workload: the N=64800 rate-1/2 DVB-S2-shaped IRA code (E = 226,799 edges),
512 frames of seeded BPSK/AWGN channel LLRs at Eb/N0 = 1.0 dB, 6-bit fixed
point (int8), normalised min-sum alpha = 0.8, a fixed 50 iterations (no early
stop), single-scan schedule.  One step = one ldpc_decode_batch call over the
whole batch (every iteration of every frame), with inputs and outputs
resident in device memory.

Prints ONE JSON line: coded Gbit/s (value), edge-updates/s, the roofline of
the decode kernel (HIP events on the launch stream), the other message types
and the two-scan baseline as context, the learned decoder against plain NMS
(FER and average iterations at the same Eb/N0, trained in the run on a
bounded budget), and the CPU oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# context variants of the default run: calls timed after warm-up calls (the
# first calls after a switch of kernel run slower)
VAR_STEPS, VAR_WARMUP = 10, 3
# Packed 16-bit integer VALU rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2
# (two 16-bit operations per lane per instruction) x 2.4 GHz.
ALU16_PEAK_TOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Integer operations the method needs per edge and per check row and
# iteration (Eq. 3 and the NMS/OMS step): subtract, saturate, magnitude,
# min1 / min2 / argmin updates, sign-parity XOR, emitted magnitude select,
# sign application and the posterior add per edge; multiply, round, shift,
# offset and clamp for each of the two normalised magnitudes per row.
ALG_OPS_PER_EDGE = 10
ALG_OPS_PER_ROW = 10

# The decoding kernel of each plan (ldpc_decode_plan): its source files and
# the resource that bounds it.  The fixed-point register kernels keep every
# message on chip (VALU-issue bound); the binary32 and two-scan paths stream
# their per-edge arrays through HBM every iteration.
KERNELS = {
    "packed": (("ss_pk.hip",), "alu"),
    "reg1": (("ss_reg.hip",), "alu"),
    "generic_int": (("ss_int.hip",), "alu"),
    "generic_f32": (("ss_f32.hip",), "hbm"),
    "two_scan": (("two_scan.hip",), "hbm"),
    "f32_frames": (("ss_f32_fl.hip", "fl_common.h"), "hbm"),
    "two_scan_frames": (("two_scan_fl.hip", "fl_common.h"), "hbm"),
}

# HBM bytes per decode call of the benchmark workload measured with rocprofv3
# (FETCH_SIZE x 2 + WRITE_SIZE, calibrated on a device copy, summed over the
# path's kernels), keyed by the hash of the kernel sources the counters were
# taken on; any other source reports traffic as null.
MEASURED_TRAFFIC = [
    {"kernel": "packed", "hash": "b02a9fc1700f7c6d", "workload": ("int8", "single_scan", 512, 50),
     "bytes": 240.7e6, "profile": "profiles/ss_pk_int8_ira64800_512f.md"},
    {"kernel": "packed", "hash": "b02a9fc1700f7c6d", "workload": ("1bit", "single_scan", 512, 50),
     "bytes": 240.6e6, "profile": "profiles/ss_pk_1bit_ira64800_512f.md"},
    {"kernel": "f32_frames", "hash": "1c5cdaa9c2275be3", "workload": ("fp32", "single_scan", 512, 50),
     "bytes": 105147.1e6, "profile": "profiles/fl_f32_ira64800_512f.md"},
    {"kernel": "reg1", "hash": "e7d86239f37f995e", "workload": ("int8", "single_scan", 512, 50),
     "bytes": 221.2e6, "profile": "profiles/ss_reg_int8_ira64800_512f.md"},
    {"kernel": "two_scan_frames", "hash": "0f330c006512febe", "workload": ("int8", "two_scan", 512, 50),
     "bytes": 29393.9e6, "profile": "profiles/ts_fl_int8_ira64800_512f.md"},
    {"kernel": "two_scan_frames", "hash": "0f330c006512febe", "workload": ("fp32", "two_scan", 512, 50),
     "bytes": 107937.4e6, "profile": "profiles/ts_fl_f32_ira64800_512f.md"},
]


# Algorithmic bytes per frame and iteration of each path (E edges, N
# variables, M checks): what a decoder that keeps nothing on chip between
# iterations must move.
def alg_bytes_per_frame_iter(msg: str, sched: str, E: int, N: int, M: int) -> int:
    if sched == "two_scan":
        return 4 * E + 3 * N if msg == "int8" else 16 * E + 8 * N
    if msg == "int8":
        return 2 * E + 5 * N
    if msg == "1bit":
        return 2 * ((E + 7) // 8) + 4 * M + 5 * N
    return 8 * E + 12 * N


def source_hash(names) -> str:
    """sha256 prefix of the kernel's source files, concatenated in order."""
    import hashlib
    h = hashlib.sha256()
    for name in names:
        h.update(open(os.path.join(ROOT, "paper_cs_0609090_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


# Workload codes: (constructor name in workloads.py, default Eb/N0 in dB)
CODES = {"ira64800": ("code_c2_ira64800", 1.0), "peg1008": ("code_c0_peg1008", 2.0),
         "qc7493": ("code_c1_qc7493", 2.0), "ira16200": ("code_ira16200", 1.2)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_decode(torch, gcode, ldpc, x, params, steps, warmup, with_llr=True):
    F = x.shape[0]
    out = gcode.alloc_outputs(F, x.device, with_llr)
    ws = gcode.alloc_workspace(F, params, x.device)
    stream = torch.cuda.current_stream(x.device)

    def step():
        gcode.decode_into(x, params, out["hard"], out["llr"], out["iters"], out["ok"], ws, stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) * 1e-3 for a, b in ev]
    return wall, per, out


def _oracle_wall(code, q, algo: str, threads: int, max_iter: int = 50) -> float:
    """Wall time of the fixed-point oracle (max_iter iterations, no early stop) on
    the frames of q, split evenly over `threads` threads (ctypes releases
    the GIL, so the threads run the C decoder in parallel)."""
    import oracle
    chunks = np.array_split(np.arange(q.shape[0]), threads)
    ts = [threading.Thread(target=lambda idx=idx: oracle.decode(
        code, q[idx], algo=algo, arith="int", max_iter=max_iter, alpha=0.8, early_stop=False))
        for idx in chunks if idx.size]
    t0 = time.perf_counter()
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    return time.perf_counter() - t0


def host_threads() -> tuple[int, int]:
    """(threads used, CPUs the host reports): the process's CPU affinity,
    capped at 16, the host CPU share given to one GPU."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail)), os.cpu_count() or avail


def cpu_baseline(code, q, frames: int, single_frames: int, max_iter: int = 50) -> dict:
    """The oracle timed on the host: fixed-point single-scan on `frames`
    frames over all threads of the host share (the headline figure), the
    same decoder single-threaded on `single_frames` frames, and the oracle's
    two-scan decoder single-threaded on those same frames for the
    single-scan / two-scan ratio (the paper's speed claim is a ratio of
    software decoders)."""
    import oracle
    oracle.lib()
    threads, host_cpus = host_threads()
    wall_mt = _oracle_wall(code, q[:frames], "single_scan", threads, max_iter)
    qs = q[:single_frames]
    wall_1 = _oracle_wall(code, qs, "single_scan", 1, max_iter)
    wall_two = _oracle_wall(code, qs, "two_scan", 1, max_iter)
    rate = lambda nf, w: nf * code.N / w / 1e9  # noqa: E731
    return {"value": rate(frames, wall_mt), "unit": "coded Gbit/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{frames} of the {q.shape[0]} frames, {max_iter} iterations each, fixed-point single-scan "
                      f"oracle (C, -O2), frames split over {threads} threads; single-thread figures "
                      f"on the first {single_frames} frames",
            "host_cpus": host_cpus,
            "wall_s": round(wall_mt, 3),
            "edge_updates_per_s": frames * max_iter * code.E / wall_mt,
            "single_thread": {"coded_gbps": rate(single_frames, wall_1),
                              "edge_updates_per_s": single_frames * max_iter * code.E / wall_1,
                              "wall_s": round(wall_1, 3)},
            "two_scan_single_thread": {"coded_gbps": rate(single_frames, wall_two),
                                       "wall_s": round(wall_two, 3)},
            "single_scan_over_two_scan": round(wall_two / wall_1, 3),
            "paper_ratio": "more than 2x (software, Sec. I; hardware not stated)",
            "ratio_note": "both oracle decoders are literal transcriptions (exclusion-form check "
                          "update; two-scan forms every Z_mn as its own exclusion sum of Eq. 2), "
                          "not tuned software decoders"}


def learned_vs_nms(steps: int, eval_frames: int) -> dict:
    """Learned per-iteration, per-class normalisation and offset (T = 20
    pairs per check-degree class, trained with Adam on the adjoint kernels)
    against NMS alpha = 0.8, both binary32 with early stop and at most 50
    iterations, on the same fresh frames of the N=7493 QC code at 3.25 dB.
    Training: `steps` batches of 1024 random codewords at 2.75-3.75 dB, from
    (0.6, 0): the range where this code decodes (it does not below 2.75 dB
    with any constant normalisation)."""
    from paper_cs_0609090_amd import learn as LRN
    from paper_cs_0609090_amd import ldpc
    from paper_cs_0609090_amd import workloads as W
    log(f"[bench] learned decoder: {steps} x 1024 training frames, {eval_frames} evaluation frames")
    gq = ldpc.Code.from_parity_check(W.code_c1_qc7493())
    t0 = time.time()
    w, tlog = LRN.train(gq, T=20, steps=steps, batch=1024, ebn0=(2.75, 3.75), lr=0.02, init=(0.6, 0.0),
                        log_every=max(steps, 1))
    t_train = time.time() - t0
    ev = LRN.evaluate(gq, w, 3.25, eval_frames, nms_alpha=0.8)
    gq.close()
    return {"code": "qc7493", "ebn0_db": 3.25, "fer_learned": ev["learned"]["fer"], "fer_nms": ev["nms"]["fer"],
            "avg_iters_learned": round(ev["learned"]["avg_iters"], 3), "avg_iters_nms": round(ev["nms"]["avg_iters"], 3),
            "iter_saving": round(ev["iter_saving"], 4), "eval_frames": eval_frames, "max_iter": 50,
            "nms_alpha": 0.8, "T": 20, "train_frames": steps * 1024, "train_ebn0_db": [2.75, 3.75],
            "train_s": round(t_train, 2), "final_val_loss": tlog[-1]["val_loss"] if tlog else None,
            "dtype": "f32"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=512)
    ap.add_argument("--code", default="ira64800", choices=sorted(CODES),
                    help="workload code (default: the N=64800 IRA code of the headline figure; the "
                         "others profile their own shapes)")
    ap.add_argument("--ebn0", type=float, default=None, help="Eb/N0 in dB (default: the code's own)")
    ap.add_argument("--max-iter", type=int, default=50)
    ap.add_argument("--msg", default="int8", choices=["int8", "1bit", "fp32"])
    ap.add_argument("--sched", default="single_scan", choices=["single_scan", "two_scan"])
    ap.add_argument("--layout", default="auto", choices=["auto", "lds", "hbm", "reg", "reg1", "frames"])
    ap.add_argument("--msg-bits", type=int, default=6, choices=[6, 7, 8],
                    help="fixed-point message width (int8 only; the LLR step halves per extra bit)")
    ap.add_argument("--cpu-frames", type=int, default=192)
    ap.add_argument("--cpu-single-frames", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-steps", type=int, default=256,
                    help="training steps of 1024 frames for the learned-decoder comparison")
    ap.add_argument("--learned-eval-frames", type=int, default=65536)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after timing, copy a buffer of this size once (calibrates "
                         "the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: frames are independent, so the decoder "
              "shards by splitting the batch; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_cs_0609090_amd import ldpc
    from paper_cs_0609090_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    ctor, ebn0_default = CODES[args.code]
    code = getattr(W, ctor)()
    N, M, E, F = code.N, code.M, code.E, args.frames
    ebn0 = ebn0_default if args.ebn0 is None else args.ebn0
    max_iter, alpha = args.max_iter, 0.8
    log(f"[bench] generating {F} frames of N={N} at {ebn0} dB")
    key = (0xC2, 0xBE) if args.code == "ira64800" else (0xBE, sorted(CODES).index(args.code))
    llr = W.awgn_llr(N, F, ebn0, code.design_rate, key=key)
    step = 0.5 / (1 << (args.msg_bits - 6))
    q = W.quantize_llr(llr, step=step, qmax=(1 << (args.msg_bits - 1)) - 1)
    gcode = ldpc.Code.from_parity_check(code, device=0)
    xq = torch.from_numpy(q).to(dev)
    xf = torch.from_numpy(llr).to(dev)

    def run(msg, sched, steps, warmup, layout="auto", early_stop=False, with_llr=True):
        bits = args.msg_bits if msg == "int8" else 0
        p = ldpc.make_params(max_iter=max_iter, alpha=alpha, early_stop=early_stop, msg=msg,
                             sched=sched, layout=layout, msg_bits=bits, llr_step=step)
        x = xf if msg == "fp32" else xq
        wall, per, out = time_decode(torch, gcode, ldpc, x, p, steps, warmup, with_llr)
        iters = out["iters"].to(torch.int64).sum().item()
        ok = out["ok"].to(torch.int64).sum().item()
        kern = float(np.mean(per))
        return {"wall": wall, "kernel_s": kern, "per": per, "iters": iters, "ok": ok,
                "gbps": F * N * steps / wall / 1e9,
                "eups": iters * E * steps / wall,
                "alg_bytes": alg_bytes_per_frame_iter(msg, sched, E, N, M) * iters}

    log(f"[bench] main: msg={args.msg} sched={args.sched} steps={args.steps} warmup={args.warmup}")
    r = run(args.msg, args.sched, args.steps, args.warmup, args.layout)
    achieved_hbm = r["alg_bytes"] / r["kernel_s"] / 1e9
    alg_ops = (ALG_OPS_PER_EDGE * E + ALG_OPS_PER_ROW * M) * r["iters"]
    achieved_alu = alg_ops / r["kernel_s"] / 1e12
    plan = gcode.plan(F, ldpc.make_params(max_iter=max_iter, alpha=alpha, early_stop=False, msg=args.msg,
                                          sched=args.sched, layout=args.layout,
                                          msg_bits=args.msg_bits if args.msg == "int8" else 0))
    srcs, bound = KERNELS[plan["kernel"]]
    h = source_hash(srcs)
    traffic = next((t["bytes"] for t in MEASURED_TRAFFIC if t["kernel"] == plan["kernel"] and t["hash"] == h
                    and t["workload"] == (args.msg, args.sched, F, max_iter) and args.msg_bits == 6
                    and t.get("code", "ira64800") == args.code), None)
    kernel_desc = {"kernel": plan["kernel"], "sources": list(srcs), "threads": plan["threads"]}
    if plan["frames_per_lane"]:
        kernel_desc["frames_per_lane"] = plan["frames_per_lane"]
        kernel_desc["launch"] = "one decode call: check and variable pass per iteration"
    res = {
        "metric": f"coded Gbit/s + edge-updates/s at max {max_iter} iters; learned vs plain NMS FER @ same Eb/N0",
        "value": round(r["gbps"], 4),
        "unit": "coded Gbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["wall"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"int8": "int8", "1bit": "1bit+int8", "fp32": "f32"}[args.msg],
        "data": f"synthetic: seeded Philox4x32-10 BPSK/AWGN LLRs, seeded {args.code} code",
        "config": {"workload": (f"{args.code}_r{code.N - code.M}/{code.N}_{F}frames_{ebn0}dB_{args.msg}_"
                                f"{args.sched}_max{max_iter}_noearlystop"
                                if args.code != "ira64800" else
                                f"ira64800_r1/2_{F}frames_{ebn0}dB_{args.msg}_{args.sched}_"
                                f"max{max_iter}_noearlystop") + (f"_{args.msg_bits}bit" if args.msg_bits != 6 else ""),
                   "N": N, "M": M, "E": E, "frames": F, "max_iter": max_iter,
                   "early_stop": False, "alpha": alpha, "ebn0_db": ebn0,
                   "msg": args.msg, "sched": args.sched, "layout": args.layout,
                   **({"msg_bits": args.msg_bits, "llr_step": step} if args.msg_bits != 6 else {})},
        "edge_updates_per_s": r["eups"],
    }
    if bound == "alu":
        res["roofline"] = {"bound": "alu", "achieved": round(achieved_alu, 3),
                           "peak": round(ALU16_PEAK_TOPS, 2), "unit": "TOP/s",
                           "frac": round(achieved_alu / ALU16_PEAK_TOPS, 4),
                           "traffic": traffic,
                           "kernel_ms": round(r["kernel_s"] * 1e3, 4),
                           "alg_ops_per_launch": alg_ops, **kernel_desc}
        res["hbm_equivalent"] = {"achieved": round(achieved_hbm, 2), "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": round(achieved_hbm / HBM_PEAK_GBS, 4),
                                 "alg_bytes_per_launch": r["alg_bytes"],
                                 "note": "bytes a decoder that streams messages and posteriors "
                                         "through HBM every iteration would move"}
    else:
        res["roofline"] = {"bound": "hbm", "achieved": round(achieved_hbm, 2), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(achieved_hbm / HBM_PEAK_GBS, 4),
                           "traffic": traffic,
                           "kernel_ms": round(r["kernel_s"] * 1e3, 4),
                           "alg_bytes_per_launch": r["alg_bytes"], **kernel_desc}
    if not args.no_variants:
        var = {}
        for msg, sched in (("1bit", "single_scan"), ("fp32", "single_scan"),
                           ("int8", "two_scan"), ("fp32", "two_scan")):
            if (msg, sched) == (args.msg, args.sched):
                continue
            log(f"[bench] variant {msg} {sched}")
            v = run(msg, sched, VAR_STEPS, VAR_WARMUP)
            var[f"{msg}_{sched}"] = {"coded_gbps": round(v["gbps"], 4),
                                     "edge_updates_per_s": v["eups"],
                                     "ms_per_step": round(v["wall"] / VAR_STEPS * 1e3, 4),
                                     "hbm_frac_alg": round(v["alg_bytes"] / v["kernel_s"] / 1e9 / HBM_PEAK_GBS, 4)}
        log("[bench] early-stop regime")
        # the early-stop regime as a FER measurement runs it: hard decisions only
        v = run(args.msg, args.sched, VAR_STEPS, VAR_WARMUP, early_stop=True, with_llr=False)
        var["early_stop"] = {"coded_gbps": round(v["gbps"], 4),
                             "avg_iters": v["iters"] / F, "fer": 1.0 - v["ok"] / F,
                             "ms_per_step": round(v["wall"] / VAR_STEPS * 1e3, 4), "outputs": "hard decisions"}
        res["variants"] = var
    if not args.no_learned:
        res["learned"] = learned_vs_nms(args.learned_steps, args.learned_eval_frames)
    if not args.no_cpu_baseline:
        threads, host_cpus = host_threads()
        log(f"[bench] cpu oracle baseline: {args.cpu_frames} frames on {threads} of {host_cpus} host CPUs, "
            f"then {args.cpu_single_frames} frames on one thread (single- and two-scan)")
        res["cpu_baseline"] = cpu_baseline(code, q, min(args.cpu_frames, F), min(args.cpu_single_frames, F),
                                           max_iter)
    if args.copy_probe_mib > 0:
        src = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device=dev)
        src.fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        res["copy_probe_bytes"] = args.copy_probe_mib << 20
    gcode.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
