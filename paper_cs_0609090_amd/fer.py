"""FER/BER measurement with random codewords, entirely on the GPU.

Per batch: Philox information bits -> systematic encoder -> BPSK/AWGN
channel LLRs (binary32, or b-bit fixed point for the int8 / 1-bit decoders:
b = 6 by default, 7 or 8 with ``msg_bits``)
-> ``ldpc_decode_batch`` -> per-frame bit errors against the transmitted
codeword.  All steps are library calls (include/ldpc.h, include/ldpc_sim.h);
this module only drives them and adds up the counts.

Eb/N0 uses the true code rate K/N (K = N - rank H from the encoder):
sigma^2 = 1 / (2 (K/N) 10^(Eb/N0 / 10)).  Information bits use Philox stream
1 and the channel stream 0, both keyed by ``key``; frame f of the point uses
frame counter ``frame_offset + f``, so a point's frames are reproducible and
independent of the batch size.

    python -m paper_cs_0609090_amd.fer --code peg1008 --ebn0 1.5 2.0 2.5 --frames 20000
    python -m paper_cs_0609090_amd.fer --msg-bits 7 --llr-step 0.25 --schedule "0.7,0;0.8,0;0.9,0"
"""
from __future__ import annotations

import argparse
import json
import math
import time

import torch

from . import ldpc
from . import workloads as W

CODES = {"peg1008": W.code_c0_peg1008, "qc7493": W.code_c1_qc7493, "ira64800": W.code_c2_ira64800,
         "ira16200": W.code_ira16200}


def sigma_for(ebn0_db: float, rate: float) -> float:
    return math.sqrt(1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0)))


def run_point(gcode: "ldpc.Code", ebn0_db: float, frames: int, batch: int = 4096, msg: str = "int8",
              sched: str = "single_scan", max_iter: int = 50, alpha: float = 0.8, beta: float = 0.0,
              early_stop: bool = True, llr_step: float = 0.5, key=(0x5EED, 1), frame_offset: int = 0,
              device="cuda", msg_bits: int = 0, schedule=None, layout: str = "auto") -> dict:
    """Decode ``frames`` random codewords at one Eb/N0; returns the counts.
    ``schedule``: None or a float32 device tensor [T][1][2] of per-iteration
    (alpha_k, beta_k) pairs (one pair for every row)."""
    enc = gcode.encoder_info()
    K, N = enc["K"], gcode.N
    rate = K / N
    sg = sigma_for(ebn0_db, rate)
    params = ldpc.make_params(max_iter=max_iter, alpha=alpha, beta=beta, early_stop=early_stop, msg=msg,
                              sched=sched, llr_step=llr_step, layout=layout, weights=schedule,
                              weight_classes=1 if schedule is not None else 0, msg_bits=msg_bits)
    qmax = (1 << ((msg_bits or 6) - 1)) - 1
    bsz = min(batch, frames)
    ws = gcode.alloc_workspace(bsz, params, device)
    outs = gcode.alloc_outputs(bsz, device, with_llr=False)
    sigma = torch.full((bsz,), sg, dtype=torch.float64, device=device)
    fe = torch.zeros((), dtype=torch.int64, device=device)   # frames in error
    be = torch.zeros((), dtype=torch.int64, device=device)   # bit errors
    fail = torch.zeros((), dtype=torch.int64, device=device)  # syndrome not satisfied
    its = torch.zeros((), dtype=torch.int64, device=device)
    t_dec = 0.0
    done = 0
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    while done < frames:
        n = min(bsz, frames - done)
        off = frame_offset + done
        info = ldpc.random_bits(n, K, key=key, stream_id=1, frame_offset=off, device=device)
        cw = gcode.encode(info)
        f32, q = ldpc.channel_awgn(sigma[:n], N, codewords=cw, key=key, stream_id=0, frame_offset=off,
                                   want_f32=msg == "fp32", want_q=msg != "fp32", step=llr_step, qmax=qmax)
        x = f32 if msg == "fp32" else q
        o = {k: (v[:n] if v is not None else None) for k, v in outs.items()}
        ev0.record()
        gcode.decode_into(x, params, o["hard"], None, o["iters"], o["ok"], ws)
        ev1.record()
        errs = ldpc.count_errors(o["hard"], cw)
        fe += (errs > 0).sum()
        be += errs.sum()
        fail += (o["ok"] == 0).sum()
        its += o["iters"].sum()
        torch.cuda.synchronize()
        t_dec += ev0.elapsed_time(ev1) * 1e-3
        done += n
    fe_, be_, fail_, its_ = int(fe), int(be), int(fail), int(its)
    return {"ebn0_db": ebn0_db, "frames": frames, "K": K, "N": N, "rate": rate, "sigma": sg,
            "frame_errors": fe_, "bit_errors": be_, "fer": fe_ / frames, "ber": be_ / (frames * N),
            "detected_failures": fail_, "avg_iters": its_ / frames, "decode_s": t_dec,
            "coded_gbps": frames * N / t_dec / 1e9 if t_dec > 0 else None}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--code", default="peg1008", choices=sorted(CODES))
    ap.add_argument("--ebn0", type=float, nargs="+", default=[1.5, 2.0, 2.5])
    ap.add_argument("--frames", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--msg", default="int8", choices=["int8", "1bit", "fp32"])
    ap.add_argument("--sched", default="single_scan", choices=["single_scan", "two_scan"])
    ap.add_argument("--max-iter", type=int, default=50)
    ap.add_argument("--alpha", type=float, default=0.8)
    ap.add_argument("--beta", type=float, default=0.0)
    ap.add_argument("--msg-bits", type=int, default=0, help="fixed-point message width: 6 (default), 7 or 8")
    ap.add_argument("--llr-step", type=float, default=0.5, help="LLR value of one fixed-point unit")
    ap.add_argument("--schedule", default=None,
                    help="per-iteration pairs 'a1,b1;a2,b2;...' (the last repeats), instead of alpha/beta")
    ap.add_argument("--layout", default="auto", choices=sorted(ldpc.LAYOUT))
    args = ap.parse_args(argv)
    code = CODES[args.code]()
    gcode = ldpc.Code.from_parity_check(code)
    sch = None
    if args.schedule:
        rows = [[float(v) for v in r.split(",")] for r in args.schedule.split(";") if r.strip()]
        sch = torch.tensor(rows, dtype=torch.float32, device="cuda").reshape(-1, 1, 2)
    for e in args.ebn0:
        r = run_point(gcode, e, args.frames, batch=args.batch, msg=args.msg, sched=args.sched,
                      max_iter=args.max_iter, alpha=args.alpha, beta=args.beta, llr_step=args.llr_step,
                      msg_bits=args.msg_bits, schedule=sch, layout=args.layout)
        r.update(code=args.code, msg=args.msg, sched=args.sched, alpha=args.alpha, beta=args.beta,
                 max_iter=args.max_iter, msg_bits=args.msg_bits or 6, llr_step=args.llr_step,
                 schedule=args.schedule)
        print(json.dumps(r), flush=True)
    gcode.close()


if __name__ == "__main__":
    main()
