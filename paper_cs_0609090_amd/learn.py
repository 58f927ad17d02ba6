"""Learned normalised/offset min-sum (include/ldpc_learn.h): training and
evaluation on the GPU.

``LearnedMinSum.apply(weights, code, llr, target, ckpt, workspace)`` is the
summed BCE loss of the decoder unrolled over T = weights.shape[0] iterations
with the per-iteration, per-class pairs ``weights`` [T][C][2]; its backward
is the library's adjoint kernel.  ``train`` fits the pairs with Adam on
frames drawn on the GPU (random codewords, BPSK/AWGN with Eb/N0 uniform per
frame); ``evaluate`` decodes fresh frames with the trained pairs through
``ldpc_decode_batch`` (per-frame early stop) next to plain NMS, on the same
frames, and reports FER and average iterations.

    python -m paper_cs_0609090_amd.learn --code peg1008 --T 20 --steps 1024
    python -m paper_cs_0609090_amd.learn --code qc7493 --ebn0-lo 2.75 --ebn0-hi 3.75 --init-alpha 0.6 \
        --lr 0.02 --eval-ebn0 3.0 3.25 3.5 --eval-frames 20000 --nms-alpha 0.8 0.5
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import fer as FER
from . import ldpc


class LearnedMinSum(torch.autograd.Function):
    """Loss of the unrolled decoder, sum_t w_t loss_t (w_t = ``loss_weights``,
    a host sequence of T numbers, or all ones); gradients only for the weights."""

    @staticmethod
    def forward(ctx, weights, gcode, llr, target, ckpt, workspace, loss_weights=None):
        w = weights.detach().contiguous()
        loss_t = gcode.learn_forward(llr, target, w, ckpt, workspace)
        ctx.gcode, ctx.target, ctx.ckpt, ctx.workspace, ctx.n = gcode, target, ckpt, workspace, llr.shape[0]
        ctx.lw = None if loss_weights is None else [float(v) for v in loss_weights]
        ctx.save_for_backward(w)
        if ctx.lw is None:
            return loss_t.sum()
        return (loss_t * torch.tensor(ctx.lw, dtype=loss_t.dtype, device=loss_t.device)).sum()

    @staticmethod
    def backward(ctx, g):
        (w,) = ctx.saved_tensors
        grad = ctx.gcode.learn_backward(ctx.n, ctx.target, w, ctx.ckpt, ctx.workspace, loss_weights=ctx.lw)
        return grad * g, None, None, None, None, None, None


def _frames(gcode, K, n, ebn0_lo, ebn0_hi, key, offset, rng):
    """n random codewords and their binary32 channel LLRs (Eb/N0 uniform per frame)."""
    info = ldpc.random_bits(n, K, key=key, stream_id=1, frame_offset=offset)
    cw = gcode.encode(info)
    eb = rng.uniform(ebn0_lo, ebn0_hi, size=n)
    rate = K / gcode.N
    sig = torch.tensor([FER.sigma_for(float(e), rate) for e in eb], dtype=torch.float64, device="cuda")
    llr, _ = ldpc.channel_awgn(sig, gcode.N, codewords=cw, key=key, stream_id=0, frame_offset=offset)
    return llr, cw


def init_weights(n_classes: int, T: int, alpha: float = 0.8, beta: float = 0.0) -> torch.Tensor:
    w = torch.empty((T, n_classes, 2), dtype=torch.float32, device="cuda")
    w[:, :, 0] = alpha
    w[:, :, 1] = beta
    return w


def train(gcode, T: int = 20, steps: int = 1024, batch: int = 1024, ebn0=(1.5, 2.5), lr: float = 0.01,
          ckpt: int = 5, key=(0x7EA, 1), seed: int = 0, log_every: int = 64, init=(0.8, 0.0),
          tie_classes: bool = False, loss_decay: float = 1.0):
    """Adam on the [T][C][2] pairs; returns (weights [T][C][2], log).  With
    ``tie_classes`` one pair per iteration is shared by every class (its
    gradient is the sum of the classes').  ``loss_decay`` g weights iteration
    t's loss by g^(t-1) (normalised to sum T; 1 = the plain sum): g < 1
    rewards posteriors that are right early, i.e. fewer iterations.  The log
    holds the training objective and that of one fixed validation batch
    (frames outside the training stream), both per bit and iteration."""
    C = len(gcode.degree_classes())
    K = gcode.encoder_info()["K"]
    param = init_weights(1 if tie_classes else C, T, *init).requires_grad_(True)
    opt = torch.optim.Adam([param], lr=lr)

    def full():
        return param.expand(T, C, 2) if tie_classes else param
    ws = torch.empty(gcode.learn_workspace_size(batch, T, ckpt), dtype=torch.uint8, device="cuda")
    lw = None
    if loss_decay != 1.0:
        g = loss_decay ** np.arange(T, dtype=np.float64)
        lw = (g * (T / g.sum())).tolist()
    lw_t = None if lw is None else torch.tensor(lw, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(seed)
    vllr, vcw = _frames(gcode, K, batch, ebn0[0], ebn0[1], key, 1 << 28, np.random.default_rng(seed + 1))
    log = []
    scale = 1.0 / (batch * gcode.N * T)
    t0 = time.time()
    for step in range(steps):
        llr, cw = _frames(gcode, K, batch, ebn0[0], ebn0[1], key, step * batch, rng)
        loss = LearnedMinSum.apply(full(), gcode, llr, cw, ckpt, ws, lw) * scale
        opt.zero_grad()
        loss.backward()
        opt.step()
        with torch.no_grad():
            param[:, :, 0].clamp_(0.05, 1.5)
            param[:, :, 1].clamp_(0.0, 4.0)
        if step % log_every == 0 or step == steps - 1:
            with torch.no_grad():
                vlt = gcode.learn_forward(vllr, vcw, full().detach().contiguous(), ckpt, ws)
                vl = float(vlt.sum() if lw_t is None else (vlt * lw_t).sum()) * scale
            log.append({"step": step, "loss": float(loss.detach()), "val_loss": vl, "s": time.time() - t0})
    return full().detach().contiguous(), log


def evaluate(gcode, weights, ebn0_db: float, frames: int, batch: int = 4096, nms_alpha: float = 0.8,
             nms_iters: int = 50, learned_iters: int | None = None, key=(0x5EED, 9), offset: int = 1 << 24):
    """FER / BER / average iterations of the learned decoder (early stop; its
    T = weights rows apply to the first T iterations and the last row to any
    later one, up to learned_iters, default nms_iters) and of plain NMS
    (nms_iters, early stop) on the same random-codeword frames."""
    K = gcode.encoder_info()["K"]
    rate = K / gcode.N
    sg = FER.sigma_for(ebn0_db, rate)
    T = int(weights.shape[0])
    li = nms_iters if learned_iters is None else learned_iters
    pl = ldpc.make_params(max_iter=li, msg="fp32", early_stop=True, weights=weights)
    pn = ldpc.make_params(max_iter=nms_iters, alpha=nms_alpha, msg="fp32", early_stop=True, layout="frames")
    res = {"learned": np.zeros(4), "nms": np.zeros(4)}  # frame errors, bit errors, iterations, frames
    done = 0
    while done < frames:
        n = min(batch, frames - done)
        info = ldpc.random_bits(n, K, key=key, stream_id=1, frame_offset=offset + done)
        cw = gcode.encode(info)
        sig = torch.full((n,), sg, dtype=torch.float64, device="cuda")
        llr, _ = ldpc.channel_awgn(sig, gcode.N, codewords=cw, key=key, stream_id=0, frame_offset=offset + done)
        for name, p in (("learned", pl), ("nms", pn)):
            out = gcode.alloc_outputs(n, "cuda", with_llr=False)
            ws = gcode.alloc_workspace(n, p, "cuda")
            gcode.decode_into(llr, p, out["hard"], None, out["iters"], out["ok"], ws)
            errs = ldpc.count_errors(out["hard"], cw)
            r = res[name]
            r += np.array([int((errs > 0).sum()), int(errs.sum()), int(out["iters"].sum()), n])
        done += n
    out = {"ebn0_db": ebn0_db, "frames": frames, "T": T, "learned_max_iter": li, "nms_alpha": nms_alpha,
           "nms_max_iter": nms_iters}
    for name, r in res.items():
        out[name] = {"fer": r[0] / r[3], "ber": r[1] / (r[3] * gcode.N), "avg_iters": r[2] / r[3],
                     "frame_errors": int(r[0])}
    out["iter_saving"] = 1.0 - out["learned"]["avg_iters"] / out["nms"]["avg_iters"]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--code", default="peg1008", choices=sorted(FER.CODES))
    ap.add_argument("--T", type=int, default=20)
    ap.add_argument("--steps", type=int, default=1024)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=0.01)
    ap.add_argument("--ckpt", type=int, default=5)
    ap.add_argument("--eval-ebn0", type=float, nargs="+", default=[1.5, 2.0, 2.5])
    ap.add_argument("--eval-frames", type=int, default=100000)
    ap.add_argument("--save", default=None, help="write the trained pairs (.npy)")
    ap.add_argument("--init-alpha", type=float, default=0.8)
    ap.add_argument("--init-beta", type=float, default=0.0)
    ap.add_argument("--ebn0-lo", type=float, default=1.5)
    ap.add_argument("--ebn0-hi", type=float, default=2.5)
    ap.add_argument("--learned-iters", type=int, default=None,
                    help="iteration cap of the learned decoder at evaluation (default: NMS's 50)")
    ap.add_argument("--nms-alpha", type=float, nargs="+", default=[0.8],
                    help="constant normalisations the learned decoder is compared with")
    ap.add_argument("--tie-classes", action="store_true",
                    help="one pair per iteration shared by all check-degree classes")
    ap.add_argument("--loss-decay", type=float, default=1.0,
                    help="weight iteration t's loss by g^(t-1) (g < 1 favours early decoding)")
    args = ap.parse_args(argv)
    code = FER.CODES[args.code]()
    gcode = ldpc.Code.from_parity_check(code)
    w, log = train(gcode, T=args.T, steps=args.steps, batch=args.batch, lr=args.lr, ckpt=args.ckpt,
                   ebn0=(args.ebn0_lo, args.ebn0_hi), init=(args.init_alpha, args.init_beta),
                   tie_classes=args.tie_classes, loss_decay=args.loss_decay)
    for r in log:
        print(json.dumps({"train": r}), flush=True)
    if args.save:
        np.save(args.save, w.cpu().numpy())
    print(json.dumps({"weights": w.cpu().numpy().round(4).tolist(),
                      "classes": gcode.degree_classes().tolist()}), flush=True)
    for e in args.eval_ebn0:
        for na in args.nms_alpha:
            print(json.dumps(evaluate(gcode, w, e, args.eval_frames, nms_alpha=na, learned_iters=args.learned_iters)),
                  flush=True)
    gcode.close()


if __name__ == "__main__":
    main()
