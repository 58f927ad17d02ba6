"""Learned min-sum on the GPU (include/ldpc_learn.h, the weighted decode of
ldpc_decode_batch and paper_cs_0609090_amd/learn.py) against the oracle of
oracle/learned.py.

Forward: posteriors bit-exact against the oracle's binary32 mode (same
operations, same summation order); the loss (binary32 softplus sums, atomic
accumulation) within 1e-4 relative of the oracle's binary64 sum.
Adjoint: against the oracle's binary64 adjoint within 2e-3 relative (the
binary32 forward rounds differently from the binary64 one; inputs are
continuous, so ties of |t| and a*m = b have probability zero).
"""
import numpy as np
import pytest

from oracle import learned as LO
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


def _case(name, F, T, seed):
    rng = np.random.default_rng(seed)
    code = {"peg1008": W.code_c0_peg1008,
            "irregular": lambda: W.random_small_code(40, 90, (3, 9), seed=31),
            "qc7493": W.code_c1_qc7493}[name]()
    _, _, levels = LO.degree_classes(code)
    C = len(levels)
    w = np.stack([rng.uniform(0.6, 1.0, size=(T, C)), rng.uniform(0.0, 0.5, size=(T, C))],
                 axis=2).astype(np.float32)
    llr = rng.normal(1.0, 2.0, size=(F, code.N)).astype(np.float32)
    tgt = rng.integers(0, 2, size=(F, code.N)).astype(np.uint8)
    return code, w, llr, tgt


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("name,F,T", [("peg1008", 70, 5), ("irregular", 130, 6), ("qc7493", 64, 3)])
def test_forward_matches_oracle(torch_dev, L, name, F, T):
    torch = torch_dev
    code, w, llr, tgt = _case(name, F, T, 3)
    gc = L.Code.from_parity_check(code)
    assert list(gc.degree_classes()) == list(LO.degree_classes(code)[2])
    ws = torch.empty(gc.learn_workspace_size(F, T, 2), dtype=torch.uint8, device="cuda")
    post = torch.empty((F, code.N), dtype=torch.float32, device="cuda")
    loss = gc.learn_forward(_dev(torch, llr), _dev(torch, tgt), _dev(torch, w), 2, ws, post).cpu().numpy()
    gc.close()
    ref = LO.forward(code, llr, w, tgt, dtype=np.float32)
    np.testing.assert_array_equal(post.cpu().numpy(), ref["Z"][T])
    np.testing.assert_allclose(loss, ref["loss"], rtol=1e-4)


@pytest.mark.parametrize("name,F,T", [("peg1008", 70, 5), ("irregular", 66, 4)])
def test_gradient_matches_oracle_adjoint(torch_dev, L, name, F, T):
    torch = torch_dev
    code, w, llr, tgt = _case(name, F, T, 4)
    gc = L.Code.from_parity_check(code)
    grads = []
    for ckpt in (1, 2, T):
        ws = torch.empty(gc.learn_workspace_size(F, T, ckpt), dtype=torch.uint8, device="cuda")
        wd, td = _dev(torch, w), _dev(torch, tgt)
        gc.learn_forward(_dev(torch, llr), td, wd, ckpt, ws)
        grads.append(gc.learn_backward(F, td, wd, ckpt, ws).cpu().numpy())
    gc.close()
    ref, _ = LO.adjoint(code, llr.astype(np.float64), w.astype(np.float64), tgt)
    scale = np.abs(ref).max()
    for g in grads:
        np.testing.assert_allclose(g, ref, rtol=2e-3, atol=2e-3 * scale)
    # checkpointing recomputes the same forward values: same gradients up to
    # the order of the atomic per-class sums
    np.testing.assert_allclose(grads[1], grads[0], rtol=1e-5, atol=1e-6 * scale)
    np.testing.assert_allclose(grads[2], grads[0], rtol=1e-5, atol=1e-6 * scale)


def test_weighted_objective_gradient_matches_oracle(torch_dev, L):
    """Adjoint of sum_t w_t loss_t (iteration weights, some zero) against the
    oracle's weighted binary64 adjoint, and through LearnedMinSum."""
    torch = torch_dev
    from paper_cs_0609090_amd.learn import LearnedMinSum
    code, w, llr, tgt = _case("irregular", 66, 5, 5)
    lw = [2.5, 0.0, 1.0, 0.5, 0.0]
    gc = L.Code.from_parity_check(code)
    ws = torch.empty(gc.learn_workspace_size(66, 5, 2), dtype=torch.uint8, device="cuda")
    wd, td, xd = _dev(torch, w), _dev(torch, tgt), _dev(torch, llr)
    gc.learn_forward(xd, td, wd, 2, ws)
    g = gc.learn_backward(66, td, wd, 2, ws, loss_weights=lw).cpu().numpy()
    ref, fw = LO.adjoint(code, llr.astype(np.float64), w.astype(np.float64), tgt, loss_weights=lw)
    scale = np.abs(ref).max()
    np.testing.assert_allclose(g, ref, rtol=2e-3, atol=2e-3 * scale)
    assert np.all(g[4] == 0.0)  # the last iteration's loss has weight 0
    p = wd.clone().requires_grad_(True)
    obj = LearnedMinSum.apply(p, gc, xd, td, 2, ws, lw)
    obj.backward()
    np.testing.assert_allclose(float(obj), float(np.dot(lw, fw["loss"])), rtol=1e-4)
    np.testing.assert_allclose(p.grad.cpu().numpy(), g, rtol=1e-6, atol=1e-7 * scale)
    with pytest.raises(ValueError):
        gc.learn_backward(66, td, wd, 2, ws, loss_weights=lw[:4])
    with pytest.raises(L.LdpcError):
        gc.learn_backward(66, td, wd, 2, ws, loss_weights=[1.0, float("nan"), 1.0, 1.0, 1.0])
    gc.close()


def _syndrome_ok(code, hard):
    rp, ci = np.asarray(code.row_ptr), np.asarray(code.col_idx)
    rows = np.repeat(np.arange(code.M), np.diff(rp))
    s = np.zeros(code.M, dtype=np.int64)
    np.add.at(s, rows, hard[ci])
    return not (s & 1).any()


@pytest.mark.parametrize("early_stop", [False, True])
def test_weighted_decode(torch_dev, L, early_stop):
    """ldpc_decode_batch with per-iteration, per-class pairs equals the
    oracle's binary32 forward, with the per-frame stop at the first
    iteration whose hard decision is a codeword."""
    torch = torch_dev
    code = W.random_small_code(40, 90, (3, 9), seed=31)
    _, _, levels = LO.degree_classes(code)
    T, F = 8, 75
    rng = np.random.default_rng(8)
    w = np.stack([rng.uniform(0.6, 1.0, size=(T, len(levels))), rng.uniform(0.0, 0.4, size=(T, len(levels)))],
                 axis=2).astype(np.float32)
    llr = (W.awgn_llr(code.N, F, 3.0, code.design_rate, key=(0xD3, 1))).astype(np.float32)
    gc = L.Code.from_parity_check(code)
    out = gc.decode(_dev(torch, llr), msg="fp32", max_iter=T, early_stop=early_stop, weights=_dev(torch, w))
    g = {k: v.cpu().numpy() for k, v in out.items()}
    gc.close()
    ref = LO.forward(code, llr, w, dtype=np.float32)
    for f in range(F):
        k = T
        if early_stop:
            for t in range(1, T + 1):
                if _syndrome_ok(code, (ref["Z"][t][f] <= 0).astype(np.int64)):
                    k = t
                    break
        assert g["iters"][f] == k
        np.testing.assert_array_equal(g["llr"][f], ref["Z"][k][f])
        np.testing.assert_array_equal(g["hard"][f], (ref["Z"][k][f] <= 0).astype(np.uint8))
    if early_stop:
        assert len(set(g["iters"].tolist())) > 1


def test_constant_weights_equal_plain_decode(torch_dev, L):
    torch = torch_dev
    code = W.code_c0_peg1008()
    llr = _dev(torch, W.awgn_llr(code.N, 100, 1.8, code.design_rate, key=(0xD3, 2)))
    gc = L.Code.from_parity_check(code)
    w = torch.empty((3, 1, 2), dtype=torch.float32, device="cuda")
    w[:, :, 0], w[:, :, 1] = 0.75, 0.5
    a = gc.decode(llr, msg="fp32", max_iter=20, alpha=0.75, beta=0.5, layout="frames")
    b = gc.decode(llr, msg="fp32", max_iter=20, weights=w)
    gc.close()
    for k in ("hard", "llr", "iters", "ok"):
        np.testing.assert_array_equal(a[k].cpu().numpy(), b[k].cpu().numpy())


def test_training_lowers_the_loss(torch_dev, L):
    from paper_cs_0609090_amd import learn
    code = W.code_c0_peg1008()
    gc = L.Code.from_parity_check(code)
    w, log = learn.train(gc, T=5, steps=40, batch=256, lr=0.05, ckpt=2, log_every=39, init=(1.0, 0.0))
    gc.close()
    assert log[-1]["loss"] < log[0]["loss"]
    assert w.shape == (5, 1, 2) and float(w[:, 0, 0].max()) < 1.0


def test_training_with_tied_classes(torch_dev, L):
    """One pair per iteration shared by every degree class: the returned
    [T][C][2] pairs are equal across classes and training lowers the loss."""
    from paper_cs_0609090_amd import learn
    code = W.random_small_code(40, 90, (3, 9), seed=31)
    gc = L.Code.from_parity_check(code)
    C = len(gc.degree_classes())
    assert C > 1
    w, log = learn.train(gc, T=4, steps=40, batch=256, lr=0.05, ckpt=2, log_every=39, init=(1.0, 0.0),
                         ebn0=(2.0, 3.0), tie_classes=True)
    gc.close()
    assert w.shape == (4, C, 2)
    assert bool((w == w[:, :1, :]).all())
    assert log[-1]["loss"] < log[0]["loss"]
