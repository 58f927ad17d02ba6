"""Pins of the learned-decoder oracle (oracle/learned.py), CPU only.

Forward: with the same (a, b) at every iteration and class, the unrolled
posteriors are the plain NMS/OMS single-scan posteriors of the binary64 C
oracle, iteration by iteration and bit for bit (same summation order).
Per-class, per-iteration pairs: a class-zeroing identity against the C
oracle on H restricted to one class's rows (below), with planted mapping
mistakes that it must catch.
Adjoint: central finite differences of the binary64 loss, on codes with
several check-degree classes, with a nonzero transmitted codeword; with the
forward pinned, this pins the adjoint of the same decoder.
"""
import numpy as np
import pytest

from oracle import learned as LO
from paper_cs_0609090_amd import workloads as W


@pytest.mark.parametrize("alpha,beta", [(0.8, 0.0), (1.0, 0.5), (0.7, 0.25)])
def test_forward_equals_single_scan_f64(orc, alpha, beta):
    code = W.code_c0_peg1008()
    llr = W.awgn_llr(code.N, 3, 1.8, code.design_rate, key=(0x1EA, 1))
    T = 6
    w = np.zeros((T, 1, 2))
    w[:, :, 0], w[:, :, 1] = alpha, beta
    fw = LO.forward(code, llr, w)
    r = orc.decode(code, llr, algo="single_scan", arith="f64", max_iter=T, alpha=alpha, beta=beta,
                   early_stop=False, trace=True)
    for t in range(1, T + 1):
        np.testing.assert_array_equal(fw["Z"][t], r["Z"][:, t - 1, :])


def test_forward_binary32_equals_single_scan_f32(orc):
    code = W.code_c0_peg1008()
    llr = W.awgn_llr(code.N, 3, 1.8, code.design_rate, key=(0x1EA, 3))
    T = 6
    w = np.zeros((T, 1, 2), dtype=np.float32)
    w[:, :, 0], w[:, :, 1] = 0.8, 0.25
    fw = LO.forward(code, llr, w, dtype=np.float32)
    r = orc.decode(code, llr, algo="single_scan", arith="f32", max_iter=T, alpha=0.8, beta=0.25,
                   early_stop=False, trace=True)
    assert fw["Z"].dtype == np.float32
    for t in range(1, T + 1):
        np.testing.assert_array_equal(fw["Z"][t], r["Z"][:, t - 1, :])


def test_classes_of_irregular_rows():
    code = W.random_small_code(12, 30, (3, 7), seed=5)
    deg, cls, levels = LO.degree_classes(code)
    assert list(levels) == sorted(set(deg.tolist()))
    assert np.all(levels[cls] == deg)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_adjoint_matches_finite_differences(seed):
    rng = np.random.default_rng(seed)
    code = W.random_small_code(10, 24, (3, 6), seed=40 + seed)
    _, _, levels = LO.degree_classes(code)
    C, T, F = len(levels), 4, 3
    assert C >= 2
    llr = rng.normal(1.2, 2.0, size=(F, code.N))
    target = rng.integers(0, 2, size=(F, code.N))
    w = np.stack([rng.uniform(0.6, 1.0, size=(T, C)), rng.uniform(0.0, 0.4, size=(T, C))], axis=2)
    grad, fw = LO.adjoint(code, llr, w, target)
    eps = 1e-6
    num = np.zeros_like(w)
    for i in np.ndindex(*w.shape):
        wp, wm = w.copy(), w.copy()
        wp[i] += eps
        wm[i] -= eps
        num[i] = (LO.forward(code, llr, wp, target)["loss"].sum() -
                  LO.forward(code, llr, wm, target)["loss"].sum()) / (2 * eps)
    np.testing.assert_allclose(grad, num, rtol=2e-5, atol=2e-5 * np.abs(num).max())
    # the early iterations matter through the later ones: gradients are not
    # just the direct terms of the own iteration
    assert np.all(np.abs(grad[:, :, 0]).sum(axis=1) > 0)


def test_weighted_adjoint_matches_finite_differences():
    """The adjoint of sum_t w_t loss_t (iteration weights, some zero) against
    central differences of that same weighted sum of the forward's losses."""
    rng = np.random.default_rng(7)
    code = W.random_small_code(10, 24, (3, 6), seed=47)
    _, _, levels = LO.degree_classes(code)
    C, T, F = len(levels), 5, 3
    llr = rng.normal(1.0, 2.0, size=(F, code.N))
    target = rng.integers(0, 2, size=(F, code.N))
    w = np.stack([rng.uniform(0.6, 1.0, size=(T, C)), rng.uniform(0.0, 0.4, size=(T, C))], axis=2)
    lw = np.array([3.0, 0.0, 1.5, 0.25, 0.0])
    grad, _ = LO.adjoint(code, llr, w, target, loss_weights=lw)
    eps = 1e-6
    num = np.zeros_like(w)
    for i in np.ndindex(*w.shape):
        wp, wm = w.copy(), w.copy()
        wp[i] += eps
        wm[i] -= eps
        num[i] = (lw @ LO.forward(code, llr, wp, target)["loss"] - lw @ LO.forward(code, llr, wm, target)["loss"]) / (
            2 * eps)
    np.testing.assert_allclose(grad, num, rtol=2e-5, atol=2e-5 * np.abs(num).max())
    # the last iteration's loss has weight 0: its own pairs get no gradient
    assert np.all(grad[T - 1] == 0.0)
    # linear in the iteration weights
    g1, _ = LO.adjoint(code, llr, w, target, loss_weights=np.eye(T)[0])
    g3, _ = LO.adjoint(code, llr, w, target, loss_weights=np.eye(T)[2])
    g4, _ = LO.adjoint(code, llr, w, target, loss_weights=np.eye(T)[3])
    np.testing.assert_allclose(grad, 3.0 * g1 + 1.5 * g3 + 0.25 * g4, rtol=1e-12, atol=1e-12 * np.abs(grad).max())


def test_loss_of_the_transmitted_word_direction():
    """Raising every a when the decoder is confidently right lowers the loss
    (messages grow in the direction of the codeword)."""
    code = W.code_c0_peg1008()
    llr = W.awgn_llr(code.N, 2, 4.0, code.design_rate, key=(0x1EA, 2))
    w = np.zeros((3, 1, 2))
    w[:, :, 0] = 0.7
    g, _ = LO.adjoint(code, llr, w)
    assert np.all(g[:, :, 0] < 0)


# --------------------------------------------------------------------------
# Per-class and per-iteration pairs: a class-zeroing identity.
#
# A pair (a, b) = (1, 1e12) makes every message of its rows exactly zero
# (max(m - 1e12, 0) = 0 for any finite minimum), so those rows drop out of
# Eq. (3) and of the posterior sums.  With every class but one zeroed at
# every iteration, and every class zeroed during the first t0 iterations,
# the unrolled decoder must reproduce the plain single-scan decoder of the
# binary64 C oracle run for T - t0 iterations with the kept class's pair on
# H restricted to that class's rows (the zeroed iterations leave L = 0 and
# Z = Z(0), the decoder's initial state).  A wrong class-to-row mapping or a
# shifted iteration index makes the kept rows take another pair or start
# early, and the posteriors differ.
# --------------------------------------------------------------------------
_ZERO_PAIR = (1.0, 1e12)


def _restrict_rows(code, keep_rows):
    rp, ci = np.asarray(code.row_ptr), np.asarray(code.col_idx)
    rows = [ci[rp[m]:rp[m + 1]] for m in keep_rows]
    return W.ParityCheck.from_rows(len(rows), code.N, rows, code.name + "_restricted")


def _classy_code():
    # row degrees 3..7: five classes, cycles allowed
    code = W.random_small_code(30, 64, (3, 7), seed=909)
    _, cls, levels = LO.degree_classes(code)
    assert len(levels) >= 3
    return code, cls, levels


def check_class_identity(orc, code, cls, levels, kept, pair, t0, T, llr):
    """Run the identity for one kept class; raises AssertionError on mismatch."""
    C = len(levels)
    w = np.empty((T, C, 2))
    w[:, :, 0], w[:, :, 1] = _ZERO_PAIR
    w[t0:, kept, 0], w[t0:, kept, 1] = pair
    fw = LO.forward(code, llr, w)
    keep_rows = np.nonzero(cls == kept)[0]
    sub = _restrict_rows(code, keep_rows)
    r = orc.decode(sub, llr, algo="single_scan", arith="f64", max_iter=T - t0, alpha=pair[0],
                   beta=pair[1], early_stop=False, trace=True)
    rp = np.asarray(code.row_ptr)
    kept_edges = np.concatenate([np.arange(rp[m], rp[m + 1]) for m in keep_rows])
    other_edges = np.setdiff1d(np.arange(code.E), kept_edges)
    for t in range(1, T + 1):
        if t <= t0:
            np.testing.assert_array_equal(fw["Z"][t], llr)
            assert not np.any(fw["L"][t])
            continue
        np.testing.assert_array_equal(fw["Z"][t], r["Z"][:, t - t0 - 1, :])
        np.testing.assert_array_equal(fw["L"][t][:, kept_edges], r["L"][:, t - t0 - 1, :])
        assert not np.any(fw["L"][t][:, other_edges])
    # the kept rows really decode: some of their messages are nonzero
    assert np.any(fw["L"][T][:, kept_edges])


@pytest.mark.parametrize("t0", [0, 2])
def test_class_zeroing_identity(orc, t0):
    code, cls, levels = _classy_code()
    llr = W.awgn_llr(code.N, 4, 1.5, code.design_rate, key=(0x1EA, 7))
    pairs = [(0.55, 0.0), (0.7, 0.25), (0.85, 0.125), (1.0, 0.5), (0.625, 0.375), (0.9, 0.0)]
    T = 5
    for kept in range(len(levels)):
        check_class_identity(orc, code, cls, levels, kept, pairs[kept % len(pairs)], t0, T, llr)


def test_class_identity_catches_planted_mapping_errors(orc, monkeypatch):
    """Plant mistakes in the oracle's pair lookup (on the CPU): a reversed
    class order, an off-by-one class and an off-by-one iteration.  Each must
    fail the identity."""
    code, cls, levels = _classy_code()
    llr = W.awgn_llr(code.N, 4, 1.5, code.design_rate, key=(0x1EA, 7))
    good = LO._pair
    C = len(levels)
    planted = {
        "reversed classes": lambda Wt, t, c: good(Wt, t, C - 1 - c),
        "class + 1": lambda Wt, t, c: good(Wt, t, np.minimum(c + 1, C - 1)),
        "iteration + 1": lambda Wt, t, c: good(Wt, min(t + 1, Wt.shape[0]), c),
        "iteration - 1": lambda Wt, t, c: good(Wt, max(t - 1, 1), c),
    }
    for name, fn in planted.items():
        monkeypatch.setattr(LO, "_pair", fn)
        caught = False
        for kept in range(C):
            try:
                check_class_identity(orc, code, cls, levels, kept, (0.7, 0.25), 2, 5, llr)
            except AssertionError:
                caught = True
                break
        assert caught, f"planted mistake not caught: {name}"
    monkeypatch.setattr(LO, "_pair", good)
    check_class_identity(orc, code, cls, levels, 0, (0.7, 0.25), 2, 5, llr)
