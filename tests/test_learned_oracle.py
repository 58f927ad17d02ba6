"""Pins of the learned-decoder oracle (oracle/learned.py), CPU only.

Forward: with the same (a, b) at every iteration and class, the unrolled
posteriors are the plain NMS/OMS single-scan posteriors of the binary64 C
oracle, iteration by iteration and bit for bit (same summation order).
Adjoint: central finite differences of the binary64 loss, on codes with
several check-degree classes, with a nonzero transmitted codeword.
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


def test_loss_of_the_transmitted_word_direction():
    """Raising every a when the decoder is confidently right lowers the loss
    (messages grow in the direction of the codeword)."""
    code = W.code_c0_peg1008()
    llr = W.awgn_llr(code.N, 2, 4.0, code.design_rate, key=(0x1EA, 2))
    w = np.zeros((3, 1, 2))
    w[:, :, 0] = 0.7
    g, _ = LO.adjoint(code, llr, w)
    assert np.all(g[:, :, 0] < 0)
