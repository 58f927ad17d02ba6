"""GPU channel simulation (include/ldpc_sim.h) against host references:
Philox bits and the AWGN channel against the host generator written from
the same published definitions, codewords against H c^T = 0, error counts
against numpy, and the FER harness against the oracle on host-generated
inputs.

The channel's Box-Muller step uses binary64 log/sqrt/cos/sin on both sides
(GPU device library, host numpy); each is accurate to about an ulp of
binary64, so the binary32 LLRs (rounded once from binary64) agree except
where a binary64 result lies within a few ulps of a binary32 rounding
boundary: at most one binary32 ulp, on a vanishing fraction of values.  The
fixed-point LLRs are decided from the binary32 values, so they can differ
only where the binary32 values do.
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


@pytest.mark.parametrize("F,nbits,key,stream,off", [(3, 1, (1, 2), 0, 0), (7, 127, (0x5EED, 1), 1, 0),
                                                    (5, 129, (0xFFFFFFFF, 7), 3, 1000),
                                                    (64, 32400, (0x5EED, 1), 1, 77)])
def test_random_bits_match_host(torch_dev, L, F, nbits, key, stream, off):
    g = L.random_bits(F, nbits, key=key, stream_id=stream, frame_offset=off).cpu().numpy()
    h = W.random_bits(F, nbits, key, stream, off)
    np.testing.assert_array_equal(g, h)
    assert 0.45 < h.mean() < 0.55 or h.size < 1000


def _ulp_diff(a, b):
    ai = a.view(np.int32).astype(np.int64)
    bi = b.view(np.int32).astype(np.int64)
    ai = np.where(ai < 0, -(ai & 0x7FFFFFFF), ai)
    bi = np.where(bi < 0, -(bi & 0x7FFFFFFF), bi)
    return np.abs(ai - bi)


@pytest.mark.parametrize("N,F", [(1008, 64), (1003, 17)])
def test_channel_matches_host(torch_dev, L, N, F):
    torch = torch_dev
    key = (0xC0FFEE, 3)
    rng = np.random.default_rng(5)
    cw = rng.integers(0, 2, size=(F, N)).astype(np.uint8)
    ebn0 = np.linspace(0.5, 4.0, F)
    rate = 0.5
    sig = np.array([W.ebn0_to_sigma(float(e), rate) for e in ebn0])
    f32, q = L.channel_awgn(torch.tensor(sig, device="cuda"), N, codewords=torch.from_numpy(cw).cuda(),
                            key=key, stream_id=0, frame_offset=11, want_f32=True, want_q=True, step=0.5, qmax=31)
    f32, q = f32.cpu().numpy(), q.cpu().numpy()
    h = W.awgn_llr(N, F, ebn0, rate, key=key, stream=0, codewords=cw, frame_offset=11)
    hq = W.quantize_llr(h)
    d = _ulp_diff(f32, h)
    assert d.max() <= 1
    assert (d > 0).sum() <= max(1, f32.size // 100000)
    same = d == 0
    np.testing.assert_array_equal(q[same], hq[same])
    # the channel really depends on the codeword: flipping the bits flips the mean
    assert np.mean(h[cw == 1]) < 0 < np.mean(h[cw == 0])


def _syndrome(code, cw):
    rp, ci = np.asarray(code.row_ptr), np.asarray(code.col_idx)
    rows = np.repeat(np.arange(code.M), np.diff(rp))
    s = np.zeros((cw.shape[0], code.M), dtype=np.int64)
    for f in range(cw.shape[0]):
        np.add.at(s[f], rows, cw[f, ci])
    return s & 1


@pytest.mark.parametrize("name,F", [("peg1008", 33), ("qc7493", 9), ("ira16200", 12), ("ira64800", 3),
                                    ("tiny", 50)])
def test_encoder_codewords(torch_dev, L, name, F):
    code = {"peg1008": W.code_c0_peg1008, "qc7493": W.code_c1_qc7493, "ira16200": W.code_ira16200,
            "ira64800": W.code_c2_ira64800,
            "tiny": lambda: W.random_small_code(9, 20, (2, 6), seed=77)}[name]()
    gc = L.Code.from_parity_check(code)
    e = gc.encoder_info()
    K, pos = e["K"], e["info_pos"]
    info = W.random_bits(F, K, (0xE1, 2), 5, 0)
    info[0] = 0                       # the all-zero word encodes to the zero codeword
    cw = gc.encode(torch_dev.from_numpy(info).cuda()).cpu().numpy()
    gc.close()
    assert cw.shape == (F, code.N) and set(np.unique(cw)) <= {0, 1}
    np.testing.assert_array_equal(cw[:, pos[:K]], info)
    assert not _syndrome(code, cw).any()
    assert not cw[0].any()
    assert cw[1:].any()


def _host_codewords(code, pos, K, info):
    """Codewords with the given information bits at columns pos[:K]: the
    parity bits solve H_P p = H_I u over GF(2) (plain elimination, host)."""
    H = code.dense().astype(np.uint8)
    Hp = H[:, pos[K:]].copy()
    S = (H[:, pos[:K]].astype(np.int64) @ info.T.astype(np.int64) % 2).astype(np.uint8)
    r = 0
    for c in range(Hp.shape[1]):
        piv = np.nonzero(Hp[r:, c])[0]
        assert piv.size, "parity columns must carry a nonsingular submatrix"
        p_ = r + piv[0]
        Hp[[r, p_]] = Hp[[p_, r]]
        S[[r, p_]] = S[[p_, r]]
        hit = np.nonzero(Hp[:, c])[0]
        hit = hit[hit != r]
        Hp[hit] ^= Hp[r]
        S[hit] ^= S[r]
        r += 1
    cw = np.zeros((info.shape[0], code.N), dtype=np.uint8)
    cw[:, pos[:K]] = info
    cw[:, pos[K:]] = S[:r].T
    return cw


def test_count_errors(torch_dev, L):
    torch = torch_dev
    rng = np.random.default_rng(9)
    hard = (rng.random((40, 777)) < 0.01).astype(np.uint8)
    cw = (rng.random((40, 777)) < 0.5).astype(np.uint8)
    g = L.count_errors(torch.from_numpy(hard).cuda(), torch.from_numpy(cw).cuda()).cpu().numpy()
    np.testing.assert_array_equal(g, (hard != cw).sum(axis=1))
    g0 = L.count_errors(torch.from_numpy(hard).cuda()).cpu().numpy()
    np.testing.assert_array_equal(g0, hard.sum(axis=1))


def test_fer_harness_matches_oracle(torch_dev, L, orc):
    """The harness's counts for the (3,6) PEG code at 1.5 dB equal the
    oracle's on the same frames regenerated on the host (host bits, the
    library's information positions, host AWGN and quantiser)."""
    from paper_cs_0609090_amd import fer
    code = W.code_c0_peg1008()
    gc = L.Code.from_parity_check(code)
    frames, key, ebn0 = 150, (0x5EED, 1), 1.5
    r = fer.run_point(gc, ebn0, frames, batch=64, msg="int8", max_iter=30, alpha=0.8, key=key)
    e = gc.encoder_info()
    K, pos = e["K"], e["info_pos"]
    gc.close()
    info = W.random_bits(frames, K, key, 1, 0)
    cw = _host_codewords(code, pos, K, info)
    assert not _syndrome(code, cw).any()
    llr = W.awgn_llr(code.N, frames, ebn0, K / code.N, key=key, stream=0, codewords=cw)
    q = W.quantize_llr(llr)
    o = orc.decode(code, q, algo="single_scan", arith="int", max_iter=30, alpha=0.8, early_stop=True)
    errs = (o["hard"] != cw).sum(axis=1)
    assert r["frame_errors"] == int((errs > 0).sum())
    assert r["bit_errors"] == int(errs.sum())
    assert r["detected_failures"] == int((o["ok"] == 0).sum())
    assert r["avg_iters"] == pytest.approx(o["iters"].mean())
    assert 0 < r["frame_errors"] < frames  # 1.5 dB sits in the waterfall of this code
