"""The binary16 arithmetic the packed kernel runs on stored integers, checked
exhaustively on the host with IEEE binary16 (numpy float16 keeps subnormals).

The kernel reads the stored Z_old + ZB and L + ZB values (non-negative
integers below 1024, so binary16 subnormals with the same bits) as binary16:
  * their difference is exact and in sign-magnitude form: bit 15 is the sign
    of the integer difference (clear for zero) and the other bits are its
    magnitude;
  * a magnitude m <= Q times +-1.0 plus ZB (Q < ZB) is exact and its bits are
    the integer ZB +- m.
"""
import numpy as np


def _h(bits):
    return np.asarray(bits, dtype=np.uint16).view(np.float16)


def _bits(x):
    return np.asarray(x, dtype=np.float16).view(np.uint16).astype(np.int64)


def test_difference_of_stored_values_is_sign_magnitude():
    z = np.arange(0, 1024, dtype=np.int64)
    zz, ll = np.meshgrid(z, z, indexing="ij")
    t = _bits(_h(zz) - _h(ll))
    diff = zz - ll
    assert np.array_equal(t & 0x7FFF, np.abs(diff))
    assert np.array_equal((t >> 15) & 1, (diff < 0).astype(np.int64))


def test_signed_message_plus_bias_is_the_integer():
    for zb, q in ((63, 31), (127, 63)):
        m = np.arange(0, q + 1, dtype=np.int64)
        for s in (1.0, -1.0):
            one = np.float16(s)
            # the product is exact, so a fused multiply-add rounds once as the
            # two steps here do
            r = _bits(_h(m) * one + _h(np.full_like(m, zb)))
            assert np.array_equal(r, zb + (m if s > 0 else -m))


def test_sign_word_of_the_row_parity():
    # (t & 0x8000) ^ ((par & 0x8000) | 0x3C00) is +-1.0 with the XOR of both signs
    for ts in (0, 1):
        for ps in (0, 1):
            w = ((ts << 15) & 0x8000) ^ (((ps << 15) & 0x8000) | 0x3C00)
            assert float(_h(w)) == (-1.0 if ts ^ ps else 1.0)
