"""The binary16 identities behind the uint8 working form (no GPU).

uint8 data is computed on as binary16 values.  The batched closure widens a
byte b by placing it under the high byte 0x64 -- the binary16 pattern of
1024 + b -- and subtracting 1024, and narrows a value v in 0..255 by adding
1024 and keeping the low byte.  Both are exact for every byte, and agree with
the plain conversion through float, which the other kernels use."""
import numpy as np


def f16(bits):
    return np.array(bits, dtype=np.uint16).view(np.float16)


def bits16(x):
    return np.array(x, dtype=np.float16).view(np.uint16)


def test_widen_every_byte():
    b = np.arange(256, dtype=np.uint16)
    under = f16(0x6400 | b)
    assert np.array_equal(under.astype(np.float64), 1024.0 + b)
    w = under - np.float16(1024.0)  # binary16 arithmetic, round to nearest
    assert np.array_equal(bits16(w), bits16(b.astype(np.float32).astype(np.float16)))
    assert bits16(w)[0] == 0  # 0 comes out as +0


def test_narrow_every_value():
    v = np.arange(256).astype(np.float16)
    up = v + np.float16(1024.0)
    assert np.array_equal(bits16(up), 0x6400 | np.arange(256, dtype=np.uint16))
    assert np.array_equal(bits16(up) & 0xFF, np.arange(256))
    # -0 (which the kernels never produce) would narrow to 0 as well
    assert bits16(np.float16(-0.0) + np.float16(1024.0)) == 0x6400
