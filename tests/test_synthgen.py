"""The seeded input generators and the Boolean bit packing (no GPU)."""
import numpy as np
import pytest

import synthgen


def test_pack_lsb_first_matches_listing_bit_order():
    """Entry (r, c) is bit c & 7 of byte c >> 3 of the row (Sec. IV Boolean
    listing), i.e. bit c % 64 of word c // 64 on a little-endian machine."""
    M = np.zeros((2, 130), np.uint8)
    M[0, 0] = 1
    M[0, 65] = 1
    M[1, 129] = 1
    W = synthgen.pack_bits(M, 4)
    assert W.shape == (2, 4)
    assert W[0, 0] == 1 and W[0, 1] == 2 and W[0, 2] == 0
    assert W[1, 2] == 2
    by = W.astype("<u8").view(np.uint8).reshape(2, -1)
    assert by[0, 65 >> 3] & (1 << (65 & 7))


@pytest.mark.parametrize("R,C,ld", [(1, 1, None), (3, 64, None), (5, 65, 4), (7, 300, 6)])
def test_pack_roundtrip_and_padding(R, C, ld):
    gen = synthgen.generator(1)
    M = (gen.random((R, C)) < 0.4).astype(np.uint8)
    W = synthgen.pack_bits(M, ld)
    assert np.array_equal(synthgen.unpack_bits(W, C), M)
    assert synthgen.padding_bits_clear(W, C)


def test_bernoulli_edges_no_self_loops_and_density():
    gen = synthgen.generator(2)
    D, p = 600, 0.05
    r, c = synthgen.bernoulli_edges(D, p, gen, chunk_rows=97)
    assert not np.any(r == c)
    n = D * (D - 1)
    mean, sd = n * p, np.sqrt(n * p * (1 - p))
    assert abs(len(r) - mean) < 5 * sd
    assert len(set(zip(r.tolist(), c.tolist()))) == len(r)


def test_seeded_reproducible():
    a = synthgen.cfg_antidist(D=128, seed=9)
    b = synthgen.cfg_antidist(D=128, seed=9)
    c = synthgen.cfg_antidist(D=128, seed=9, which=1)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_encode_antidist():
    M = synthgen.encode_antidist(3, [0, 1, 2, 2], [1, 2, 0, 1], [0, 5, 255, 300], np.uint8, ld=16)
    assert M.shape == (3, 16) and M.dtype == np.uint8
    assert M[0, 1] == 255 and M[1, 2] == 250 and M[2, 0] == 0 and M[2, 1] == 0
    M16 = synthgen.encode_antidist(3, [2], [0], [255], np.uint16)
    assert M16[2, 0] == 65535 - 255


def test_cfg_antidist_heavy_fraction():
    M = synthgen.cfg_antidist(D=512, seed=4)
    vals = M[M > 0].astype(np.int64)
    heavy = (vals < 1000).mean()
    assert 0.003 < heavy < 0.02
    assert M.shape[1] % 8 == 0


def test_aligned_ld():
    assert synthgen.aligned_ld(37, np.uint8) == 48
    assert synthgen.aligned_ld(37, np.uint16) == 40
    assert synthgen.aligned_ld_words(257) == 6
    assert synthgen.aligned_ld_words(1) == 2


def test_planted_cycles_disjoint():
    gen = synthgen.generator(3)
    s, d = synthgen.planted_cycles(1000, 3, 100, gen)
    assert len(np.unique(s)) == 300 and len(s) == 300
    assert set(s.tolist()) == set(d.tolist())


def test_batch_and_trace_shapes():
    b = synthgen.cfg_batch(count=50, seed=5)
    assert len(b) == 50 and all(32 <= n <= 1024 for n, *_ in b)
    t = synthgen.serving_trace(40, seed=6)
    assert {k for _, k, _ in t} <= {"bool", "u16"} and all(64 <= n <= 8192 for n, _, _ in t)
